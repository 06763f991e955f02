"""Plain FP64 CPU oracle of the FE-LBM time step in 3-D: D3Q19 populations g
and h on linear tetrahedra, the paper's own setting (Sec. II.A: D3Q19 lattice;
Sec. II.C: linear tetrahedral elements).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this module; only the tests use it.  It shares no code with the GPU
library (nor with the 2-D oracle): it reads the same seeded mesh and input
arrays, and nothing else.

The scheme is the one of the 2-D oracle with the tetrahedral forms:
  * finite element matrices of eq:fem_matrices assembled from element
    integrals: M11 = V/20 (1 + delta_ij), M10 = V/4, C_r = (V/4) d_r N_j,
    D_sr = (V/2) d_s N_i d_r N_j, K_r = (V/2) d_r N_i;
  * the weak form +(dt M10 + dt^2 K_a) Phi (reading R1 of the 2-D oracle),
    PCG with the lumped mass as preconditioner, x0 = b/m;
  * the nodal Laplacian of C over the vertex patch (eqn:lapl_int_mp): the
    faces opposite the node in every patch element, with the average of the
    two adjacent element gradients (reading R2), and wall faces (opposite the
    node, or containing it) carrying the wetting flux of eq. bc2 with n into
    the fluid (R3), integrated exactly over each triangle (phi_c and C linear
    on it: the integrand is a cubic in the barycentric coordinates);
  * the element Laplacian of mu over the element's four faces with averaged
    gradients, zero on wall faces (eqn:bc1);
  * P0 forces at barycentric values (R5), the wall operator on opposite pairs
    (R4), moments without a half-force shift (R6).
The outward area vector of the face opposite vertex l of a tetrahedron is
-3 V grad N_l.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

# ---------------------------------------------------------------------------
# D3Q19 lattice (textbook constants)
# ---------------------------------------------------------------------------
_dirs = [(0, 0, 0)]
for d in range(3):
    for s in (1, -1):
        v = [0, 0, 0]
        v[d] = s
        _dirs.append(tuple(v))
for a, b in ((0, 1), (0, 2), (1, 2)):
    for sa, sb in ((1, 1), (-1, -1), (1, -1), (-1, 1)):
        v = [0, 0, 0]
        v[a], v[b] = sa, sb
        _dirs.append(tuple(v))
E = np.array(_dirs, dtype=np.float64)
Q = 19
W = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)
CS2 = 1.0 / 3.0
OPPOSITE = np.array([next(j for j in range(Q) if np.all(E[j] == -E[i])) for i in range(Q)])


class Params:
    def __init__(self, sigma, xi, mobility, rho_l, rho_v, nu_l, nu_v, dt):
        # xi = sqrt(8 kappa / beta), sigma = sqrt(2 kappa beta) / 6  (Sec. II)
        self.kappa = 1.5 * sigma * xi
        self.beta = 12.0 * sigma / xi
        self.mobility, self.rho_l, self.rho_v, self.dt = mobility, rho_l, rho_v, dt
        # nu = c_s^2 tau dt (Sec. II.A)
        self.tau_l, self.tau_v = nu_l / (CS2 * dt), nu_v / (CS2 * dt)


# ---------------------------------------------------------------------------
# Geometry of P1 tetrahedra
# ---------------------------------------------------------------------------
class Geometry:
    def __init__(self, mesh):
        self.mesh = mesh
        xyz, tet = mesh.xyz, np.asarray(mesh.tet, dtype=np.int64)
        self.N, self.NT = xyz.shape[0], tet.shape[0]
        self.tet = tet
        p = xyz[tet].copy()                                          # (NT, 4, 3)
        for d, L in enumerate(mesh.period):
            if L > 0:
                for k in (1, 2, 3):
                    p[:, k, d] -= L * np.round((p[:, k, d] - p[:, 0, d]) / L)
        self.p = p
        J = np.stack([p[:, 1] - p[:, 0], p[:, 2] - p[:, 0], p[:, 3] - p[:, 0]], axis=2)  # columns
        det = np.linalg.det(J)
        if np.any(det <= 0):
            raise ValueError("non-positive tetrahedron volume")
        self.vol = det / 6.0
        Jinv = np.linalg.inv(J)                                        # rows: grad of barycentric 1..3
        g = np.empty((self.NT, 4, 3))
        g[:, 1:] = Jinv
        g[:, 0] = -Jinv.sum(axis=1)
        self.gradN = g
        self.centroid = p.mean(axis=1)
        # face l of a tetrahedron is the one opposite vertex l
        others = [[1, 2, 3], [0, 2, 3], [0, 1, 3], [0, 1, 2]]
        self.face_nodes = np.stack([tet[:, o] for o in others], axis=1)   # (NT, 4, 3)
        key = np.sort(self.face_nodes, axis=2)
        flat = key.reshape(-1, 3)
        order = np.lexsort((flat[:, 2], flat[:, 1], flat[:, 0]))
        ks = flat[order]
        same = np.all(ks[1:] == ks[:-1], axis=1)
        i0, i1 = order[:-1][same], order[1:][same]
        self.face_nbr = -np.ones((self.NT, 4), dtype=np.int64)
        self.face_nbr.ravel()[i0] = i1 // 4
        self.face_nbr.ravel()[i1] = i0 // 4
        self.face_area_vec = -3.0 * self.vol[:, None, None] * g           # |f| n_out, (NT, 4, 3)
        wall = np.asarray(mesh.wall_faces, dtype=np.int64)
        self.wall_faces = wall
        wkey = np.sort(wall, axis=1)
        code = lambda k: (k[..., 0] * self.N + k[..., 1]) * self.N + k[..., 2]
        self.face_is_wall = np.isin(code(key), code(wkey))
        if np.any((self.face_nbr < 0) & ~self.face_is_wall):
            raise ValueError("boundary face that is neither a wall nor periodic")
        # wall face areas from the unwrapped triangle
        q = xyz[wall].copy()
        for d, L in enumerate(mesh.period):
            if L > 0:
                for k in (1, 2):
                    q[:, k, d] -= L * np.round((q[:, k, d] - q[:, 0, d]) / L)
        self.wall_area = 0.5 * np.linalg.norm(np.cross(q[:, 1] - q[:, 0], q[:, 2] - q[:, 0]), axis=1)
        self.is_wall_node = np.zeros(self.N, dtype=bool)
        self.is_wall_node[wall.ravel()] = True
        self.patch_volume = np.zeros(self.N)
        np.add.at(self.patch_volume, tet.ravel(), np.repeat(self.vol, 4))


# ---------------------------------------------------------------------------
# Finite element matrices (eq:fem_matrices) for P1 tetrahedra
# ---------------------------------------------------------------------------
class Matrices:
    def __init__(self, geo: Geometry):
        N, NT, tet, V, G = geo.N, geo.NT, geo.tet, geo.vol, geo.gradN
        I = np.repeat(tet, 4, axis=1).ravel()
        J = np.tile(tet, (1, 4)).ravel()
        li = np.repeat(np.arange(4), 4)
        lj = np.tile(np.arange(4), 4)
        # int_T phi_i phi_j = V/20 (1 + delta_ij)
        self.M11 = sp.csr_matrix((((V[:, None] / 20.0) * (1.0 + (li == lj))[None, :]).ravel(), (I, J)), shape=(N, N))
        self.lumped = np.asarray(self.M11.sum(axis=1)).ravel()
        # int_T phi_i d_r phi_j = (V/4) d_r N_j
        self.C = [sp.csr_matrix((((V[:, None] / 4.0) * G[:, lj, r]).ravel(), (I, J)), shape=(N, N)) for r in range(3)]
        # 1/2 int_T d_s phi_i d_r phi_j = (V/2) d_s N_i d_r N_j
        self.D = [[sp.csr_matrix((((V[:, None] / 2.0) * G[:, li, s] * G[:, lj, r]).ravel(), (I, J)), shape=(N, N))
                   for r in range(3)] for s in range(3)]
        Ie = tet.ravel()
        Te = np.repeat(np.arange(NT), 4)
        # int_T phi_i = V/4; 1/2 int_T d_r phi_i = (V/2) d_r N_i
        self.M10 = sp.csr_matrix((np.repeat(V / 4.0, 4), (Ie, Te)), shape=(N, NT))
        self.K = [sp.csr_matrix((((V[:, None] / 2.0) * G[:, :, r]).ravel(), (Ie, Te)), shape=(N, NT)) for r in range(3)]
        self.Ca = [sum(E[a, r] * self.C[r] for r in range(3)) for a in range(Q)]
        self.Da = [sum(E[a, s] * E[a, r] * self.D[s][r] for s in range(3) for r in range(3)) for a in range(Q)]
        self.Ka = [sum(E[a, r] * self.K[r] for r in range(3)) for a in range(Q)]


# ---------------------------------------------------------------------------
# Kinetic model (Sec. II.A) in three dimensions
# ---------------------------------------------------------------------------
def edot(u):
    """e_a . u for u of shape (n, 3): (n, 19)."""
    return u @ E.T


def gamma(u):
    """Gamma_a(u) = w_a [1 + e.u/cs^2 + ((e.u)^2 - cs^2 u.u)/(2 cs^4)]."""
    eu = edot(u)
    uu = np.sum(u * u, axis=1)[:, None]
    return W * (1.0 + eu / CS2 + (eu * eu - CS2 * uu) / (2.0 * CS2 * CS2))


def density(C, prm):
    return C * prm.rho_l + (1.0 - C) * prm.rho_v


def moments(g, h, prm):
    C = h.sum(axis=1)
    p = g.sum(axis=1)
    rho = density(C, prm)
    u = (g @ E) / CS2 / rho[:, None]
    return C, p, rho, u


def relaxation_time(C, prm):
    return 1.0 / (C / prm.tau_l + (1.0 - C) / prm.tau_v)


def equilibria(C, p, rho, u):
    """g_eq (eqn::g_eq) and h_eq = Gamma(u) C (eqn::f_eq)."""
    eu = edot(u)
    uu = np.sum(u * u, axis=1)[:, None]
    g_eq = W * (p[:, None] + rho[:, None] * CS2 * (eu / CS2 + (eu * eu - CS2 * uu) / (2.0 * CS2 * CS2)))
    return g_eq, gamma(u) * C[:, None]


def collide(psi, psi_eq, tau):
    """psi_hat = psi_bar - (psi_bar - psi_eq)/(tau + 0.5)  (eqn::collide)."""
    return psi - (psi - psi_eq) / (tau[:, None] + 0.5)


def wall_operator(geo, psi):
    """Reading R4: at wall nodes each opposite pair is replaced by its mean."""
    out = psi.copy()
    w = geo.is_wall_node
    for a in range(1, Q):
        out[w, a] = 0.5 * (psi[w, a] + psi[w, OPPOSITE[a]])
    return out


# ---------------------------------------------------------------------------
# Gradients, the wetting flux and the Laplacians (Sec. II.C-D)
# ---------------------------------------------------------------------------
def element_gradient(geo, f):
    return np.einsum("tl,tlr->tr", f[geo.tet], geo.gradN)


def triangle_monomial(i, j, k):
    """int over a triangle of area 1 of lambda_i lambda_j lambda_k (the
    barycentric coordinates): 2 a! b! c! / 5! for the exponents a, b, c."""
    from math import factorial
    ex = [0, 0, 0]
    for v in (i, j, k):
        ex[v] += 1
    return 2.0 * factorial(ex[0]) * factorial(ex[1]) * factorial(ex[2]) / factorial(5)


def wall_flux(Cf, rf, area):
    """Outward flux int_f grad C . n_out dA through a wall face from eq. bc2
    with n into the fluid (reading R3): -int (phi_c/kappa)(C - C^2) dA with
    C (Cf, three vertex values) and r = phi_c/kappa (rf) linear on the face;
    the cubic integrand is integrated exactly term by term."""
    lin = sum(rf[i] * Cf[j] * (area / 12.0) * (1.0 + (i == j)) for i in range(3) for j in range(3))
    cub = sum(rf[i] * Cf[j] * Cf[k] * area * triangle_monomial(i, j, k)
              for i in range(3) for j in range(3) for k in range(3))
    return -(lin - cub)


def laplacian_C(geo, C, gradC, bc):
    """Nodal Laplacian of C over the vertex patch: the faces opposite the node
    in every patch element (averaged gradients, or the wetting flux on a wall
    face) plus the wall faces that contain the node, over the patch volume."""
    flux = np.zeros(geo.N, dtype=np.result_type(C, gradC))
    for l in range(4):
        k = geo.tet[:, l]
        nbr = geo.face_nbr[:, l]
        on_wall = geo.face_is_wall[:, l]
        inner = ~on_wall
        fl = np.zeros(geo.NT, dtype=flux.dtype)
        Gavg = 0.5 * (gradC[inner] + gradC[nbr[inner]])
        fl[inner] = (geo.face_area_vec[inner, l] * Gavg).sum(1)
        fn = geo.face_nodes[on_wall, l]
        area = np.linalg.norm(geo.face_area_vec[on_wall, l], axis=1)
        fl[on_wall] = wall_flux(C[fn].T, bc[fn].T, area)
        np.add.at(flux, k, fl)
    wf = geo.wall_faces
    fw = wall_flux(C[wf].T, bc[wf].T, geo.wall_area)
    for c in range(3):
        np.add.at(flux, wf[:, c], fw)
    return flux / geo.patch_volume


def chemical_potential(prm, C, lapC):
    # mu = 2 beta C (C - 1)(2C - 1) - kappa lap C  (eqn:mp_mu)
    return 2.0 * prm.beta * C * (C - 1.0) * (2.0 * C - 1.0) - prm.kappa * lapC


def laplacian_mu(geo, gradmu):
    """Element Laplacian of mu: sum over the four faces of |f| n . (average of
    the two adjacent element gradients), zero on wall faces, over the volume."""
    acc = np.zeros(geo.NT, dtype=gradmu.dtype)
    for l in range(4):
        nbr = geo.face_nbr[:, l]
        inner = ~geo.face_is_wall[:, l]
        Gavg = 0.5 * (gradmu[inner] + gradmu[nbr[inner]])
        acc[inner] += (geo.face_area_vec[inner, l] * Gavg).sum(1)
    return acc / geo.vol


def point_forces(prm, C, rho, u, mu, gradC, gradp, gradrho, lapmu):
    """eq:G and eq:H at points with the given values and gradients, (n, 19) each."""
    Gu = gamma(u)
    G0 = W[None, :]

    def e_minus_u_dot(X):
        return edot(X) - np.sum(u * X, axis=1)[:, None]
    Phi_g = e_minus_u_dot(gradrho) * CS2 * (Gu - G0) + e_minus_u_dot(mu[:, None] * gradC) * Gu
    X = gradC - (C / (rho * CS2))[:, None] * (gradp - mu[:, None] * gradC)
    Phi_h = e_minus_u_dot(X) * Gu + prm.mobility * lapmu[:, None] * Gu
    return Phi_g, Phi_h


def rhs(mat, dt, psi_hat, Phi):
    """b_a = (-dt C_a - dt^2 D_a) psi_hat_a + (dt M10 + dt^2 K_a) Phi_a."""
    return np.stack([-dt * (mat.Ca[a] @ psi_hat[:, a]) - dt * dt * (mat.Da[a] @ psi_hat[:, a])
                     + dt * (mat.M10 @ Phi[:, a]) + dt * dt * (mat.Ka[a] @ Phi[:, a]) for a in range(Q)], axis=1)


def pcg(M, m, b, tol=1e-13, max_it=200):
    x = b / m
    r = b - M @ x
    bn = np.sqrt(np.sum(b * b))
    if bn == 0.0:
        return x
    z = r / m
    pdir = z.copy()
    rz = np.sum(r * z)
    for _ in range(max_it):
        if np.sqrt(np.sum(r * r)) <= tol * bn:
            return x
        q = M @ pdir
        alpha = rz / np.sum(pdir * q)
        x = x + alpha * pdir
        r = r - alpha * q
        z = r / m
        rz_new = np.sum(r * z)
        pdir = z + (rz_new / rz) * pdir
        rz = rz_new
    if np.sqrt(np.sum(r * r)) <= tol * bn:
        return x
    raise RuntimeError("PCG did not converge")


class Oracle3D:
    """State: (g, h), each (N, 19), in the variables of eqn::new_variable."""

    def __init__(self, mesh, phys, omega_c, tol=1e-13, with_matrices=True):
        self.geo = Geometry(mesh)
        self.mat = Matrices(self.geo) if with_matrices else None
        self.prm = Params(phys.sigma, phys.xi, phys.mobility, phys.rho_l, phys.rho_v, phys.nu_l, phys.nu_v, phys.dt)
        om = np.zeros(self.geo.N)
        om[self.geo.is_wall_node] = np.asarray(omega_c)[self.geo.is_wall_node]
        # Young: phi_c = Omega_c sqrt(2 kappa beta) (Sec. II.B); eq. bc2 uses phi_c / kappa
        self.bc = om * np.sqrt(2.0 * self.prm.kappa * self.prm.beta) / self.prm.kappa if self.prm.kappa > 0 else 0 * om
        self.tol = tol

    def init_state(self, C, u=None, p=None):
        N = self.geo.N
        u = np.zeros((N, 3)) if u is None else np.asarray(u)
        p = np.zeros(N) if p is None else np.asarray(p)
        g, h = equilibria(np.asarray(C), p, density(np.asarray(C), self.prm), u)
        return wall_operator(self.geo, g), wall_operator(self.geo, h)

    def fields(self, g, h):
        geo, prm = self.geo, self.prm
        C, p, rho, u = moments(g, h, prm)
        gradC = element_gradient(geo, C)
        lapC = laplacian_C(geo, C, gradC, self.bc)
        mu = chemical_potential(prm, C, lapC)
        gradmu = element_gradient(geo, mu)
        lapmu = laplacian_mu(geo, gradmu)
        gradp = element_gradient(geo, p)
        gradrho = element_gradient(geo, rho)
        bary = lambda f: f[geo.tet].mean(1)
        Phi_g, Phi_h = point_forces(prm, bary(C), bary(rho), bary(u), bary(mu), gradC, gradp, gradrho, lapmu)
        return dict(C=C, p=p, rho=rho, u=u, gradC=gradC, lapC=lapC, mu=mu, gradmu=gradmu, lapmu=lapmu,
                    gradp=gradp, tau=relaxation_time(C, prm), Phi_g=Phi_g, Phi_h=Phi_h)

    def step(self, g, h, return_fields=False):
        f = self.fields(g, h)
        g_eq, h_eq = equilibria(f["C"], f["p"], f["rho"], f["u"])
        g_hat, h_hat = collide(g, g_eq, f["tau"]), collide(h, h_eq, f["tau"])
        dt = self.prm.dt
        b_g, b_h = rhs(self.mat, dt, g_hat, f["Phi_g"]), rhs(self.mat, dt, h_hat, f["Phi_h"])
        d_g = np.stack([pcg(self.mat.M11, self.mat.lumped, b_g[:, a], self.tol) for a in range(Q)], 1)
        d_h = np.stack([pcg(self.mat.M11, self.mat.lumped, b_h[:, a], self.tol) for a in range(Q)], 1)
        g_new, h_new = wall_operator(self.geo, g_hat + d_g), wall_operator(self.geo, h_hat + d_h)
        if return_fields:
            f.update(g_hat=g_hat, h_hat=h_hat, b_g=b_g, b_h=b_h, d_g=d_g, d_h=d_h)
            return g_new, h_new, f
        return g_new, h_new

    def run(self, g, h, n):
        for _ in range(n):
            g, h = self.step(g, h)
        return g, h

    def mass(self, h):
        return float(np.sum(self.mat.lumped * h.sum(axis=1)))

    def diagnostics(self, g, h):
        C, p, rho, u = moments(g, h, self.prm)
        uu = np.sum(u * u, axis=1)
        return dict(mass=float(np.sum(self.mat.lumped * C)), mean_ke=float(0.5 * np.sum(rho * uu) / self.geo.N),
                    max_u=float(np.sqrt(uu.max())))


__all__ = ["E", "W", "Q", "CS2", "OPPOSITE", "Geometry", "Matrices", "Oracle3D", "Params", "gamma", "equilibria",
           "moments", "wall_flux", "laplacian_C", "laplacian_mu", "element_gradient", "point_forces", "rhs", "pcg",
           "wall_operator", "collide", "triangle_monomial"]
