"""Plain FP64 CPU oracle of the characteristic-based FE-LBM time step
(Matin, Misztal, Hernandez-Garcia, Mathiesen, arXiv:1708.04678).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this module; only the tests, the smoke check and the benchmark's
CPU-baseline leg use it.  It shares no code with the GPU library: it reads the
same seeded mesh and input arrays, and nothing else.

Formulation, chosen to be checkable by eye against the paper rather than fast:
  * the finite element matrices M11, M10, C_a, D_a, K_a of Sec. II.C
    (eq:fem_matrices) are assembled explicitly as scipy sparse matrices from
    their element integrals, and the weak form (eq:galerkin_lbm) is applied
    as sparse matrix-vector products;
  * the mass-matrix system is solved by preconditioned conjugate gradients
    with the lumped mass vector as preconditioner (end of Sec. II.C);
  * the Laplacians of Sec. II.D enumerate the outer edges of each vertex
    patch / each element and integrate grad(.) . n over them with explicit
    outward normals.

Every array operation is written so that complex inputs propagate
analytically (no abs, max, conj or branch on values inside a step), so the
complex-step method gives the exact forward-mode tangent of a step.

Readings of points the paper leaves open (each used identically on both
sides of every parity test):
  R1  weak form: the force enters as +(dt M10 + dt^2 K_a) Phi; the printed
      minus sign on dt M10 contradicts the streaming equation (eqn::stream)
      integrated by parts and the static-interface balance of Sec. II.C.
      The population vector on the right-hand side is the post-collision one.
  R2  nodal Laplacian of C: the gradient on an interior outer edge is the
      average of the two adjacent element gradients (as the paper states for
      the Laplacian of mu); wall edges of the patch, including the wall
      edges incident to the centre node, carry the wetting flux.
  R3  wetting flux: eq. bc2 holds with n pointing into the fluid, so the
      outward flux through a wall edge is -(1/kappa) int phi_c (C - C^2) ds,
      integrated exactly (Simpson) with phi_c and C linear along the edge;
      phi_c = Omega_c sqrt(2 kappa beta) per wall node.
  R4  wall operator ("bounce-back"): at wall nodes every opposite pair of g
      and of h is replaced by its mean, after every update and at init.
  R5  forces per element use the barycentric values of the P1 fields and the
      element gradients; grad(rho) is the gradient of the P1 field rho.
  R6  velocity is the literal first moment over c_s^2 rho (no half-force
      shift); the initial populations are the equilibria of (C, u, p).
  R7  solver: initial guess = lumped solve b/m; stop at ||r||_2 <= tol ||b||_2.

The nodal-force scheme (the comparison column of the parasitic-current table,
Sec. III.A; force_scheme="nodal") is not specified in the paper beyond
"the same discretization scheme for the force terms" as for the populations:
  N1  the forces are P1 fields, F_a(x) = N1(x)^T F_a, in the same streaming
      step: the weak form becomes +(dt M11 + dt^2 K1_a) F_a with
      K1_a = 1/2 int (e_a . grad N1) N1^T;
  N2  nodal grad C, grad p, grad rho: area-weighted means of the element
      gradients over the vertex patch (the lumped L2 projection of P0 onto P1);
  N3  nodal lap mu: the vertex-patch operator of eqn:lapl_int_mp applied to
      mu, with zero flux through wall edges (eqn:bc1);
  N4  F at node i: eq:G and eq:H with the nodal values of the fields.

The comparison scheme of the authors' earlier work integrates the nodal force
locally in the collision step instead (force_scheme="nodal_collide"):
  NC1 the trapezoid rule of eqn::integrated is applied to F as to the BGK
      term, and the new variable absorbs both: psi_bar = psi + dt/2 (Omega - F).
      Then psi_bar(x + dt e, t + dt) = psi_hat(x, t) with the collision
      psi_hat = psi_bar - (psi_bar - psi_eq + dt/2 F)/(tau + 1/2) + dt F,
      and the streaming is eqn::stream without the force;
  NC2 F at the nodes as in N2-N4;
  NC3 the moments of psi_bar then carry half the force's moments:
      rho u = sum e g_bar / c_s^2 + dt/2 mu grad C (first moment of F_g),
      p = sum g_bar + dt/2 c_s^2 u . grad rho (zeroth moment of F_g);
      C = sum h_bar + dt/2 M lap mu would make the composition implicit, so
      the fields use C = sum h_bar and only the h equilibrium of the
      collision uses C* = C + dt/2 M lap mu, which gives
      sum_a h_hat = sum_a h_bar + dt M lap mu exactly (mass conserving);
  NC4 wall nodes are at rest (the wall operator zeroes the first moments):
      u = 0 there, F_g = 0 and F_h keeps its even part M lap mu w_a only;
  NC5 initial state: at equilibrium Omega = 0, so psi_bar^0 = psi_eq - dt/2 F
      with F from the given (C, u, p); for h only the part of F_h with zero
      sum (the (e - u) . X Gamma term) is subtracted, so that sum h_bar^0 = C.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

# ---------------------------------------------------------------------------
# D2Q9 lattice (textbook constants; the paper uses D3Q19 in 3-D, Sec. II.A)
# ---------------------------------------------------------------------------
E = np.array([[0, 0], [1, 0], [0, 1], [-1, 0], [0, -1], [1, 1], [-1, 1], [-1, -1], [1, -1]], dtype=np.float64)
W = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
CS2 = 1.0 / 3.0
OPPOSITE = np.array([0, 3, 4, 1, 2, 7, 8, 5, 6])
Q = 9


# ---------------------------------------------------------------------------
# Parameters (Sec. II intro and II.A-B)
# ---------------------------------------------------------------------------
@dataclass
class Params:
    kappa: float
    beta: float
    mobility: float
    rho_l: float
    rho_v: float
    tau_l: float
    tau_v: float
    dt: float

    @staticmethod
    def from_physics(sigma, xi, mobility, rho_l, rho_v, nu_l, nu_v, dt):
        # xi = sqrt(8 kappa / beta), sigma = sqrt(2 kappa beta) / 6  (Sec. II, after eqn:mp_mu)
        # => kappa = 3 sigma xi / 2, beta = 12 sigma / xi
        kappa = 1.5 * sigma * xi
        beta = 12.0 * sigma / xi
        # nu = c_s^2 tau dt (Sec. II.A)
        return Params(kappa=kappa, beta=beta, mobility=mobility, rho_l=rho_l, rho_v=rho_v,
                      tau_l=nu_l / (CS2 * dt), tau_v=nu_v / (CS2 * dt), dt=dt)

    def phi_c(self, omega_c):
        # Young: cos(theta) = -Omega_c = -phi_c / sqrt(2 kappa beta)  (Sec. II.B)
        return np.asarray(omega_c) * np.sqrt(2.0 * self.kappa * self.beta)


# ---------------------------------------------------------------------------
# Mesh geometry (Sec. II.C: P1 shape functions on triangles)
# ---------------------------------------------------------------------------
class Geometry:
    def __init__(self, mesh):
        self.mesh = mesh
        xy, tri = mesh.xy, np.asarray(mesh.tri, dtype=np.int64)
        self.N, self.NT = xy.shape[0], tri.shape[0]
        self.tri = tri
        p = xy[tri].copy()                                     # (NT, 3, 2)
        if mesh.period_x > 0:                                  # minimum image w.r.t. vertex 0
            for k in (1, 2):
                p[:, k, 0] -= mesh.period_x * np.round((p[:, k, 0] - p[:, 0, 0]) / mesh.period_x)
        self.p = p
        x0, y0 = p[:, 0, 0], p[:, 0, 1]
        x1, y1 = p[:, 1, 0], p[:, 1, 1]
        x2, y2 = p[:, 2, 0], p[:, 2, 1]
        twoA = (x1 - x0) * (y2 - y0) - (x2 - x0) * (y1 - y0)
        if np.any(twoA <= 0):
            raise ValueError("non-positive triangle area")
        self.area = 0.5 * twoA
        # gradients of the barycentric (P1) shape functions, constant per element
        g = np.empty((self.NT, 3, 2))
        g[:, 0] = np.stack([y1 - y2, x2 - x1], 1) / twoA[:, None]
        g[:, 1] = np.stack([y2 - y0, x0 - x2], 1) / twoA[:, None]
        g[:, 2] = np.stack([y0 - y1, x1 - x0], 1) / twoA[:, None]
        self.gradN = g
        self.centroid = p.mean(axis=1)

        # edges: local edge l of element T is the one opposite vertex l,
        # running counter-clockwise from vertex l+1 to vertex l+2
        a = tri[:, [1, 2, 0]]
        b = tri[:, [2, 0, 1]]
        key = np.minimum(a, b) * self.N + np.maximum(a, b)           # (NT, 3)
        order = np.argsort(key.ravel(), kind="stable")
        ks = key.ravel()[order]
        self.edge_nbr = -np.ones((self.NT, 3), dtype=np.int64)      # element across local edge l
        same = ks[1:] == ks[:-1]
        i0, i1 = order[:-1][same], order[1:][same]
        self.edge_nbr.ravel()[i0] = i1 // 3
        self.edge_nbr.ravel()[i1] = i0 // 3
        # outward (from T) normal of local edge l scaled by the edge length
        pa = p[:, [1, 2, 0]]
        pb = p[:, [2, 0, 1]]
        d = pb - pa
        self.edge_normal = np.stack([d[..., 1], -d[..., 0]], -1)  # (NT, 3, 2) = |e| n_out
        self.edge_len = np.sqrt(d[..., 0] ** 2 + d[..., 1] ** 2)

        wall = np.asarray(mesh.wall_edges, dtype=np.int64)
        self.wall_edges = wall
        wkey = np.minimum(wall[:, 0], wall[:, 1]) * self.N + np.maximum(wall[:, 0], wall[:, 1])
        self.edge_is_wall = np.isin(key, wkey)
        if np.any((self.edge_nbr < 0) & ~self.edge_is_wall):
            raise ValueError("boundary edge that is neither a wall nor periodic")
        wl = xy[wall[:, 1]] - xy[wall[:, 0]]
        if mesh.period_x > 0:
            wl[:, 0] -= mesh.period_x * np.round(wl[:, 0] / mesh.period_x)
        self.wall_len = np.sqrt((wl ** 2).sum(1))
        self.is_wall_node = np.zeros(self.N, dtype=bool)
        self.is_wall_node[wall.ravel()] = True
        self.patch_volume = np.zeros(self.N)
        np.add.at(self.patch_volume, tri.ravel(), np.repeat(self.area, 3))


# ---------------------------------------------------------------------------
# Finite element matrices (eq:fem_matrices), assembled from element integrals
# ---------------------------------------------------------------------------
class Matrices:
    """M11 = int N1 N1^T, M10 = int N1 N0^T, C_r = int N1 d_r N1^T,
    D_sr = 1/2 int d_s N1 d_r N1^T, K_r = 1/2 int d_r N1 N0^T.
    With e_a = (e_x, e_y): C_a = sum_r e_r C_r, D_a = sum_{s,r} e_s e_r D_sr,
    K_a = sum_r e_r K_r (the index contractions of eq:fem_matrices)."""

    def __init__(self, geo: Geometry):
        N, NT, tri, A, G = geo.N, geo.NT, geo.tri, geo.area, geo.gradN
        I = np.repeat(tri, 3, axis=1).ravel()           # row vertex i of (i, j) pairs
        J = np.tile(tri, (1, 3)).ravel()                # column vertex j
        li = np.repeat(np.arange(3), 3)
        lj = np.tile(np.arange(3), 3)
        # int_T phi_i phi_j = A/12 (1 + delta_ij)
        m11 = (A[:, None] / 12.0) * (1.0 + (li == lj))[None, :]
        self.M11 = sp.csr_matrix((m11.ravel(), (I, J)), shape=(N, N))
        self.lumped = np.asarray(self.M11.sum(axis=1)).ravel()
        # int_T phi_i d_r phi_j = (A/3) d_r N_j
        self.C = [sp.csr_matrix((((A[:, None] / 3.0) * G[:, lj, r]).ravel(), (I, J)), shape=(N, N)) for r in (0, 1)]
        # 1/2 int_T d_s phi_i d_r phi_j = A/2 d_s N_i d_r N_j
        self.D = [[sp.csr_matrix((((A[:, None] / 2.0) * G[:, li, s] * G[:, lj, r]).ravel(), (I, J)), shape=(N, N))
                   for r in (0, 1)] for s in (0, 1)]
        Ie = tri.ravel()
        Te = np.repeat(np.arange(NT), 3)
        # int_T phi_i * 1 = A/3
        self.M10 = sp.csr_matrix((np.repeat(A / 3.0, 3), (Ie, Te)), shape=(N, NT))
        # 1/2 int_T d_r phi_i * 1 = A/2 d_r N_i
        self.K = [sp.csr_matrix((((A[:, None] / 2.0) * G[:, :, r]).ravel(), (Ie, Te)), shape=(N, NT)) for r in (0, 1)]
        self.Ca = [E[a, 0] * self.C[0] + E[a, 1] * self.C[1] for a in range(Q)]
        self.Da = [sum(E[a, s] * E[a, r] * self.D[s][r] for s in (0, 1) for r in (0, 1)) for a in range(Q)]
        self.Ka = [E[a, 0] * self.K[0] + E[a, 1] * self.K[1] for a in range(Q)]
        self._geo = geo
        self.K1a = None

    def nodal_force_matrices(self):
        """K1_r = 1/2 int d_r N1 N1^T (reading N1), built on first use:
        1/2 int_T d_r phi_i phi_j = (A/6) d_r N_i."""
        if self.K1a is None:
            geo = self._geo
            tri, A, G = geo.tri, geo.area, geo.gradN
            I = np.repeat(tri, 3, axis=1).ravel()
            J = np.tile(tri, (1, 3)).ravel()
            li = np.repeat(np.arange(3), 3)
            self.K1 = [sp.csr_matrix((((A[:, None] / 6.0) * G[:, li, r]).ravel(), (I, J)), shape=(geo.N, geo.N))
                       for r in (0, 1)]
            self.K1a = [E[a, 0] * self.K1[0] + E[a, 1] * self.K1[1] for a in range(Q)]
        return self.K1a


# ---------------------------------------------------------------------------
# Kinetic model (Sec. II.A)
# ---------------------------------------------------------------------------
def gamma(u):
    """Gamma_a(u) = w_a [1 + e.u/cs^2 + ((e.u)^2 - cs^2 u.u)/(2 cs^4)], shape (..., 9)."""
    eu = u[..., 0, None] * E[:, 0] + u[..., 1, None] * E[:, 1]
    uu = (u[..., 0] * u[..., 0] + u[..., 1] * u[..., 1])[..., None]
    return W * (1.0 + eu / CS2 + (eu * eu - CS2 * uu) / (2.0 * CS2 * CS2))


def density(C, prm: Params):
    # rho = C rho_l + (1 - C) rho_v  (after eqn:mp_ns)
    return C * prm.rho_l + (1.0 - C) * prm.rho_v


def moments(g, h, prm: Params):
    """C = sum h, p = sum g, rho u = (1/cs^2) sum e g  (eq:velocity, eq:pressure); g, h: (N, 9)."""
    C = h.sum(axis=1)
    p = g.sum(axis=1)
    rho = density(C, prm)
    mom = np.stack([g @ E[:, 0], g @ E[:, 1]], axis=1) / CS2
    u = mom / rho[:, None]
    return C, p, rho, u


def relaxation_time(C, prm: Params):
    # 1/tau = C/tau_l + (1 - C)/tau_v  (Sec. II.A)
    return 1.0 / (C / prm.tau_l + (1.0 - C) / prm.tau_v)


def equilibria(C, p, rho, u):
    """g_eq (eqn::g_eq) and h_eq = Gamma(u) C (eqn::f_eq)."""
    eu = u[:, 0, None] * E[:, 0] + u[:, 1, None] * E[:, 1]
    uu = (u[:, 0] * u[:, 0] + u[:, 1] * u[:, 1])[:, None]
    g_eq = W * (p[:, None] + rho[:, None] * CS2 * (eu / CS2 + (eu * eu - CS2 * uu) / (2.0 * CS2 * CS2)))
    h_eq = gamma(u) * C[:, None]
    return g_eq, h_eq


def collide(psi, psi_eq, tau):
    """psi_hat = psi_bar - (psi_bar - psi_eq)/(tau + 0.5)  (eqn::collide)."""
    return psi - (psi - psi_eq) / (tau[:, None] + 0.5)


def collide_with_force(psi, psi_eq, F, tau, dt):
    """Collision with the force integrated locally (reading NC1):
    psi_hat = psi_bar - (psi_bar - psi_eq + dt/2 F)/(tau + 0.5) + dt F."""
    return psi - (psi - psi_eq + 0.5 * dt * F) / (tau[:, None] + 0.5) + dt * F


def wall_operator(geo: Geometry, psi):
    """Reading R4: replace each opposite pair at wall nodes by the pair mean."""
    out = psi.copy()
    w = geo.is_wall_node
    for a in range(1, Q):
        b = OPPOSITE[a]
        out[w, a] = 0.5 * (psi[w, a] + psi[w, b])
    return out


# ---------------------------------------------------------------------------
# Element gradients and Laplacians (Sec. II.C-D)
# ---------------------------------------------------------------------------
def element_gradient(geo: Geometry, f):
    """Constant gradient of the P1 interpolant of nodal f on each element, (NT, 2)."""
    return np.einsum("tl,tlr->tr", f[geo.tri], geo.gradN)


def wall_flux(C_a, C_b, r_a, r_b, length):
    """Outward flux int_e grad C . n_out ds on a wall edge from eq. bc2 with n
    pointing into the fluid (reading R3): -int (phi_c/kappa)(C - C^2) ds, with
    r = phi_c/kappa and C linear along the edge; Simpson's rule is exact for
    this cubic integrand."""
    f = lambda c, r: r * (c - c * c)
    C_m, r_m = 0.5 * (C_a + C_b), 0.5 * (r_a + r_b)
    return -length / 6.0 * (f(C_a, r_a) + 4.0 * f(C_m, r_m) + f(C_b, r_b))


def laplacian_C(geo: Geometry, C, gradC, bc):
    """Nodal Laplacian of C over the vertex patch (eqn:lapl_int_mp): the sum
    over the outer edges of the patch of int grad C . n, divided by the patch
    volume.  Outer edges are the edges opposite the centre node in every patch
    element, plus the wall edges incident to the centre node.  bc = phi_c/kappa
    per node (read at wall nodes)."""
    flux = np.zeros(geo.N, dtype=np.result_type(C, gradC))
    tri = geo.tri
    for l in range(3):
        k = tri[:, l]                               # patch centre
        nbr = geo.edge_nbr[:, l]
        on_wall = geo.edge_is_wall[:, l]
        inner = ~on_wall
        Gavg = 0.5 * (gradC[inner] + gradC[nbr[inner]])
        fl = np.zeros(geo.NT, dtype=flux.dtype)
        fl[inner] = (geo.edge_normal[inner, l] * Gavg).sum(1)
        a, b = tri[on_wall, (l + 1) % 3], tri[on_wall, (l + 2) % 3]
        fl[on_wall] = wall_flux(C[a], C[b], bc[a], bc[b], geo.edge_len[on_wall, l])
        np.add.at(flux, k, fl)
    a, b = geo.wall_edges[:, 0], geo.wall_edges[:, 1]
    fw = wall_flux(C[a], C[b], bc[a], bc[b], geo.wall_len)
    np.add.at(flux, a, fw)
    np.add.at(flux, b, fw)
    return flux / geo.patch_volume


def chemical_potential(prm: Params, C, lapC):
    # mu = 2 beta C (C - 1)(2C - 1) - kappa lap C  (eqn:mp_mu)
    return 2.0 * prm.beta * C * (C - 1.0) * (2.0 * C - 1.0) - prm.kappa * lapC


def laplacian_mu(geo: Geometry, gradmu):
    """Element Laplacian of mu (Sec. II.D): sum over the element's edges of
    |e| n . (average of the two adjacent element gradients), zero on wall
    edges (eqn:bc1), divided by the element area."""
    acc = np.zeros(geo.NT, dtype=gradmu.dtype)
    for l in range(3):
        nbr = geo.edge_nbr[:, l]
        inner = ~geo.edge_is_wall[:, l]
        Gavg = 0.5 * (gradmu[inner] + gradmu[nbr[inner]])
        acc[inner] += (geo.edge_normal[inner, l] * Gavg).sum(1)
    return acc / geo.area


# ---------------------------------------------------------------------------
# Element (P0) forces, eq:G and eq:H at barycentric values (eq:intF, reading R5)
# ---------------------------------------------------------------------------
def point_forces(prm: Params, C, rho, u, mu, gradC, gradp, gradrho, lapmu):
    """eq:G and eq:H at a set of points given the values of C, rho, u, mu,
    grad C, grad p, grad rho and lap mu there; (n, 9) each."""
    Gu = gamma(u)                                        # (n, 9)
    G0 = W[None, :]
    # (e_a - u) . X for a vector X per point
    def edot(X):
        return (E[:, 0][None, :] - u[:, 0, None]) * X[:, 0, None] + (E[:, 1][None, :] - u[:, 1, None]) * X[:, 1, None]
    # eq:G: (e - u) . [grad rho c_s^2 (Gamma(u) - Gamma(0)) + mu grad C Gamma(u)]
    Phi_g = edot(gradrho) * CS2 * (Gu - G0) + edot(mu[:, None] * gradC) * Gu
    # eq:H: (e - u) . [grad C - C/(rho c_s^2)(grad p - mu grad C)] Gamma(u) + M lap mu Gamma(u)
    X = gradC - (C / (rho * CS2))[:, None] * (gradp - mu[:, None] * gradC)
    Phi_h = edot(X) * Gu + prm.mobility * lapmu[:, None] * Gu
    return Phi_g, Phi_h


def element_forces(geo: Geometry, prm: Params, C, rho, u, mu, gradC, gradp, gradrho, lapmu):
    """P0 forces: eq:G and eq:H at the barycentric values of the P1 fields with
    the element gradients (reading R5), (NT, 9) each."""
    return point_forces(prm, C[geo.tri].mean(1), rho[geo.tri].mean(1), u[geo.tri].mean(1), mu[geo.tri].mean(1),
                        gradC, gradp, gradrho, lapmu)


# ---------------------------------------------------------------------------
# Nodal (P1) forces, the comparison scheme of the parasitic-current table
# (readings N1-N4)
# ---------------------------------------------------------------------------
def nodal_average(geo: Geometry, elem_vec):
    """Area-weighted mean over each vertex patch of an element (P0) field
    (reading N2), (N, ...)."""
    shape = (-1,) + (1,) * (elem_vec.ndim - 1)
    acc = np.zeros((geo.N,) + elem_vec.shape[1:], dtype=elem_vec.dtype)
    weighted = geo.area.reshape(shape) * elem_vec
    for l in range(3):
        np.add.at(acc, geo.tri[:, l], weighted)
    return acc / geo.patch_volume.reshape(shape)


def nodal_laplacian_mu(geo: Geometry, mu, gradmu):
    """Vertex-patch Laplacian of mu (eqn:lapl_int_mp) with zero flux through
    wall edges (eqn:bc1) (reading N3), (N,)."""
    return laplacian_C(geo, mu, gradmu, np.zeros(geo.N))


# ---------------------------------------------------------------------------
# Streaming in weak form (eq:galerkin_lbm, reading R1) and the PCG solve
# ---------------------------------------------------------------------------
def rhs(mat: Matrices, dt, psi_hat, Phi):
    """b_a = (-dt C_a - dt^2 D_a) psi_hat_a + (dt M10 + dt^2 K_a) Phi_a, (N, 9)."""
    cols = []
    for a in range(Q):
        b = -dt * (mat.Ca[a] @ psi_hat[:, a]) - dt * dt * (mat.Da[a] @ psi_hat[:, a])
        b = b + dt * (mat.M10 @ Phi[:, a]) + dt * dt * (mat.Ka[a] @ Phi[:, a])
        cols.append(b)
    return np.stack(cols, axis=1)


def rhs_nodal(mat: Matrices, dt, psi_hat, F):
    """b_a = (-dt C_a - dt^2 D_a) psi_hat_a + (dt M11 + dt^2 K1_a) F_a with the
    force a P1 field (reading N1), (N, 9)."""
    K1a = mat.nodal_force_matrices()
    cols = []
    for a in range(Q):
        b = -dt * (mat.Ca[a] @ psi_hat[:, a]) - dt * dt * (mat.Da[a] @ psi_hat[:, a])
        b = b + dt * (mat.M11 @ F[:, a]) + dt * dt * (K1a[a] @ F[:, a])
        cols.append(b)
    return np.stack(cols, axis=1)


class SolverError(RuntimeError):
    pass


def pcg(M, m, b, tol=1e-13, max_it=100):
    """Conjugate gradients on M x = b with preconditioner diag(m) (the lumped
    mass vector), x0 = b/m; plain (non-conjugating) products so that a
    complex-step perturbation propagates analytically."""
    x = b / m
    r = b - M @ x
    bn = np.sqrt(np.sum(b.real * b.real))
    if bn == 0.0:
        return x, 0
    z = r / m
    pdir = z.copy()
    rz = np.sum(r * z)
    for it in range(1, max_it + 1):
        if np.sqrt(np.sum(r.real * r.real)) <= tol * bn:
            return x, it - 1
        q = M @ pdir
        alpha = rz / np.sum(pdir * q)
        x = x + alpha * pdir
        r = r - alpha * q
        z = r / m
        rz_new = np.sum(r * z)
        pdir = z + (rz_new / rz) * pdir
        rz = rz_new
    if np.sqrt(np.sum(r.real * r.real)) <= tol * bn:
        return x, max_it
    raise SolverError("PCG did not converge")


# ---------------------------------------------------------------------------
# The model: state = (g, h), each (N, 9), in the "bar" variables of eqn::new_variable
# ---------------------------------------------------------------------------
class Oracle:
    def __init__(self, mesh, phys, omega_c, tol=1e-13, force_scheme="mixed"):
        if force_scheme not in ("mixed", "nodal", "nodal_collide"):
            raise ValueError("force_scheme is 'mixed' (P0 element forces), 'nodal' (P1 nodal forces in the streaming "
                             "step) or 'nodal_collide' (nodal forces integrated in the collision step)")
        self.force_scheme = force_scheme
        self.geo = Geometry(mesh)
        self.mat = Matrices(self.geo)
        self.prm = Params.from_physics(phys.sigma, phys.xi, phys.mobility, phys.rho_l, phys.rho_v,
                                       phys.nu_l, phys.nu_v, phys.dt)
        self.set_wetting(omega_c)
        self.tol = tol
        self.last_iterations = 0

    def set_wetting(self, omega_c):
        om = np.zeros(self.geo.N, dtype=np.result_type(omega_c, np.float64))
        om[self.geo.is_wall_node] = np.asarray(omega_c)[self.geo.is_wall_node]
        self.omega_c = om
        self.phi = self.prm.phi_c(om)
        if self.prm.kappa > 0:
            self.bc = self.phi / self.prm.kappa          # the coefficient phi_c/kappa of eq. bc2
        elif np.any(om != 0):
            raise ValueError("a wetting potential needs kappa > 0")
        else:
            self.bc = np.zeros_like(self.phi)

    def init_state(self, C, u=None, p=None):
        """psi_bar^0 = psi_eq(C, u, p) (reading R6), then the wall operator."""
        N = self.geo.N
        C = np.asarray(C)
        u = np.zeros((N, 2)) if u is None else np.asarray(u)
        p = np.zeros(N) if p is None else np.asarray(p)
        rho = density(C, self.prm)
        g, h = equilibria(C, p, rho, u)
        if self.force_scheme == "nodal_collide":
            # reading NC5: psi_bar^0 = psi_eq - dt/2 F, with F from the given fields
            geo, prm = self.geo, self.prm
            gradC = element_gradient(geo, C)
            mu = chemical_potential(prm, C, laplacian_C(geo, C, gradC, self.bc))
            f = self._collision_forces(C, rho, u, mu, gradC, element_gradient(geo, p), element_gradient(geo, rho),
                                       element_gradient(geo, mu))
            odd_h = f["F_h"] - prm.mobility * f["lapmu_n"][:, None] * gamma(u)
            odd_h[geo.is_wall_node] = 0.0
            g = g - 0.5 * prm.dt * f["F_g"]
            h = h - 0.5 * prm.dt * odd_h
        return wall_operator(self.geo, g), wall_operator(self.geo, h)

    def _collision_forces(self, C, rho, u, mu, gradC, gradp, gradrho, gradmu):
        """Nodal forces of the collision-step scheme (readings NC2, NC4)."""
        geo, prm = self.geo, self.prm
        wall = geo.is_wall_node
        gradC_n, gradp_n, gradrho_n = (nodal_average(geo, x) for x in (gradC, gradp, gradrho))
        lapmu_n = nodal_laplacian_mu(geo, mu, gradmu)
        F_g, F_h = point_forces(prm, C, rho, u, mu, gradC_n, gradp_n, gradrho_n, lapmu_n)
        F_g[wall] = 0.0
        F_h[wall] = prm.mobility * lapmu_n[wall, None] * W[None, :]
        return dict(gradC_n=gradC_n, gradp_n=gradp_n, gradrho_n=gradrho_n, lapmu_n=lapmu_n, F_g=F_g, F_h=F_h,
                    C_star=C + 0.5 * prm.dt * prm.mobility * lapmu_n)

    def fields(self, g, h):
        """Everything the step derives from (g, h) before streaming."""
        geo, prm = self.geo, self.prm
        C, p, rho, u = moments(g, h, prm)
        gradC = element_gradient(geo, C)
        lapC = laplacian_C(geo, C, gradC, self.bc)
        mu = chemical_potential(prm, C, lapC)
        gradmu = element_gradient(geo, mu)
        lapmu = laplacian_mu(geo, gradmu)
        gradp = element_gradient(geo, p)
        gradrho = element_gradient(geo, rho)
        out = dict(C=C, p=p, rho=rho, u=u, gradC=gradC, lapC=lapC, mu=mu, gradmu=gradmu, lapmu=lapmu,
                   gradp=gradp, gradrho=gradrho, tau=relaxation_time(C, prm))
        if self.force_scheme == "mixed":
            out["Phi_g"], out["Phi_h"] = element_forces(geo, prm, C, rho, u, mu, gradC, gradp, gradrho, lapmu)
        elif self.force_scheme == "nodal_collide":
            # reading NC3: the half-force moments of psi_bar; walls at rest (NC4)
            wall = geo.is_wall_node
            gradC_n, gradrho_n = nodal_average(geo, gradC), nodal_average(geo, gradrho)
            u = u + (0.5 * prm.dt * mu / rho)[:, None] * gradC_n
            u[wall] = 0.0
            p = p + 0.5 * prm.dt * CS2 * (u[:, 0] * gradrho_n[:, 0] + u[:, 1] * gradrho_n[:, 1])
            gradp = element_gradient(geo, p)
            out.update(u=u, p=p, gradp=gradp)
            out.update(self._collision_forces(C, rho, u, mu, gradC, gradp, gradrho, gradmu))
        else:
            gradC_n, gradp_n, gradrho_n = (nodal_average(geo, x) for x in (gradC, gradp, gradrho))
            lapmu_n = nodal_laplacian_mu(geo, mu, gradmu)
            out.update(gradC_n=gradC_n, gradp_n=gradp_n, gradrho_n=gradrho_n, lapmu_n=lapmu_n)
            out["F_g"], out["F_h"] = point_forces(prm, C, rho, u, mu, gradC_n, gradp_n, gradrho_n, lapmu_n)
        return out

    def step(self, g, h, return_fields=False):
        """One time step: collision (eqn::collide) then Galerkin streaming
        with the element force (eqn::stream, eq:galerkin_lbm; the nodal force
        of readings N1-N4 for force_scheme="nodal"), the mass matrix solve and
        the wall operator."""
        f = self.fields(g, h)
        dt = self.prm.dt
        if self.force_scheme == "nodal_collide":
            g_eq, h_eq = equilibria(f["C_star"], f["p"], f["rho"], f["u"])
            g_hat = collide_with_force(g, g_eq, f["F_g"], f["tau"], dt)
            h_hat = collide_with_force(h, h_eq, f["F_h"], f["tau"], dt)
        else:
            g_eq, h_eq = equilibria(f["C"], f["p"], f["rho"], f["u"])
            g_hat = collide(g, g_eq, f["tau"])
            h_hat = collide(h, h_eq, f["tau"])
        if self.force_scheme == "mixed":
            b_g = rhs(self.mat, dt, g_hat, f["Phi_g"])
            b_h = rhs(self.mat, dt, h_hat, f["Phi_h"])
        elif self.force_scheme == "nodal_collide":
            zero = np.zeros((self.geo.NT, Q))
            b_g = rhs(self.mat, dt, g_hat, zero)
            b_h = rhs(self.mat, dt, h_hat, zero)
        else:
            b_g = rhs_nodal(self.mat, dt, g_hat, f["F_g"])
            b_h = rhs_nodal(self.mat, dt, h_hat, f["F_h"])
        d_g = np.empty_like(b_g)
        d_h = np.empty_like(b_h)
        its = 0
        for a in range(Q):
            d_g[:, a], i1 = pcg(self.mat.M11, self.mat.lumped, b_g[:, a], self.tol)
            d_h[:, a], i2 = pcg(self.mat.M11, self.mat.lumped, b_h[:, a], self.tol)
            its = max(its, i1, i2)
        self.last_iterations = its
        g_new = wall_operator(self.geo, g_hat + d_g)
        h_new = wall_operator(self.geo, h_hat + d_h)
        if return_fields:
            f.update(g_hat=g_hat, h_hat=h_hat, b_g=b_g, b_h=b_h, d_g=d_g, d_h=d_h)
            return g_new, h_new, f
        return g_new, h_new

    def run(self, g, h, n):
        for _ in range(n):
            g, h = self.step(g, h)
        return g, h

    # -- diagnostics (Sec. III) ---------------------------------------------
    def mass(self, h):
        """Total composition int C = sum_i m_i C_i (m = lumped mass)."""
        return float(np.sum(self.mat.lumped * h.sum(axis=1).real))

    def diagnostics(self, g, h, band=None):
        C, p, rho, u = moments(g.real, h.real, self.prm)
        if self.force_scheme == "nodal_collide":
            u = self.fields(g.real, h.real)["u"]
        uu = u[:, 0] ** 2 + u[:, 1] ** 2
        out = dict(mass=float(np.sum(self.mat.lumped * C)), mean_ke=float(0.5 * np.sum(rho * uu) / self.geo.N),
                   max_u=float(np.sqrt(uu.max())))
        if band is not None:
            xc, yc, R, xi = band
            dx = self.geo.mesh.xy[:, 0] - xc
            if self.geo.mesh.period_x > 0:
                dx -= self.geo.mesh.period_x * np.round(dx / self.geo.mesh.period_x)
            d = np.sqrt(dx ** 2 + (self.geo.mesh.xy[:, 1] - yc) ** 2)
            sel = (d >= R - xi) & (d <= R + xi)
            out["band_ke"] = float(np.mean(rho[sel] * uu[sel])) if sel.any() else 0.0
        return out


# ---------------------------------------------------------------------------
# Contact angle from the C = 0.5 contour (Sec. III.B), flat bottom wall y = 0
# ---------------------------------------------------------------------------
def contact_angle(mesh, C, level=0.5):
    """theta from droplet height h and base b on the C = level contour.  The
    printed formula evaluates to pi - theta on an exact circular cap; the
    cap identity tan(theta/2) = 2h/b is used instead (reading).  b comes from
    the contour's crossings of the wall, h from the contour apex."""
    xy = mesh.xy
    bottom = np.unique(mesh.wall_edges[mesh.wall_side == 0].ravel())
    order = bottom[np.argsort(xy[bottom, 0])]
    xs, cs = xy[order, 0], C[order]
    P = mesh.period_x
    crossings = []
    n = xs.size
    for k in range(n if P > 0 else n - 1):
        k2 = (k + 1) % n
        x1, x2 = xs[k], xs[k2] + (P if k2 == 0 else 0.0)
        c1, c2 = cs[k], cs[k2]
        if (c1 < level) != (c2 < level):
            crossings.append(x1 + (level - c1) / (c2 - c1) * (x2 - x1))
    if len(crossings) != 2:
        raise ValueError(f"expected two wall crossings, found {len(crossings)}")
    xl, xr = sorted(crossings)
    b = xr - xl
    # contour points on all element edges, take the highest one
    tri = mesh.tri
    best = 0.0
    for (i, j) in ((0, 1), (1, 2), (2, 0)):
        a, c = tri[:, i], tri[:, j]
        ca, cc = C[a], C[c]
        s = (ca < level) != (cc < level)
        t = (level - ca[s]) / (cc[s] - ca[s])
        y = xy[a[s], 1] + t * (xy[c[s], 1] - xy[a[s], 1])
        if y.size:
            best = max(best, float(y.max()))
    h = best
    return float(np.degrees(2.0 * np.arctan2(2.0 * h, b))), h, b
