"""Pins of the 3-D CPU oracle (D3Q19 on P1 tetrahedra) against what the paper
and mathematics fix.  Each function returns an error measure bounded by
tests/test_oracle3d_pins.py; tests/test_oracle3d_mutations.py plants mistakes
in the oracle and checks that a pin fails.  No expected value retypes an
oracle formula: closed forms, exact identities, brute-force quadrature and
continuum results."""
from __future__ import annotations

import numpy as np

from oracle import felbm3d_oracle as fo3
from workloads import make_physics
from workloads.mesh3d import TetMesh, droplet_field_3d, tet_box_mesh, wetting_from_angles_3d


def single_tet() -> TetMesh:
    xyz = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.0, 1.0, 0.0], [0.0, 0.0, 1.0]])
    tet = np.array([[0, 1, 2, 3]], dtype=np.int32)
    faces = np.array([[1, 2, 3], [0, 2, 3], [0, 1, 3], [0, 1, 2]], dtype=np.int32)
    return TetMesh(xyz=xyz, tet=tet, wall_faces=faces, wall_side=np.zeros(4, np.int8), period=(0.0, 0.0),
                   shape=(1, 1, 1))


def small_box(jitter=0.2, seed=3, n=4, nz=4):
    return tet_box_mesh(float(n), float(n), float(nz), n, n, nz, seed=[seed], jitter=jitter)


def _bary(P, x):
    A = np.vstack([P.T, np.ones(4)])
    return np.linalg.solve(A, np.array([x[0], x[1], x[2], 1.0]))


def _unwrapped(mesh, vs):
    P = mesh.xyz[vs].copy()
    for d, L in enumerate(mesh.period):
        if L > 0:
            P[:, d] -= L * np.round((P[:, d] - P[0, d]) / L)
    return P


def fem_bruteforce_error(mesh: TetMesh) -> float:
    """Dense M11, M10, C_r, D_sr, K_r by the 4-point tetrahedral rule (exact for
    degree 2), shape functions from a barycentric solve, gradients by central
    differences, against the oracle's assembled matrices."""
    N, NT = mesh.n_nodes, mesh.n_tets
    M11 = np.zeros((N, N)); M10 = np.zeros((N, NT))
    C = np.zeros((3, N, N)); D = np.zeros((3, 3, N, N)); K = np.zeros((3, N, NT))
    a, b = 0.5854101966249685, 0.1381966011250105
    for t, vs in enumerate(mesh.tet):
        P = _unwrapped(mesh, vs)
        vol = abs(np.linalg.det(np.vstack([P.T, np.ones(4)]))) / 6.0
        eps = 1e-6
        grads = np.zeros((4, 3))
        c = P.mean(0)
        for r in range(3):
            dx = np.zeros(3); dx[r] = eps
            grads[:, r] = (_bary(P, c + dx) - _bary(P, c - dx)) / (2 * eps)
        for q in range(4):
            lam_q = np.full(4, b); lam_q[q] = a
            xq = lam_q @ P
            lam = _bary(P, xq)
            wq = vol / 4.0
            for i in range(4):
                M10[vs[i], t] += wq * lam[i]
                for r in range(3):
                    K[r, vs[i], t] += 0.5 * wq * grads[i, r]
                for j in range(4):
                    M11[vs[i], vs[j]] += wq * lam[i] * lam[j]
                    for r in range(3):
                        C[r, vs[i], vs[j]] += wq * lam[i] * grads[j, r]
                        for s in range(3):
                            D[s, r, vs[i], vs[j]] += 0.5 * wq * grads[i, s] * grads[j, r]
    mat = fo3.Matrices(fo3.Geometry(mesh))
    errs = [abs(mat.M11.toarray() - M11).max(), abs(mat.M10.toarray() - M10).max()]
    for r in range(3):
        errs.append(abs(mat.C[r].toarray() - C[r]).max())
        errs.append(abs(mat.K[r].toarray() - K[r]).max())
        for s in range(3):
            errs.append(abs(mat.D[s][r].toarray() - D[s, r]).max())
    for al in range(fo3.Q):
        e = fo3.E[al]
        errs.append(abs(mat.Ca[al].toarray() - sum(e[r] * C[r] for r in range(3))).max())
        errs.append(abs(mat.Da[al].toarray() - sum(e[s] * e[r] * D[s, r] for s in range(3) for r in range(3))).max())
        errs.append(abs(mat.Ka[al].toarray() - sum(e[r] * K[r] for r in range(3))).max())
    return float(max(errs))


def single_tet_mass_error() -> float:
    """The reference tetrahedron (volume 1/6): int phi_i phi_j = 1/60 on the
    diagonal and 1/120 off it (hand-integrated), lumped mass 1/24 per vertex."""
    mat = fo3.Matrices(fo3.Geometry(single_tet()))
    ref = (np.ones((4, 4)) + np.eye(4)) / 120.0
    return float(max(abs(mat.M11.toarray() - ref).max(), abs(mat.lumped - 1.0 / 24.0).max()))


def identities_error() -> dict:
    mesh = small_box()
    geo = fo3.Geometry(mesh)
    mat = fo3.Matrices(geo)
    one = np.ones(geo.N)
    out = {"M11_one_is_lumped": abs(mat.M11 @ one - mat.lumped).max(),
           "lumped_sum_is_volume": abs(mat.lumped.sum() - 4.0 * 4.0 * 4.0),
           "D_one": max(abs(mat.Da[a] @ one).max() for a in range(fo3.Q)),
           "K_colsum": max(abs(one @ mat.Ka[a]).max() for a in range(fo3.Q))}
    z = mesh.xyz[:, 2]
    lin = 0.2 + 0.6 * z             # linear and periodic in x, y
    out["C_linear"] = max(abs(mat.Ca[a] @ lin - fo3.E[a, 2] * 0.6 * mat.lumped).max() for a in range(fo3.Q))
    s = 1.0 / np.sqrt(mat.lumped)
    ev = np.linalg.eigvalsh(s[:, None] * mat.M11.toarray() * s[None, :])
    out["wathen_low"] = max(0.0, 0.2 - ev.min())      # P1 tetrahedra: [1/5, 1]
    out["wathen_high"] = max(0.0, ev.max() - 1.0)
    return {k: float(v) for k, v in out.items()}


def lattice_identities_error() -> float:
    """D3Q19: weights sum to 1, isotropy of the second and fourth moments,
    opposite directions, and the equilibrium moments up to second order."""
    e, w = fo3.E, fo3.W
    d = np.eye(3)
    m4 = np.einsum("a,ai,aj,ak,al->ijkl", w, e, e, e, e)
    iso4 = fo3.CS2 ** 2 * (np.einsum("ij,kl->ijkl", d, d) + np.einsum("ik,jl->ijkl", d, d)
                           + np.einsum("il,jk->ijkl", d, d))
    rng = np.random.default_rng(5)
    n = 40
    C = rng.uniform(0, 1, n); p = rng.normal(0, 1e-3, n)
    u = rng.normal(0, 0.05, (n, 3))
    rho = 0.1 + 0.9 * C
    geq, heq = fo3.equilibria(C, p, rho, u)
    G = fo3.gamma(u)
    uu = u[:, :, None] * u[:, None, :]
    errs = [abs(w.sum() - 1), abs(np.einsum("a,ai,aj->ij", w, e, e) - fo3.CS2 * d).max(), abs(m4 - iso4).max(),
            abs(e[fo3.OPPOSITE] + e).max(), abs(np.einsum("a,ai->i", w, e)).max(),
            abs(heq.sum(1) - C).max(), abs(geq.sum(1) - p).max(),
            abs(geq @ e - (rho * fo3.CS2)[:, None] * u).max(), abs(G.sum(1) - 1).max(), abs(G @ e - u).max(),
            abs(np.einsum("na,ai,aj->nij", G, e, e) - (fo3.CS2 * d[None] + uu)).max(),
            abs(np.einsum("na,ai,aj->nij", geq, e, e) - fo3.CS2 * (p[:, None, None] * d[None]
                                                                   + rho[:, None, None] * uu)).max()]
    return float(max(errs))


def phys3d(sigma=0.01, mobility=0.02, dt=0.1):
    return make_physics(sigma=sigma, m_rho=10, m_nu=2, dt=dt, mobility=mobility)


def static_balance_drift(seed=3) -> float:
    """Sec. II.C: u = 0, p = 0, no surface tension, no mobility: with h = w C
    and g = 0 the P0 force balances the streaming of any P1 profile exactly."""
    mesh = small_box(seed=seed)
    o = fo3.Oracle3D(mesh, phys3d(sigma=0.0, mobility=0.0), np.zeros(mesh.n_nodes))
    C = np.random.default_rng(seed).uniform(0.0, 1.0, mesh.n_nodes)
    g, h = o.init_state(C)
    g1, h1 = o.step(g, h)
    return float(max(abs(h1 - h).max(), abs(g1 - g).max()) / abs(h).max())


def face_flux_quadrature_error() -> float:
    """The wetting flux through a triangle with C and phi_c/kappa linear on it
    against a 12 x 12 Gauss-Legendre rule on the square mapped onto the
    triangle (Duffy), for random vertex values and areas."""
    rng = np.random.default_rng(2)
    gx, gw = np.polynomial.legendre.leggauss(12)
    s, ws = 0.5 * (gx + 1), 0.5 * gw
    err = 0.0
    for _ in range(20):
        Cf, rf, area = rng.uniform(0, 1, 3), rng.normal(size=3), rng.uniform(0.1, 2.0)
        tot = 0.0
        for a, wa in zip(s, ws):
            for b, wb in zip(s, ws):
                l1, l2 = a, (1 - a) * b                  # Duffy map of the unit square onto the triangle
                lam = np.array([1 - l1 - l2, l1, l2])
                Cq, rq = lam @ Cf, lam @ rf
                tot += wa * wb * (1 - a) * rq * (Cq - Cq * Cq)
        exact = -2.0 * area * tot                     # reference triangle has area 1/2
        err = max(err, abs(fo3.wall_flux(Cf, rf, area) - exact))
    return float(err)


def uniform_box(n=8):
    return tet_box_mesh(float(n), float(n), float(n), n, n, n, seed=[0], jitter=0.0)


def laplacian_quadratic_error() -> float:
    """Nodal patch Laplacian (eqn:lapl_int_mp) and element Laplacian of mu
    (Sec. II.D) of the quadratics z^2, x^2, y^2 and x z on the uniform Kuhn
    mesh: the nodal one equals the exact Laplacian at every node two or more
    layers from the walls; the element one alternates between the six
    tetrahedra of a cell, and its volume average over each cell equals the
    exact Laplacian.  Returns the max error over the fields."""
    mesh = uniform_box()
    geo = fo3.Geometry(mesh)
    x, y, z = mesh.xyz.T
    cell = np.floor(geo.centroid + 1e-9).astype(int)
    key = (cell[:, 0] * 8 + cell[:, 1]) * 8 + cell[:, 2]
    # two or more layers from the walls and from the periodic seams (x^2, x z are not periodic)
    inner_c = np.all((cell >= 2) & (cell <= 5), axis=1)
    inner_n = np.all((mesh.xyz >= 2) & (mesh.xyz <= 5), axis=1)
    err = 0.0
    for f, ref in ((z * z, 2.0), (x * x, 2.0), (y * y, 2.0), (x * z, 0.0)):
        lapC = fo3.laplacian_C(geo, f, fo3.element_gradient(geo, f), np.zeros(geo.N))
        lapE = fo3.laplacian_mu(geo, fo3.element_gradient(geo, f))
        num = np.bincount(key[inner_c], weights=(geo.vol * lapE)[inner_c], minlength=512)
        den = np.bincount(key[inner_c], weights=geo.vol[inner_c], minlength=512)
        err = max(err, abs(lapC[inner_n] - ref).max(), abs(num[den > 0] / den[den > 0] - ref).max())
    return float(err)


def wall_linear_laplacian_error() -> float:
    """C = c0 + s z near the bottom wall with the wetting potential chosen so
    that eq. bc2 holds there (n into the fluid) and at the top: the patch
    integral of the linear field with the wetting flux vanishes at every
    wall node."""
    mesh = small_box(jitter=0.2)
    phys = phys3d()
    prm = fo3.Params(phys.sigma, phys.xi, phys.mobility, phys.rho_l, phys.rho_v, phys.nu_l, phys.nu_v, phys.dt)
    c0, s, lz = 0.3, 0.02, 4.0
    om = np.zeros(mesh.n_nodes)
    root = np.sqrt(2 * prm.kappa * prm.beta)
    om[mesh.wall_nodes(0)] = (s * prm.kappa / (c0 - c0 * c0)) / root
    ct = c0 + s * lz
    om[mesh.wall_nodes(1)] = (-s * prm.kappa / (ct - ct * ct)) / root
    o = fo3.Oracle3D(mesh, phys, om, with_matrices=False)
    C = c0 + s * mesh.xyz[:, 2]
    lap = fo3.laplacian_C(o.geo, C, fo3.element_gradient(o.geo, C), o.bc)
    return float(abs(lap).max())


def mass_drift(steps=10) -> float:
    mesh = small_box(n=6, nz=4)
    phys = phys3d()
    o = fo3.Oracle3D(mesh, phys, wetting_from_angles_3d(mesh, 60.0))
    g, h = o.init_state(droplet_field_3d(mesh, [(3.0, 3.0, 0.0, 2.5)], phys.xi))
    m0 = o.mass(h)
    g, h = o.run(g, h, steps)
    return float(abs(o.mass(h) - m0) / m0)


def wall_velocity_after_steps() -> float:
    mesh = small_box(n=6, nz=4)
    phys = phys3d()
    o = fo3.Oracle3D(mesh, phys, wetting_from_angles_3d(mesh, 60.0))
    g, h = o.init_state(droplet_field_3d(mesh, [(3.0, 3.0, 0.0, 2.5)], phys.xi))
    g, h = o.run(g, h, 3)
    u = fo3.moments(g, h, o.prm)[3]
    return float(abs(u[o.geo.is_wall_node]).max())


def laplace_jump(R: float, h: float, xi: float = 2.0):
    """3-D Laplace law for the tanh droplet of radius R (Sec. II): the pressure
    jump balancing -C grad mu is p_in - p_out = int C dmu/dr dr across the
    interface.  Over the shell R/2 <= r <= R + 2 xi (the integrand vanishes at
    both ends to e^-8), the discrete value sum_T V_T C_T (grad mu_T . r_hat) /
    (4 pi r_T^2) with the oracle's element gradients of mu is compared with the
    same integral of the continuum fields of this profile, mu = 2 beta C (C-1)
    (2C-1) - kappa (C'' + 2 C'/r) by fine 1-D quadrature; that integral tends
    to 2 sigma / R as xi / R -> 0.  Returns (discrete / continuum,
    continuum R / (2 sigma))."""
    L = 2.0 * (R + 2.0 * xi)
    n = int(round(L / h))
    mesh = tet_box_mesh(L, L, L, n, n, n, seed=[8], jitter=0.0)
    phys = make_physics(sigma=0.01, m_rho=10, m_nu=2, dt=0.1, xi=xi)
    o = fo3.Oracle3D(mesh, phys, np.zeros(mesh.n_nodes), with_matrices=False)
    c = np.array([L / 2, L / 2, L / 2])
    C = droplet_field_3d(mesh, [(c[0], c[1], c[2], R)], phys.xi)
    g, hh = o.init_state(C)
    f = o.fields(g, hh)
    geo = o.geo
    rv = geo.centroid - c
    rr = np.sqrt((rv ** 2).sum(1))
    shell = (rr >= 0.5 * R) & (rr <= R + 2.0 * xi)
    Cb = C[geo.tet].mean(1)
    dp = np.sum((geo.vol * Cb * (f["gradmu"] * rv).sum(1) / rr ** 3)[shell]) / (4 * np.pi)
    kap, bet = 1.5 * phys.sigma * xi, 12.0 * phys.sigma / xi
    r = np.linspace(0.5 * R, R + 2.0 * xi, 200001)
    t = np.tanh(2.0 * (R - r) / xi)
    Cr = 0.5 + 0.5 * t
    d1 = -(1.0 - t * t) / xi
    d2 = -4.0 * t * (1.0 - t * t) / xi ** 2
    mu = 2 * bet * Cr * (Cr - 1) * (2 * Cr - 1) - kap * (d2 + 2.0 * d1 / r)
    cont = np.trapezoid(Cr * np.gradient(mu, r), r)
    return float(dp / cont), float(cont * R / (2 * phys.sigma))


def shear_wave_viscosity_ratio(tau=2.0, n_steps=300) -> float:
    """Lowest channel shear mode u_x = U sin(pi z / H) between no-slip walls in
    single-phase liquid: decay rate nu (pi/H)^2 with nu = c_s^2 tau dt."""
    H = 12
    mesh = tet_box_mesh(3.0, 3.0, float(H), 3, 3, H, seed=[13])
    dt = 0.1
    phys = phys3d(dt=dt)
    phys.nu_l = fo3.CS2 * tau * dt
    o = fo3.Oracle3D(mesh, phys, np.zeros(mesh.n_nodes))
    k = np.pi / H
    z = mesh.xyz[:, 2]
    u = np.zeros((mesh.n_nodes, 3)); u[:, 0] = 1e-3 * np.sin(k * z)
    g, h = o.init_state(np.ones(mesh.n_nodes), u=u)
    s = np.sin(k * z)

    def amp(g, h):
        return np.sum(fo3.moments(g, h, o.prm)[3][:, 0] * s) / np.sum(s * s)
    g, h = o.run(g, h, 50)
    a1 = amp(g, h)
    g, h = o.run(g, h, n_steps)
    a2 = amp(g, h)
    return float(np.log(a1 / a2) / (n_steps * dt) / (phys.nu_l * k * k))


def mixture_viscosity_ratio(tau_l=2.0, tau_v=0.5, n_steps=300, H=12) -> float:
    """The same shear mode in a uniform mixture C = 1/2 (mobility 0; mu = 0
    and grad C = 0 there, so C stays uniform) of density (rho_l + rho_v)/2 =
    0.55: the decay rate gives nu = c_s^2 tau(1/2) dt with the relaxation time
    of Sec. II.A, 1/tau = C/tau_l + (1 - C)/tau_v (tau(1/2) = 0.8 here).
    Returns the measured decay rate over nu (pi/H)^2."""
    mesh = tet_box_mesh(3.0, 3.0, float(H), 3, 3, H, seed=[13])
    dt = 0.1
    phys = make_physics(sigma=0.01, m_rho=10, m_nu=1, dt=dt, mobility=0.0)
    phys.nu_l, phys.nu_v = fo3.CS2 * tau_l * dt, fo3.CS2 * tau_v * dt
    nu = fo3.CS2 * dt / (0.5 / tau_l + 0.5 / tau_v)
    o = fo3.Oracle3D(mesh, phys, np.zeros(mesh.n_nodes))
    k = np.pi / H
    z = mesh.xyz[:, 2]
    u = np.zeros((mesh.n_nodes, 3)); u[:, 0] = 1e-3 * np.sin(k * z)
    g, h = o.init_state(np.full(mesh.n_nodes, 0.5), u=u)
    s = np.sin(k * z)

    def amp(g, h):
        return np.sum(fo3.moments(g, h, o.prm)[3][:, 0] * s) / np.sum(s * s)
    g, h = o.run(g, h, 50)
    a1 = amp(g, h)
    g, h = o.run(g, h, n_steps)
    a2 = amp(g, h)
    with np.errstate(invalid="ignore", divide="ignore"):  # a broken oracle may flip or lose the mode
        return float(np.log(a1 / a2) / (n_steps * dt) / (nu * k * k))


def force_moments_error() -> float:
    """sum_a Phi_h = M lap mu, sum_a Phi_g = c_s^2 u . grad rho, and at u = 0
    sum_a e Phi_g = c_s^2 mu grad C (barycentric values)."""
    mesh = small_box(n=6, nz=4)
    phys = phys3d()
    o = fo3.Oracle3D(mesh, phys, np.zeros(mesh.n_nodes), with_matrices=False)
    rng = np.random.default_rng(9)
    C = droplet_field_3d(mesh, [(3.0, 3.0, 2.0, 2.0)], phys.xi)
    g, h = o.init_state(C, u=rng.normal(0, 0.02, (mesh.n_nodes, 3)), p=rng.normal(0, 1e-3, mesh.n_nodes))
    f = o.fields(g, h)
    tet = o.geo.tet
    ub = f["u"][tet].mean(1)
    gradrho = fo3.element_gradient(o.geo, f["rho"])
    e1 = abs(f["Phi_h"].sum(1) - o.prm.mobility * f["lapmu"]).max()
    e2 = abs(f["Phi_g"].sum(1) - fo3.CS2 * (ub * gradrho).sum(1)).max()
    g0, h0 = o.init_state(C)
    f0 = o.fields(g0, h0)
    e3 = abs(f0["Phi_g"] @ fo3.E - fo3.CS2 * f0["mu"][tet].mean(1)[:, None] * f0["gradC"]).max()
    return float(max(e1, e2, e3))


def first_step_composition_error_3d(h: float, rho_l: float = 3.0, rho_v: float = 1.0, p0: float = 2e-3) -> float:
    """Composition change over the first step from rest (u = 0, populations
    at equilibrium) with mobility M = 0, as in 2-D.  The continuum equations of
    Sec. II give dC/dt = -div(C u) and, with rho du/dt = -grad p + mu grad C at
    rest, d2C/dt2 = div[(C / rho)(grad p - mu grad C)]; so over one step
    dC = dt^2/2 d/dx[(C / rho)(p' - mu C')] + O(dt^3), which the h-scheme
    carries only through the C/(rho c_s^2)(grad p - mu grad C) term of eq:H.
    Layers C = 0.5 + 0.3 cos(k x), p = p0 sin(k x) along the periodic x axis of
    an unjittered box (3 cells in y, walls at z = 0 and z = 6h with a neutral
    wall); mu from the closed form 2 beta C (C - 1)(2C - 1) - kappa C''
    (kappa = 1.5 sigma xi, beta = 12 sigma / xi).  Returns the max error at the
    nodes two or more layers from the walls, relative to the max exact change."""
    L = 32.0
    nx, ny, nz = int(round(L / h)), 3, 6
    mesh = tet_box_mesh(L, ny * h, nz * h, nx, ny, nz, seed=[5], jitter=0.0)
    phys = make_physics(sigma=0.01, m_rho=rho_l / rho_v, m_nu=1, dt=0.1, mobility=0.0, rho_l=rho_l)
    o = fo3.Oracle3D(mesh, phys, np.zeros(mesh.n_nodes))
    k = 2 * np.pi / L
    x, z = mesh.xyz[:, 0], mesh.xyz[:, 2]
    g, hh = o.init_state(0.5 + 0.3 * np.cos(k * x), p=p0 * np.sin(k * x))
    g1, h1 = o.step(g, hh)
    dC = h1.sum(1) - hh.sum(1)
    kap, bet = 1.5 * phys.sigma * phys.xi, 12.0 * phys.sigma / phys.xi

    def flux(xx):
        C = 0.5 + 0.3 * np.cos(k * xx)
        Cp, Cpp = -0.3 * k * np.sin(k * xx), -0.3 * k * k * np.cos(k * xx)
        mu = 2 * bet * C * (C - 1) * (2 * C - 1) - kap * Cpp
        return (C / (C * rho_l + (1 - C) * rho_v)) * (p0 * k * np.cos(k * xx) - mu * Cp)

    eps = 1e-5
    exact = 0.5 * phys.dt ** 2 * (flux(x + eps) - flux(x - eps)) / (2 * eps)
    inner = (z > 1.5 * h) & (z < (nz - 1.5) * h)
    return float(abs(dC[inner] - exact[inner]).max() / abs(exact[inner]).max())


def diagnostics_error_3d() -> float:
    """Mass sum_i m_i C_i, <T> = 1/2 sum rho |u|^2 / N and max |u| (Sec. III)
    against a hand count on an unjittered 6 x 5 x 4 box of unit cells (x, y
    periodic: 6 x 5 x 5 nodes): C = 0.7 everywhere (rho = 0.7 rho_l + 0.3 rho_v),
    u = (0.01 (i - 2), 0.002 j, 0.003) at node (i, j, k) set through the
    equilibria, zero on the wall layers k = 0, 4 (the wall operator); the
    lumped masses of a closed box sum to its volume 6 x 5 x 4."""
    mesh = tet_box_mesh(6.0, 5.0, 4.0, 6, 5, 4, seed=[1], jitter=0.0)
    phys = make_physics(sigma=0.01, m_rho=10, m_nu=1, dt=0.1, rho_l=2.0)
    o = fo3.Oracle3D(mesh, phys, np.zeros(mesh.n_nodes))
    x, y = mesh.xyz[:, 0], mesh.xyz[:, 1]
    u = np.stack([0.01 * (x - 2.0), 0.002 * y, np.full(mesh.n_nodes, 0.003)], 1)
    g, h = o.init_state(np.full(mesh.n_nodes, 0.7), u=u)
    d = o.diagnostics(g, h)
    rho = 0.7 * 2.0 + 0.3 * 0.2
    total, peak, n = 0.0, 0.0, 0
    for k in range(5):
        for j in range(5):
            for i in range(6):
                n += 1
                if k in (0, 4):
                    continue
                ux, uy, uz = 0.01 * (i - 2.0), 0.002 * j, 0.003
                total += ux * ux + uy * uy + uz * uz
                peak = max(peak, np.sqrt(ux * ux + uy * uy + uz * uz))
    ke = 0.5 * rho * total / n
    errs = [abs(d["mass"] - 0.7 * 120.0) / 84.0, abs(d["mean_ke"] - ke) / ke, abs(d["max_u"] - peak) / peak]
    return float(max(errs))
