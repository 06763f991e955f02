"""Pins of the CPU oracle against what the paper and mathematics fix.

Each function returns an error measure; tests/test_oracle_pins.py bounds it
and tests/test_oracle_mutations.py plants plausible mistakes in the oracle
and checks that the matching pin then fails.  Nothing here retypes an oracle
formula: every expected value is a closed form, an exact identity, a
brute-force evaluation or a property of the exact continuum solution.
"""
from __future__ import annotations

import os

import numpy as np

from oracle import felbm_oracle as fo
from workloads import Mesh, make_physics, split_grid_mesh, uniform_rows

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def four_element_mesh() -> Mesh:
    """Unit square with a centre node, four triangles, walls on all sides."""
    xy = np.array([[0, 0], [1, 0], [1, 1], [0, 1], [0.5, 0.5]], dtype=np.float64)
    tri = np.array([[0, 1, 4], [1, 2, 4], [2, 3, 4], [3, 0, 4]], dtype=np.int32)
    walls = np.array([[0, 1], [1, 2], [2, 3], [3, 0]], dtype=np.int32)
    return Mesh(xy=xy, tri=tri, wall_edges=walls, period_x=0.0, ncols=0, nrows=0,
                wall_side=np.array([0, 3, 1, 2], dtype=np.int8))


def _bary(P, x):
    """Barycentric coordinates of point x in triangle P (3, 2) by a direct solve."""
    A = np.vstack([P.T, np.ones(3)])
    return np.linalg.solve(A, np.array([x[0], x[1], 1.0]))


def bruteforce_matrices(mesh: Mesh):
    """Dense FE matrices by edge-midpoint quadrature (exact for degree <= 2),
    shape functions from a barycentric solve, gradients by central differences."""
    N, NT = mesh.n_nodes, mesh.n_tris
    M11 = np.zeros((N, N)); M10 = np.zeros((N, NT))
    C = np.zeros((2, N, N)); D = np.zeros((2, 2, N, N)); K = np.zeros((2, N, NT))
    for t, vs in enumerate(mesh.tri):
        P = mesh.xy[vs].copy()
        if mesh.period_x > 0:
            P[:, 0] -= mesh.period_x * np.round((P[:, 0] - P[0, 0]) / mesh.period_x)
        area = 0.5 * abs(np.linalg.det(np.vstack([P.T, np.ones(3)])))
        eps = 1e-6
        grads = np.zeros((3, 2))
        c = P.mean(0)
        for r in range(2):
            dx = np.zeros(2); dx[r] = eps
            grads[:, r] = (_bary(P, c + dx) - _bary(P, c - dx)) / (2 * eps)
        for q in ((P[0] + P[1]) / 2, (P[1] + P[2]) / 2, (P[2] + P[0]) / 2):
            lam = _bary(P, q)
            wq = area / 3.0
            for a in range(3):
                M10[vs[a], t] += wq * lam[a]
                for r in range(2):
                    K[r, vs[a], t] += 0.5 * wq * grads[a, r]
                for b in range(3):
                    M11[vs[a], vs[b]] += wq * lam[a] * lam[b]
                    for r in range(2):
                        C[r, vs[a], vs[b]] += wq * lam[a] * grads[b, r]
                        for s in range(2):
                            D[s, r, vs[a], vs[b]] += 0.5 * wq * grads[a, s] * grads[b, r]
    return M11, M10, C, D, K


def fem_bruteforce_error(mesh: Mesh | None = None) -> float:
    mesh = four_element_mesh() if mesh is None else mesh
    mat = fo.Matrices(fo.Geometry(mesh))
    M11, M10, C, D, K = bruteforce_matrices(mesh)
    errs = [abs(mat.M11.toarray() - M11).max(), abs(mat.M10.toarray() - M10).max()]
    for r in range(2):
        errs.append(abs(mat.C[r].toarray() - C[r]).max())
        errs.append(abs(mat.K[r].toarray() - K[r]).max())
        for s in range(2):
            errs.append(abs(mat.D[s][r].toarray() - D[s, r]).max())
    # the per-direction combinations of eq:fem_matrices
    for a in range(9):
        e = fo.E[a]
        errs.append(abs(mat.Ca[a].toarray() - (e[0] * C[0] + e[1] * C[1])).max())
        errs.append(abs(mat.Da[a].toarray() - sum(e[s] * e[r] * D[s, r] for s in range(2) for r in range(2))).max())
        errs.append(abs(mat.Ka[a].toarray() - (e[0] * K[0] + e[1] * K[1])).max())
    return float(max(errs))


def m11_golden_error() -> float:
    ref = np.loadtxt(os.path.join(GOLDEN, "m11_four_element.txt")) / 48.0
    mat = fo.Matrices(fo.Geometry(four_element_mesh()))
    lumped_ref = np.loadtxt(os.path.join(GOLDEN, "lumped_four_element.txt"))
    return float(max(abs(mat.M11.toarray() - ref).max(), abs(mat.lumped - lumped_ref).max()))


def small_mesh(jitter=0.2, seed=11, nx=16, ny=9, diag="random"):
    return split_grid_mesh(float(nx), uniform_rows(float(ny - 1), ny), nx, seed=[seed], jitter=jitter, diag=diag)


def identities_error() -> dict:
    mesh = small_mesh()
    geo = fo.Geometry(mesh)
    mat = fo.Matrices(geo)
    N = geo.N
    one = np.ones(N)
    out = {}
    out["M11_one_is_lumped"] = abs(mat.M11 @ one - np.asarray(mat.M11.sum(1)).ravel()).max()
    out["lumped_sum_is_area"] = abs(mat.lumped.sum() - 16.0 * 8.0)
    out["D_one"] = max(abs(mat.Da[a] @ one).max() for a in range(9))
    out["K_colsum"] = max(abs(one @ mat.Ka[a]).max() for a in range(9))
    y = mesh.xy[:, 1]
    lin = 0.3 + 0.7 * y        # linear and x-periodic
    out["C_linear"] = max(abs(mat.Ca[a] @ lin - fo.E[a, 1] * 0.7 * mat.lumped).max() for a in range(9))
    ev = np.linalg.eigvalsh(np.diag(1 / np.sqrt(mat.lumped)) @ mat.M11.toarray() @ np.diag(1 / np.sqrt(mat.lumped)))
    out["wathen_low"] = max(0.0, 0.25 - ev.min())
    out["wathen_high"] = max(0.0, ev.max() - 1.0)
    return {k: float(v) for k, v in out.items()}


def lattice_identities_error() -> float:
    rng = np.random.default_rng(5)
    n = 50
    C = rng.uniform(0, 1, n); p = rng.normal(0, 1e-3, n)
    u = rng.normal(0, 0.05, (n, 2))
    rho = 0.1 + 0.9 * C
    geq, heq = fo.equilibria(C, p, rho, u)
    G = fo.gamma(u)
    e = fo.E
    errs = [
        abs(heq.sum(1) - C).max(),
        abs(geq.sum(1) - p).max(),
        abs(np.stack([geq @ e[:, 0], geq @ e[:, 1]], 1) - (rho * fo.CS2)[:, None] * u).max(),
        abs(G.sum(1) - 1).max(),
        abs(np.stack([G @ e[:, 0], G @ e[:, 1]], 1) - u).max(),      # sum e Gamma = u
        abs(fo.W.sum() - 1),
        abs(np.einsum("a,ai,aj->ij", fo.W, e, e) - fo.CS2 * np.eye(2)).max(),  # isotropy
        abs(e[fo.OPPOSITE] + e).max(),
        abs(fo.W[fo.OPPOSITE] - fo.W).max(),
    ]
    return float(max(errs))


def collision_conservation_error() -> float:
    rng = np.random.default_rng(6)
    n = 40
    phys = make_physics(sigma=0.01, m_rho=10, m_nu=3, dt=0.1)
    prm = fo.Params.from_physics(phys.sigma, phys.xi, phys.mobility, phys.rho_l, phys.rho_v, phys.nu_l, phys.nu_v, phys.dt)
    C = rng.uniform(0, 1, n); p = rng.normal(0, 1e-3, n); u = rng.normal(0, 0.03, (n, 2))
    geq, heq = fo.equilibria(C, p, fo.density(C, prm), u)
    g = geq + rng.normal(0, 1e-3, geq.shape); h = heq + rng.normal(0, 1e-3, heq.shape)
    Cm, pm, rho, um = fo.moments(g, h, prm)
    geq, heq = fo.equilibria(Cm, pm, rho, um)
    tau = fo.relaxation_time(Cm, prm)
    gh, hh = fo.collide(g, geq, tau), fo.collide(h, heq, tau)
    errs = [abs(hh.sum(1) - h.sum(1)).max(), abs(gh.sum(1) - g.sum(1)).max(),
            abs(gh @ fo.E - g @ fo.E).max(),
            abs(fo.collide(geq, geq, tau) - geq).max()]
    return float(max(errs))


def static_balance_drift(seed=3) -> float:
    """Sec. II.C static interface: u = 0, p = 0, kappa = beta = 0 (no surface
    tension), no mobility term: with h = w C and g = 0 the mixed (P1 field /
    P0 force) discretisation leaves every population unchanged."""
    mesh = small_mesh(seed=seed)
    phys = make_physics(sigma=0.0, m_rho=10, m_nu=1, dt=0.1, mobility=0.0)
    o = fo.Oracle(mesh, phys, np.zeros(mesh.n_nodes))
    rng = np.random.default_rng(seed)
    C = rng.uniform(0.0, 1.0, mesh.n_nodes)
    g, h = o.init_state(C)
    g1, h1 = o.step(g, h)
    return float(max(abs(h1 - h).max(), abs(g1 - g).max()) / abs(h).max())


def advection_error(n_steps=100, with_mesh=None) -> float:
    """Pure streaming (eqn::stream with F = 0, no collision) of cos(2 pi x / 16)
    along e_1 = (1, 0) on a uniform periodic mesh: the exact solution is the
    profile shifted by n dt; the second-order Taylor-Galerkin scheme tracks it."""
    mesh = with_mesh or split_grid_mesh(64.0, uniform_rows(16.0, 17), 64, seed=[7], jitter=0.0, diag="up")
    geo = fo.Geometry(mesh); mat = fo.Matrices(geo)
    x = mesh.xy[:, 0]; k = 2 * np.pi / 16; dt = 0.1
    psi = np.zeros((mesh.n_nodes, 9)); psi[:, 1] = np.cos(k * x)
    Phi = np.zeros((mesh.n_tris, 9))
    for _ in range(n_steps):
        b = fo.rhs(mat, dt, psi, Phi)
        d, _ = fo.pcg(mat.M11, mat.lumped, b[:, 1])
        psi[:, 1] = psi[:, 1] + d
    return float(abs(psi[:, 1] - np.cos(k * (x - n_steps * dt))).max())


def force_source_error() -> float:
    """Streaming of a pure source (psi_hat = 0, F linear in y): eqn::stream gives
    psi^{n+1} = dt F - dt^2/2 e.grad F.  On a uniform mesh the P0 projection of
    a linear field and the consistent mass matrix reproduce this exactly at nodes
    far from the walls, for e along +y and -y."""
    mesh = split_grid_mesh(16.0, uniform_rows(40.0, 41), 16, seed=[7], jitter=0.0, diag="up")
    geo = fo.Geometry(mesh); mat = fo.Matrices(geo)
    dt = 0.1; slope = 0.37
    Fc = 1.0 + slope * geo.centroid[:, 1]
    Phi = np.repeat(Fc[:, None], 9, axis=1)
    b = fo.rhs(mat, dt, np.zeros((mesh.n_nodes, 9)), Phi)
    y = mesh.xy[:, 1]
    mid = (y > 15) & (y < 25)
    err = 0.0
    for a in (0, 2, 4):
        d, _ = fo.pcg(mat.M11, mat.lumped, b[:, a])
        exact = dt * (1.0 + slope * y) - 0.5 * dt * dt * fo.E[a, 1] * slope
        err = max(err, abs(d - exact)[mid].max())
    return float(err)


def laplacian_quadratic_error() -> float:
    """Nodal patch Laplacian (eqn:lapl_int_mp) of C = a + b y + c y^2 on a
    uniform mesh equals 2c at nodes two or more rows from the walls."""
    mesh = split_grid_mesh(12.0, uniform_rows(10.0, 11), 12, seed=[7], jitter=0.0, diag="up")
    phys = make_physics(sigma=0.01, m_rho=10, m_nu=1, dt=0.1)
    o = fo.Oracle(mesh, phys, np.zeros(mesh.n_nodes))
    y = mesh.xy[:, 1]
    C = 0.2 + 0.05 * y + 0.013 * y * y
    lap = fo.laplacian_C(o.geo, C, fo.element_gradient(o.geo, C), o.bc)
    inner = (y >= 2) & (y <= 8)
    return float(abs(lap[inner] - 2 * 0.013).max())


def laplacian_cosine_ratio() -> float:
    """Second-order convergence of the patch Laplacian of cos(2 pi x / 16) on
    uniform meshes of spacing 1 and 1/2: error ratio (expected ~4)."""
    errs = []
    for n in (1, 2):
        mesh = split_grid_mesh(16.0, uniform_rows(8.0, 8 * n + 1), 16 * n, seed=[7], jitter=0.0, diag="up")
        phys = make_physics(sigma=0.01, m_rho=10, m_nu=1, dt=0.1)
        o = fo.Oracle(mesh, phys, np.zeros(mesh.n_nodes))
        k = 2 * np.pi / 16
        C = np.cos(k * mesh.xy[:, 0])
        lap = fo.laplacian_C(o.geo, C, fo.element_gradient(o.geo, C), o.bc)
        y = mesh.xy[:, 1]
        inner = (y >= 2) & (y <= 6)
        errs.append(abs(lap[inner] + k * k * C[inner]).max())
    return float(errs[0] / errs[1])


def wall_linear_laplacian_error() -> float:
    """At the wall, C = c0 + s y with the wetting potential chosen so that eq.
    bc2 holds (n into the fluid): the patch integral of a linear field with the
    wetting flux on the wall edges vanishes, so lap C = 0 at wall nodes."""
    mesh = split_grid_mesh(12.0, uniform_rows(6.0, 7), 12, seed=[7], jitter=0.2)
    phys = make_physics(sigma=0.01, m_rho=10, m_nu=1, dt=0.1)
    c0, s = 0.3, 0.02
    prm = fo.Params.from_physics(phys.sigma, phys.xi, phys.mobility, phys.rho_l, phys.rho_v, phys.nu_l, phys.nu_v, phys.dt)
    # bottom wall: n_in = +y, n.grad C = s = (phi_c/kappa)(C - C^2) at C = c0
    om = np.zeros(mesh.n_nodes)
    bottom = mesh.wall_nodes(0)
    phi_needed = s * prm.kappa / (c0 - c0 * c0)
    om[bottom] = phi_needed / np.sqrt(2 * prm.kappa * prm.beta)
    # top wall: n_in = -y, n.grad C = -s at C(top) = c0 + 6 s
    ct = c0 + 6 * s
    top = mesh.wall_nodes(1)
    om[top] = (-s * prm.kappa / (ct - ct * ct)) / np.sqrt(2 * prm.kappa * prm.beta)
    o = fo.Oracle(mesh, phys, om)
    C = c0 + s * mesh.xy[:, 1]
    lap = fo.laplacian_C(o.geo, C, fo.element_gradient(o.geo, C), o.bc)
    return float(abs(lap).max())


def wall_flux_wedge_error(theta_deg=60.0) -> float:
    """The planar tanh interface meeting the wall at the Young angle satisfies
    eq. bc2 pointwise.  The oracle's wetting flux through each wall edge must
    equal the exact outward flux of that profile (fine Gauss-Legendre
    quadrature of the analytic gradient) up to O(h^2) interpolation error.
    Returns the max edge error relative to the max edge flux."""
    mesh = split_grid_mesh(64.0, uniform_rows(16.0, 17), 128, seed=[9], jitter=0.0)
    phys = make_physics(sigma=0.01, m_rho=10, m_nu=1, dt=0.1)
    prm = fo.Params.from_physics(phys.sigma, phys.xi, phys.mobility, phys.rho_l, phys.rho_v, phys.nu_l, phys.nu_v, phys.dt)
    th = np.deg2rad(theta_deg); x0 = 32.0; xi = phys.xi
    n_in_liquid = np.array([-np.sin(th), -np.cos(th)])

    def C_of(x, y):
        return 0.5 + 0.5 * np.tanh(2 * ((x - x0) * n_in_liquid[0] + y * n_in_liquid[1]) / xi)

    def gradC(x, y):
        s = (x - x0) * n_in_liquid[0] + y * n_in_liquid[1]
        return (1.0 / xi) / np.cosh(2 * s / xi) ** 2 * n_in_liquid[:, None]

    C = C_of(mesh.xy[:, 0], mesh.xy[:, 1])
    om = -np.cos(th)
    phi = om * np.sqrt(2 * prm.kappa * prm.beta)
    edges = mesh.wall_edges[mesh.wall_side == 0]
    gx, gw = np.polynomial.legendre.leggauss(20)
    errs, mags = [], []
    for a, b in edges:
        xa, xb = mesh.xy[a, 0], mesh.xy[b, 0]
        if abs(xa - x0) > 16 or abs(xb - x0) > 16:      # the planar profile is not periodic
            continue
        got = fo.wall_flux(C[a], C[b], phi / prm.kappa, phi / prm.kappa, abs(xb - xa))
        xs = 0.5 * (xa + xb) + 0.5 * (xb - xa) * gx
        exact = 0.5 * (xb - xa) * np.sum(gw * (-gradC(xs, 0 * xs)[1]))    # n_out = -y
        errs.append(abs(got - exact)); mags.append(abs(exact))
    return float(max(errs) / max(mags))


def simpson_wall_flux_error() -> float:
    """Wall flux with C and phi_c linear along the edge against brute-force
    quadrature of -(1/kappa) phi_c (C - C^2)."""
    prm = fo.Params.from_physics(0.01, 4.0, 0.02, 1.0, 0.1, 1 / 30, 1 / 30, 0.1)
    rng = np.random.default_rng(2)
    err = 0.0
    gx, gw = np.polynomial.legendre.leggauss(10)
    for _ in range(20):
        Ca, Cb, pa, pb, L = rng.uniform(0, 1), rng.uniform(0, 1), rng.normal(), rng.normal(), rng.uniform(0.2, 2)
        t = 0.5 + 0.5 * gx
        Cs, ps = Ca + (Cb - Ca) * t, pa + (pb - pa) * t
        exact = -0.5 * L * np.sum(gw * ps * (Cs - Cs * Cs)) / prm.kappa
        err = max(err, abs(fo.wall_flux(Ca, Cb, pa / prm.kappa, pb / prm.kappa, L) - exact))
    return float(err)


def flat_interface_mu(h: float) -> float:
    """Relative residual chemical potential of the exact planar tanh profile
    (mu = 0 in the continuum, Sec. II) on a uniform mesh of spacing h, measured
    away from the walls, divided by the bulk-term amplitude 2 beta max|C(C-1)(2C-1)|."""
    n = int(round(32 / h))
    mesh = split_grid_mesh(16.0, uniform_rows(32.0, n + 1), int(round(16 / h)), seed=[4], jitter=0.0, diag="up")
    phys = make_physics(sigma=0.01, m_rho=10, m_nu=1, dt=0.1)
    o = fo.Oracle(mesh, phys, np.zeros(mesh.n_nodes))
    y = mesh.xy[:, 1]
    C = 0.5 + 0.5 * np.tanh(2 * (y - 16.0) / phys.xi)
    g, hh = o.init_state(C)
    mu = o.fields(g, hh)["mu"]
    inner = (y > 4) & (y < 28)
    scale = 2 * o.prm.beta * (np.sqrt(3) / 18)      # max |C(C-1)(2C-1)| on [0, 1] = sqrt(3)/18
    return float(abs(mu[inner]).max() / scale)


def surface_tension_integral() -> float:
    """int kappa |grad C|^2 dA per unit interface length for the planar profile
    (equals sigma by equipartition); returns the relative error."""
    mesh = split_grid_mesh(16.0, uniform_rows(32.0, 129), 64, seed=[4], jitter=0.0, diag="up")
    phys = make_physics(sigma=0.01, m_rho=10, m_nu=1, dt=0.1)
    o = fo.Oracle(mesh, phys, np.zeros(mesh.n_nodes))
    C = 0.5 + 0.5 * np.tanh(2 * (mesh.xy[:, 1] - 16.0) / phys.xi)
    G = fo.element_gradient(o.geo, C)
    s = o.prm.kappa * np.sum(o.geo.area * (G * G).sum(1)) / 16.0
    return float(abs(s - phys.sigma) / phys.sigma)


def laplace_jump(R: float, h: float) -> float:
    """2-D Laplace law for the tanh droplet of radius R (Sec. II): the pressure
    jump balancing -C grad mu, p_in - p_out = int C dmu/dr dr, equals sigma / R
    up to O((xi/R)^2).  Evaluated from the oracle's element gradients of mu as
    (1/2 pi) sum_T A_T C_T (grad mu_T . r_hat) / r_T; returns dp R / sigma."""
    L = 4 * R
    n = int(round(L / h))
    mesh = split_grid_mesh(float(L), uniform_rows(float(L), n + 1), n, seed=[8], jitter=0.0, diag="up")
    phys = make_physics(sigma=0.01, m_rho=10, m_nu=1, dt=0.1)
    o = fo.Oracle(mesh, phys, np.zeros(mesh.n_nodes))
    xy = mesh.xy
    d = np.sqrt((xy[:, 0] - L / 2) ** 2 + (xy[:, 1] - L / 2) ** 2)
    C = 0.5 + 0.5 * np.tanh(2 * (R - d) / phys.xi)
    g, hh = o.init_state(C)
    f = o.fields(g, hh)
    geo = o.geo
    rv = geo.centroid - L / 2
    rr = np.sqrt((rv ** 2).sum(1))
    Cb = C[geo.tri].mean(1)
    dp = np.sum(geo.area * Cb * (f["gradmu"] * rv).sum(1) / rr ** 2) / (2 * np.pi)
    return float(dp * R / phys.sigma)


def mass_drift(n_steps=60, theta=60.0) -> float:
    """Relative change of int C = sum_i m_i C_i over n steps of a droplet on a
    wetting wall (conserved exactly by the scheme)."""
    mesh = split_grid_mesh(32.0, uniform_rows(16.0, 17), 32, seed=[12])
    phys = make_physics(sigma=0.01, m_rho=10, m_nu=2, dt=0.1)
    from workloads import droplet_field, wetting_from_angles
    om = wetting_from_angles(mesh, theta)
    o = fo.Oracle(mesh, phys, om)
    g, h = o.init_state(droplet_field(mesh, [(16.0, 0.0, 7.0)], phys.xi))
    m0 = o.mass(h)
    g, h = o.run(g, h, n_steps)
    return float(abs(o.mass(h) - m0) / m0)


def wall_velocity_after_step() -> float:
    mesh = split_grid_mesh(32.0, uniform_rows(16.0, 17), 32, seed=[12])
    phys = make_physics(sigma=0.01, m_rho=10, m_nu=2, dt=0.1)
    from workloads import droplet_field, wetting_from_angles
    o = fo.Oracle(mesh, phys, wetting_from_angles(mesh, 60.0))
    g, h = o.init_state(droplet_field(mesh, [(16.0, 0.0, 7.0)], phys.xi))
    g, h = o.run(g, h, 5)
    C, p, rho, u = fo.moments(g, h, o.prm)
    return float(abs(u[o.geo.is_wall_node]).max())


def channel_mesh_pins(n_steps=60):
    """A mesh with two holes (blocks leaving a channel, 40 x 16 box, blocks
    16 x 6): the lumped masses sum to the fluid area 40*16 - 2*16*6 = 448
    (Sec. II.C mass matrix), sum_T A_T grad N_i = 0 at every node off the
    walls, and over n steps with wetting channel walls and a liquid slab in
    the channel the composition integral is conserved and every wall node,
    on the block faces and re-entrant corners too, has zero velocity."""
    from workloads import channel_mesh
    mesh = channel_mesh(40.0, 16.0, 1.0, 12.0, 28.0, 6.0, 10.0, seed=[7])
    phys = make_physics(sigma=0.01, m_rho=10, m_nu=2, dt=0.1)
    om = np.zeros(mesh.n_nodes)
    om[mesh.wall_nodes(4)] = -0.5
    o = fo.Oracle(mesh, phys, om)
    geo = o.geo
    area_err = abs(o.mat.lumped.sum() - 448.0) / 448.0
    s = np.zeros((geo.N, 2))
    for l in range(3):
        np.add.at(s, mesh.tri[:, l], geo.area[:, None] * geo.gradN[:, l, :])
    closure = float(abs(s[~geo.is_wall_node]).max())
    x = mesh.xy[:, 0]
    C0 = 0.5 + 0.5 * np.tanh(2.0 * np.minimum(x - 4.0, 16.0 - x) / phys.xi)
    g, h = o.init_state(C0)
    m0 = o.mass(h)
    g, h = o.run(g, h, n_steps)
    C, p, rho, u = fo.moments(g, h, o.prm)
    return float(area_err), closure, float(abs(o.mass(h) - m0) / m0), float(abs(u[geo.is_wall_node]).max())


def pcg_dense_error() -> float:
    mesh = small_mesh()
    mat = fo.Matrices(fo.Geometry(mesh))
    b = np.random.default_rng(1).normal(size=mesh.n_nodes)
    x, _ = fo.pcg(mat.M11, mat.lumped, b)
    xd = np.linalg.solve(mat.M11.toarray(), b)
    return float(abs(x - xd).max() / abs(xd).max())


def complex_step_vs_fd(seed=2) -> float:
    """Derivative, with respect to the wetting potential of one wall node near
    the contact line, of a localised composition integral after 3 steps:
    complex-step tangent of the oracle versus a central difference (h = 1e-3)."""
    mesh = split_grid_mesh(24.0, uniform_rows(12.0, 13), 24, seed=[seed])
    phys = make_physics(sigma=0.01, m_rho=10, m_nu=1, dt=0.1)
    from workloads import droplet_field, wetting_from_angles
    om = wetting_from_angles(mesh, 70.0)
    C0 = droplet_field(mesh, [(12.0, 0.0, 6.0)], phys.xi)
    bottom = mesh.wall_nodes(0)
    k = bottom[np.argmin(abs(mesh.xy[bottom, 0] - 18.0))]
    wgt = np.exp(-((mesh.xy[:, 0] - 18.0) ** 2 + mesh.xy[:, 1] ** 2) / 8.0)

    def loss(omv):
        o = fo.Oracle(mesh, phys, omv)
        g, h = o.init_state(C0.astype(omv.dtype))
        g, h = o.run(g, h, 3)
        return np.sum(o.mat.lumped * wgt * h.sum(1))

    hc = 1e-30
    omc = om.astype(complex); omc[k] += 1j * hc
    d_cs = loss(omc).imag / hc
    hf = 1e-3
    op, omm = om.copy(), om.copy(); op[k] += hf; omm[k] -= hf
    d_fd = (loss(op) - loss(omm)) / (2 * hf)
    return float(abs(d_cs - d_fd) / abs(d_cs))


def force_moments_error() -> float:
    """Moments of the element forces that follow from sum Gamma = 1 and
    sum (e - u) Gamma = 0 (D2Q9): sum_a Phi_h = M lap mu, sum_a Phi_g =
    c_s^2 u.grad rho, and at u = 0 the first moment sum_a e Phi_g = c_s^2 mu grad C."""
    mesh = small_mesh()
    phys = make_physics(sigma=0.01, m_rho=10, m_nu=1, dt=0.1)
    from workloads import droplet_field
    o = fo.Oracle(mesh, phys, np.zeros(mesh.n_nodes))
    rng = np.random.default_rng(9)
    C = droplet_field(mesh, [(8.0, 2.0, 4.0)], phys.xi)
    u = rng.normal(0, 0.02, (mesh.n_nodes, 2))
    g, h = o.init_state(C, u=u, p=rng.normal(0, 1e-3, mesh.n_nodes))
    f = o.fields(g, h)
    ub = f["u"][o.geo.tri].mean(1)
    e1 = abs(f["Phi_h"].sum(1) - o.prm.mobility * f["lapmu"]).max()
    e2 = abs(f["Phi_g"].sum(1) - fo.CS2 * (ub * f["gradrho"]).sum(1)).max()
    g0, h0 = o.init_state(C)
    f0 = o.fields(g0, h0)
    mub = f0["mu"][o.geo.tri].mean(1)
    first = np.stack([f0["Phi_g"] @ fo.E[:, 0], f0["Phi_g"] @ fo.E[:, 1]], 1)
    e3 = abs(first - fo.CS2 * mub[:, None] * f0["gradC"]).max()
    return float(max(e1, e2, e3))


def relaxation_time_cases() -> float:
    """1/tau = C/tau_l + (1 - C)/tau_v: the pure phases give tau_l and tau_v and
    C = 1/2 gives the harmonic mean 2 tau_l tau_v / (tau_l + tau_v)."""
    prm = fo.Params.from_physics(0.01, 4.0, 0.02, 1.0, 0.1, 0.1 / 3, 0.4 / 3, 0.1)
    t = fo.relaxation_time(np.array([1.0, 0.0, 0.5]), prm)
    ref = np.array([1.0, 4.0, 2 * 1.0 * 4.0 / 5.0])
    return float(abs(t - ref).max())


def shear_wave_viscosity_ratio(tau=2.0, n_steps=600, force_scheme="mixed") -> float:
    """Lowest channel shear mode u_x = U sin(pi y / H) between no-slip walls in
    single-phase liquid (C = 1): it decays at rate nu (pi/H)^2 with
    nu = c_s^2 tau dt (Sec. II.A).  Returns measured rate / nu (pi/H)^2."""
    H = 16
    mesh = split_grid_mesh(16.0, uniform_rows(float(H), H + 1), 16, seed=[13])
    dt = 0.1
    phys = make_physics(sigma=0.01, m_rho=10, m_nu=1, dt=dt)
    phys.nu_l = fo.CS2 * tau * dt
    o = fo.Oracle(mesh, phys, np.zeros(mesh.n_nodes), force_scheme=force_scheme)
    k = np.pi / H
    y = mesh.xy[:, 1]
    u = np.zeros((mesh.n_nodes, 2)); u[:, 0] = 1e-3 * np.sin(k * y)
    g, h = o.init_state(np.ones(mesh.n_nodes), u=u)
    s = np.sin(k * y)

    def amp(g, h):
        return np.sum(fo.moments(g, h, o.prm)[3][:, 0] * s) / np.sum(s * s)
    g, h = o.run(g, h, 100)
    a1 = amp(g, h)
    g, h = o.run(g, h, n_steps)
    a2 = amp(g, h)
    rate = np.log(a1 / a2) / (n_steps * dt)
    return float(rate / (phys.nu_l * k * k))


# ---------------------------------------------------------------------------
# Nodal-force comparison scheme (readings N1-N4 of the oracle)
# ---------------------------------------------------------------------------
def nodal_force_matrix_error() -> float:
    """K1_r = 1/2 int d_r phi_i phi_j against midpoint quadrature with the
    shape functions from a barycentric solve (the brute force of
    bruteforce_matrices), on the four-element mesh and a jittered periodic mesh."""
    errs = []
    for mesh in (four_element_mesh(), small_mesh(nx=6, ny=4)):
        N = mesh.n_nodes
        K1 = np.zeros((2, N, N))
        for vs in mesh.tri:
            P = mesh.xy[vs].copy()
            if mesh.period_x > 0:
                P[:, 0] -= mesh.period_x * np.round((P[:, 0] - P[0, 0]) / mesh.period_x)
            area = 0.5 * abs(np.linalg.det(np.vstack([P.T, np.ones(3)])))
            eps = 1e-6
            grads = np.zeros((3, 2))
            c = P.mean(0)
            for r in range(2):
                dx = np.zeros(2); dx[r] = eps
                grads[:, r] = (_bary(P, c + dx) - _bary(P, c - dx)) / (2 * eps)
            for q in ((P[0] + P[1]) / 2, (P[1] + P[2]) / 2, (P[2] + P[0]) / 2):
                lam = _bary(P, q)
                for a in range(3):
                    for b in range(3):
                        for r in range(2):
                            K1[r, vs[a], vs[b]] += 0.5 * (area / 3.0) * grads[a, r] * lam[b]
        mat = fo.Matrices(fo.Geometry(mesh))
        K1a = mat.nodal_force_matrices()
        errs += [abs(mat.K1[r].toarray() - K1[r]).max() for r in range(2)]
        errs += [abs(K1a[a].toarray() - (fo.E[a, 0] * K1[0] + fo.E[a, 1] * K1[1])).max() for a in range(9)]
    return float(max(errs))


def nodal_average_error() -> float:
    """The area-weighted patch mean of the element centroids' coordinates is
    the centroid of the vertex patch, int_patch x / |patch|, integrated here by
    midpoint quadrature triangle by triangle (exact for linear integrands)."""
    mesh = small_mesh()
    geo = fo.Geometry(mesh)
    got = fo.nodal_average(geo, geo.centroid)
    num = np.zeros((geo.N, 2)); den = np.zeros(geo.N)
    for t, vs in enumerate(mesh.tri):
        P = geo.p[t]
        area = 0.5 * abs(np.linalg.det(np.vstack([P.T, np.ones(3)])))
        mids = ((P[0] + P[1]) / 2, (P[1] + P[2]) / 2, (P[2] + P[0]) / 2)
        integral = sum(m for m in mids) * area / 3.0
        for v in vs:
            num[v] += integral; den[v] += area
    # compare in the frame of each node (the unwrapped triangle coordinates of
    # a periodic patch can differ by one period from node to node)
    diff = got - num / den[:, None]
    diff[:, 0] -= mesh.period_x * np.round(diff[:, 0] / mesh.period_x)
    return float(abs(diff).max())


def nodal_static_drift(seed=3) -> float:
    """The static interface of Sec. II.C with nodal (P1) forces: the paper's
    argument is that only the piecewise-constant force balances the streaming
    of a static profile, so the nodal scheme moves the populations.  Returns
    the relative one-step change (compare static_balance_drift)."""
    mesh = small_mesh(seed=seed)
    phys = make_physics(sigma=0.0, m_rho=10, m_nu=1, dt=0.1, mobility=0.0)
    o = fo.Oracle(mesh, phys, np.zeros(mesh.n_nodes), force_scheme="nodal")
    rng = np.random.default_rng(seed)
    C = rng.uniform(0.0, 1.0, mesh.n_nodes)
    g, h = o.init_state(C)
    g1, h1 = o.step(g, h)
    return float(max(abs(h1 - h).max(), abs(g1 - g).max()) / abs(h).max())


def nodal_force_moments_error() -> float:
    """Moments of the nodal forces from sum Gamma = 1, sum (e - u) Gamma = 0:
    sum_a F_h = M lap mu_n, sum_a F_g = c_s^2 u . grad rho_n, and at u = 0
    sum_a e F_g = c_s^2 mu grad C_n (nodal values, reading N4)."""
    mesh = small_mesh()
    phys = make_physics(sigma=0.01, m_rho=10, m_nu=1, dt=0.1)
    from workloads import droplet_field
    o = fo.Oracle(mesh, phys, np.zeros(mesh.n_nodes), force_scheme="nodal")
    rng = np.random.default_rng(9)
    C = droplet_field(mesh, [(8.0, 2.0, 4.0)], phys.xi)
    u = rng.normal(0, 0.02, (mesh.n_nodes, 2))
    g, h = o.init_state(C, u=u, p=rng.normal(0, 1e-3, mesh.n_nodes))
    f = o.fields(g, h)
    e1 = abs(f["F_h"].sum(1) - o.prm.mobility * f["lapmu_n"]).max()
    e2 = abs(f["F_g"].sum(1) - fo.CS2 * (f["u"] * f["gradrho_n"]).sum(1)).max()
    g0, h0 = o.init_state(C)
    f0 = o.fields(g0, h0)
    first = np.stack([f0["F_g"] @ fo.E[:, 0], f0["F_g"] @ fo.E[:, 1]], 1)
    e3 = abs(first - fo.CS2 * f0["mu"][:, None] * f0["gradC_n"]).max()
    return float(max(e1, e2, e3))


def nodal_mass_drift(steps=20) -> float:
    """Total composition with nodal forces and a wetting wall: the P1 force
    enters through int phi_i F and its weighted sum over nodes telescopes like
    the P0 one, so mass is conserved to the solver tolerance."""
    mesh = small_mesh()
    phys = make_physics(sigma=0.01, m_rho=10, m_nu=1, dt=0.1)
    from workloads import droplet_field, wetting_from_angles
    o = fo.Oracle(mesh, phys, wetting_from_angles(mesh, 60.0, 110.0), force_scheme="nodal")
    g, h = o.init_state(droplet_field(mesh, [(8.0, 0.0, 4.0)], phys.xi))
    m0 = o.mass(h)
    g, h = o.run(g, h, steps)
    return float(abs(o.mass(h) - m0) / m0)


# ---------------------------------------------------------------------------
# Second moments of the equilibria, the composition flux of eq:H, the element
# Laplacian of mu, the contact-angle measurement and the band energy
# ---------------------------------------------------------------------------
def second_moment_error() -> float:
    """Second moments that the D2Q9 equilibria must reproduce (eqn::g_eq,
    eqn::f_eq) for the Chapman-Enskog recovery of the momentum flux:
    sum_a e_i e_j Gamma_a = c_s^2 delta_ij + u_i u_j and
    sum_a e_i e_j g_eq_a = c_s^2 (p delta_ij + rho u_i u_j)."""
    rng = np.random.default_rng(15)
    n = 60
    C = rng.uniform(0, 1, n); p = rng.normal(0, 1e-3, n)
    u = rng.normal(0, 0.08, (n, 2))
    rho = 0.1 + 0.9 * C
    geq, heq = fo.equilibria(C, p, rho, u)
    G = fo.gamma(u)
    e = fo.E
    eye = np.eye(2)[None]
    uu = u[:, :, None] * u[:, None, :]
    m2G = np.einsum("na,ai,aj->nij", G, e, e)
    m2g = np.einsum("na,ai,aj->nij", geq, e, e)
    m2h = np.einsum("na,ai,aj->nij", heq, e, e)
    errs = [abs(m2G - (fo.CS2 * eye + uu)).max(),
            abs(m2g - fo.CS2 * (p[:, None, None] * eye + rho[:, None, None] * uu)).max(),
            abs(m2h - C[:, None, None] * (fo.CS2 * eye + uu)).max()]
    return float(max(errs))


def first_step_composition_error(h: float, rho_l: float = 3.0, rho_v: float = 1.0, p0: float = 2e-3,
                                 force_scheme: str = "mixed") -> float:
    """Composition change over the first step from rest (u = 0, populations at
    equilibrium) with mobility M = 0.  The continuum equations of Sec. II give
    dC/dt = -div(C u) and, with rho du/dt = -grad p + mu grad C at rest,
    d2C/dt2 = div[(C / rho)(grad p - mu grad C)]; so over one step
    dC = dt^2/2 d/dy[(C / rho)(p' - mu C')] + O(dt^3).  In the h-scheme this
    comes entirely from the C/(rho c_s^2)(grad p - mu grad C) term of eq:H (the
    rest of the second moment cancels against grad C).  Layered fields
    C = 0.5 + 0.3 cos(k y), p = p0 sin(k y) on a uniform mesh; the exact side
    uses the closed-form mu = 2 beta C (C-1)(2C-1) - kappa C''.  Returns the
    max error away from the walls relative to the max of the exact change."""
    L = 32.0
    n = int(round(L / h))
    mesh = split_grid_mesh(8.0, uniform_rows(L, n + 1), int(round(8 / h)), seed=[5], jitter=0.0, diag="up")
    phys = make_physics(sigma=0.01, m_rho=rho_l / rho_v, m_nu=1, dt=0.1, mobility=0.0, rho_l=rho_l)
    o = fo.Oracle(mesh, phys, np.zeros(mesh.n_nodes), force_scheme=force_scheme)
    k = 2 * np.pi / L
    y = mesh.xy[:, 1]
    g, hh = o.init_state(0.5 + 0.3 * np.cos(k * y), p=p0 * np.sin(k * y))
    g1, h1 = o.step(g, hh)
    dC = h1.sum(1) - hh.sum(1)
    kap, bet = 1.5 * phys.sigma * phys.xi, 12.0 * phys.sigma / phys.xi

    def flux(yy):
        C = 0.5 + 0.3 * np.cos(k * yy)
        Cp, Cpp = -0.3 * k * np.sin(k * yy), -0.3 * k * k * np.cos(k * yy)
        mu = 2 * bet * C * (C - 1) * (2 * C - 1) - kap * Cpp
        return (C / (C * rho_l + (1 - C) * rho_v)) * (p0 * k * np.cos(k * yy) - mu * Cp)

    eps = 1e-5
    exact = 0.5 * phys.dt ** 2 * (flux(y + eps) - flux(y - eps)) / (2 * eps)
    inner = (y > 4) & (y < L - 4)
    return float(abs(dC[inner] - exact[inner]).max() / abs(exact[inner]).max())


def element_laplacian_quadratic_error() -> float:
    """Element Laplacian of mu (Sec. II.D) of the quadratics x^2, y^2, x y and
    x^2 + y^2 on a uniform split-quad mesh with walls on all sides: every
    element's P1 gradient there is the exact gradient at the midpoint of its
    row (column) strip, and the averaged edge gradients integrate to the exact
    Laplacian (2, 2, 0, 4 times the coefficient) at every element two or more
    cells from the walls.  This fixes the operator's interior scale
    (fig:element_nabla_mu).  Returns the max error over the four fields,
    relative to the coefficient."""
    mesh = split_grid_mesh(12.0, uniform_rows(10.0, 11), 12, seed=[7], jitter=0.0, diag="up", periodic=False)
    geo = fo.Geometry(mesh)
    x, y = mesh.xy[:, 0], mesh.xy[:, 1]
    c = 0.021
    cx, cy = geo.centroid[:, 0], geo.centroid[:, 1]
    inner = (cx > 2) & (cx < 10) & (cy > 2) & (cy < 8)
    err = 0.0
    for mu, ref in ((0.3 - 0.04 * y + c * x * x, 2 * c), (0.3 + 0.05 * x + c * y * y, 2 * c),
                    (0.1 + c * x * y, 0.0), (c * (x * x + y * y), 4 * c)):
        lap = fo.laplacian_mu(geo, fo.element_gradient(geo, mu))
        err = max(err, abs(lap[inner] - ref).max() / c)
    return float(err)


def cap_field(mesh: Mesh, theta_deg: float, r: float, x0: float, xi: float) -> np.ndarray:
    """Composition of a circular cap meeting the bottom wall y = 0 at theta:
    the tanh profile about a circle of radius r centred at (x0, -r cos theta)."""
    th = np.deg2rad(theta_deg)
    yc = -r * np.cos(th)
    d = np.sqrt((mesh.xy[:, 0] - x0) ** 2 + (mesh.xy[:, 1] - yc) ** 2)
    return 0.5 + 0.5 * np.tanh(2.0 * (r - d) / xi)


def cap_mesh(h: float, rough_amp: float = 0.0) -> Mesh:
    return split_grid_mesh(128.0, uniform_rows(64.0, int(round(64 / h)) + 1), int(round(128 / h)), seed=[17],
                           jitter=0.2, rough_amp=rough_amp)


def contact_angle_cap_errors(measure, h: float, thetas=(30.0, 60.0, 90.0, 120.0, 150.0), rough_amp: float = 0.0):
    """Sec. III.B: the angle a measurement reads on exact circular caps (tanh
    profile, xi = 4) of base 2 r sin theta and height r (1 - cos theta) against
    the imposed geometric angle, on a jittered mesh of spacing h.  The cap
    radius is chosen so that the cap area is that of a half disc of radius 20.
    measure(mesh, C) -> theta in degrees.  Returns the signed errors."""
    mesh = cap_mesh(h, rough_amp)
    out = []
    for th in thetas:
        t = np.deg2rad(th)
        r = 20.0 * np.sqrt(0.5 * np.pi / (t - np.sin(t) * np.cos(t)))   # cap area = pi 20^2 / 2
        out.append(measure(mesh, cap_field(mesh, th, r, 64.0, 4.0)) - th)
    return np.asarray(out)


def band_energy_error() -> float:
    """Band average <rho u.u> of the parasitic-current table (Sec. III.A) against
    a hand count: on a unit grid, the nodes (i, j) with 3 <= |(i, j) - (16, 8)|
    <= 5 enumerated one by one, with C = 1 (rho = rho_l = 1) and the velocity
    field u = (0.01 (x - 16), 0.002 y) set through the equilibria.  Also the
    whole-domain <T> = 1/2 sum rho |u|^2 / N and max |u| (Sec. III.B)."""
    mesh = split_grid_mesh(32.0, uniform_rows(16.0, 17), 32, seed=[1], jitter=0.0, diag="up")
    phys = make_physics(sigma=0.01, m_rho=10, m_nu=1, dt=0.1)
    o = fo.Oracle(mesh, phys, np.zeros(mesh.n_nodes))
    x, y = mesh.xy[:, 0], mesh.xy[:, 1]
    u = np.stack([0.01 * (x - 16.0), 0.002 * y], 1)
    g, h = o.init_state(np.ones(mesh.n_nodes), u=u)
    d = o.diagnostics(g, h, band=(16.0, 8.0, 4.0, 1.0))
    vals, total, peak = [], 0.0, 0.0
    for j in range(17):
        for i in range(32):
            ux, uy = 0.01 * (i - 16.0), 0.002 * j
            if j in (0, 16):
                ux = uy = 0.0                  # the wall operator zeroes the wall velocity
            total += ux * ux + uy * uy
            peak = max(peak, np.hypot(ux, uy))
            r2 = (i - 16) ** 2 + (j - 8) ** 2
            if 9 <= r2 <= 25:
                vals.append(ux * ux + uy * uy)
    band_ref = sum(vals) / len(vals)
    errs = [abs(d["band_ke"] - band_ref) / band_ref, abs(d["mean_ke"] - 0.5 * total / (17 * 32)) / (0.5 * total / (17 * 32)),
            abs(d["max_u"] - peak) / peak]
    return float(max(errs))


# ---------------------------------------------------------------------------
# Nodal forces integrated in the collision step (readings NC1-NC5)
# ---------------------------------------------------------------------------
def collision_step_moment_error() -> float:
    """Trapezoid rule on the force (NC1) with the half-force moments of psi_bar
    (NC3): over one collision the populations' moments change by dt times the
    force's moments, sum_a (h_hat - h_bar) = dt M lap mu_n,
    sum_a (g_hat - g_bar) = dt c_s^2 u . grad rho_n and
    sum_a e_a (g_hat - g_bar) = dt c_s^2 mu grad C_n at every node off the walls
    (the moments of eq:G and eq:H with sum Gamma = 1, sum (e - u) Gamma = 0,
    sum e (e - u) Gamma = c_s^2 I); at wall nodes the first moment of g_hat
    stays zero (NC4)."""
    mesh = small_mesh()
    phys = make_physics(sigma=0.01, m_rho=10, m_nu=2, dt=0.1)
    from workloads import droplet_field, wetting_from_angles
    o = fo.Oracle(mesh, phys, wetting_from_angles(mesh, 60.0), force_scheme="nodal_collide")
    rng = np.random.default_rng(4)
    C = droplet_field(mesh, [(8.0, 0.0, 4.0)], phys.xi)
    g, h = o.init_state(C, u=rng.normal(0, 0.01, (mesh.n_nodes, 2)), p=rng.normal(0, 1e-3, mesh.n_nodes))
    g, h = o.step(g, h)
    _, _, f = o.step(g, h, return_fields=True)
    dt, wall = phys.dt, o.geo.is_wall_node
    inner = ~wall
    e1 = abs((f["h_hat"] - h).sum(1) - dt * o.prm.mobility * f["lapmu_n"])[inner].max()
    e2 = abs((f["g_hat"] - g).sum(1) - dt * fo.CS2 * (f["u"] * f["gradrho_n"]).sum(1))[inner].max()
    first = np.stack([(f["g_hat"] - g) @ fo.E[:, 0], (f["g_hat"] - g) @ fo.E[:, 1]], 1)
    e3 = abs(first - dt * fo.CS2 * f["mu"][:, None] * f["gradC_n"])[inner].max()
    e4 = abs(np.stack([f["g_hat"] @ fo.E[:, 0], f["g_hat"] @ fo.E[:, 1]], 1)[wall]).max()
    return float(max(e1, e2, e3, e4))


def collision_step_mass_drift(steps=20) -> float:
    mesh = small_mesh()
    phys = make_physics(sigma=0.01, m_rho=10, m_nu=1, dt=0.1)
    from workloads import droplet_field, wetting_from_angles
    o = fo.Oracle(mesh, phys, wetting_from_angles(mesh, 60.0, 110.0), force_scheme="nodal_collide")
    g, h = o.init_state(droplet_field(mesh, [(8.0, 0.0, 4.0)], phys.xi))
    m0 = o.mass(h)
    g, h = o.run(g, h, steps)
    return float(abs(o.mass(h) - m0) / m0)


def collision_step_static_drift(seed=3) -> float:
    """The static interface of Sec. II.C with the collision-step nodal force: not
    balanced (compare static_balance_drift)."""
    mesh = small_mesh(seed=seed)
    phys = make_physics(sigma=0.0, m_rho=10, m_nu=1, dt=0.1, mobility=0.0)
    o = fo.Oracle(mesh, phys, np.zeros(mesh.n_nodes), force_scheme="nodal_collide")
    rng = np.random.default_rng(seed)
    g, h = o.init_state(rng.uniform(0.0, 1.0, mesh.n_nodes))
    g1, h1 = o.step(g, h)
    return float(max(abs(h1 - h).max(), abs(g1 - g).max()) / abs(h).max())
