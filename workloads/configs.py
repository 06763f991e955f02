"""The synthetic workloads: the five droplet-on-wall configurations and the
inputs of the comparison studies (free droplet, sessile droplet, capillary
channel), each as mesh, physical constants, initial composition field and
per-node wetting potential.

Everything here is input data.  Physical constants are given in the form the
paper states them (surface tension sigma, interface width xi, mobility M,
densities, kinematic viscosities, time step); the derived free-energy
constants (kappa, beta, phi_c, relaxation times) are computed by each
consumer on its own.

Readings for constants the paper leaves open:
  * time step: dt = 0.1 on unit-spacing meshes, 0.025 on wall-graded meshes;
  * liquid viscosity nu_l = dt / 3 (liquid relaxation time 1), and the
    viscosity ratio is nu_v / nu_l;
  * mobility M = 0.02 everywhere; the top wall is neutral (theta = 90 deg);
  * the wetting potential of a wall node is Omega_c = -cos(theta) (Young).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .mesh import Mesh, channel_mesh, graded_rows, split_grid_mesh, uniform_rows


@dataclass
class Physics:
    sigma: float
    xi: float
    mobility: float
    rho_l: float
    rho_v: float
    nu_l: float
    nu_v: float
    dt: float


@dataclass
class Workload:
    name: str
    mesh: Mesh
    phys: Physics
    C0: np.ndarray                     # (N,) initial composition
    omega_c: np.ndarray                # (N,) wetting potential, read at wall nodes only
    steps: int
    droplets: list = field(default_factory=list)   # [(xc, yc, R)]
    extra: dict = field(default_factory=dict)


def make_physics(sigma, m_rho, m_nu, dt, xi=4.0, mobility=0.02, rho_l=1.0) -> Physics:
    nu_l = dt / 3.0
    return Physics(sigma=sigma, xi=xi, mobility=mobility, rho_l=rho_l, rho_v=rho_l / m_rho,
                   nu_l=nu_l, nu_v=nu_l * m_nu, dt=dt)


def droplet_field(mesh: Mesh, droplets, xi: float) -> np.ndarray:
    """C = 1/2 + 1/2 tanh(2 (R - |x - x_c|) / xi) around each centre (minimum
    image in x for periodic meshes); several droplets combine by maximum."""
    C = np.zeros(mesh.n_nodes)
    for (xc, yc, R) in droplets:
        dx = mesh.xy[:, 0] - xc
        if mesh.period_x > 0:
            dx -= mesh.period_x * np.round(dx / mesh.period_x)
        d = np.sqrt(dx * dx + (mesh.xy[:, 1] - yc) ** 2)
        C = np.maximum(C, 0.5 + 0.5 * np.tanh(2.0 * (R - d) / xi))
    return C


def wetting_from_angles(mesh: Mesh, theta_bottom_deg, theta_top_deg=90.0) -> np.ndarray:
    """Per-node Omega_c = -cos(theta).  theta_bottom_deg is a scalar or a
    callable of the node x coordinate; only wall nodes get a nonzero value."""
    om = np.zeros(mesh.n_nodes)
    for side, th in ((0, theta_bottom_deg), (1, theta_top_deg)):
        nodes = mesh.wall_nodes(side)
        t = th(mesh.xy[nodes, 0]) if callable(th) else np.full(nodes.size, float(th))
        om[nodes] = -np.cos(np.deg2rad(t))
    return om


def fourier_field(x: np.ndarray, period: float, seed, n_modes: int = 4) -> np.ndarray:
    """Normalised sum of n_modes random-phase cosines of the given period
    (mode k has amplitude 1/k); max |f| over x equals 1."""
    ph = np.random.default_rng(list(np.atleast_1d(seed)) + [3]).uniform(0, 2 * np.pi, n_modes)
    f = sum(np.cos(2 * np.pi * (k + 1) * x / period + ph[k]) / (k + 1) for k in range(n_modes))
    return f / np.max(np.abs(f))


def config(cfg: int, row_limit: int | None = None) -> Workload:
    """Build workload 1..5.  row_limit keeps only the bottom row_limit node
    rows of the mesh (the top row becomes the top wall): a bounded sample of
    the same workload for CPU timing."""
    w = _config(cfg)
    if row_limit is None or row_limit >= w.mesh.nrows:
        return w
    m = w.mesh
    keep = row_limit * m.ncols
    tri_keep = np.all(m.tri < keep, axis=1)
    top = (row_limit - 1) * m.ncols
    bi = np.arange(m.ncols - (0 if m.period_x > 0 else 1))
    bi1 = (bi + 1) % m.ncols if m.period_x > 0 else bi + 1
    walls = np.concatenate([m.wall_edges[m.wall_side == 0], np.stack([top + bi, top + bi1], 1)]).astype(np.int32)
    side = np.concatenate([np.zeros(int((m.wall_side == 0).sum()), np.int8), np.ones(bi.size, np.int8)])
    sub = Mesh(xy=m.xy[:keep].copy(), tri=m.tri[tri_keep].copy(), wall_edges=walls, period_x=m.period_x,
               ncols=m.ncols, nrows=row_limit, wall_side=side)
    om = w.omega_c[:keep].copy()
    om[sub.wall_nodes(1)] = 0.0
    return Workload(w.name + f"-bottom-{row_limit}-rows", sub, w.phys, w.C0[:keep].copy(), om, w.steps, w.droplets,
                    dict(w.extra))


def _config(cfg: int) -> Workload:
    if cfg == 1:
        mesh = split_grid_mesh(64.0, uniform_rows(32.0, 33), 64, seed=[1])
        phys = make_physics(sigma=0.01, m_rho=10.0, m_nu=1.0, dt=0.1)
        drops = [(32.0, 0.0, 12.0)]
        om = wetting_from_angles(mesh, 90.0)
        return Workload("droplet-64x32-fp64", mesh, phys, droplet_field(mesh, drops, phys.xi), om, 200, drops)
    if cfg == 2:
        mesh = split_grid_mesh(512.0, uniform_rows(256.0, 257), 512, seed=[2])
        phys = make_physics(sigma=0.005, m_rho=100.0, m_nu=10.0, dt=0.1)
        drops = [(256.0, 0.0, 64.0)]
        om = wetting_from_angles(mesh, 60.0)
        return Workload("droplet-512x256-theta60", mesh, phys, droplet_field(mesh, drops, phys.xi), om, 10000, drops)
    if cfg == 3:
        mesh = split_grid_mesh(2048.0, graded_rows(1024.0, 1.1), 2048, seed=[3], rough_amp=4.0,
                               rough_period=64.0, rough_decay=64.0)
        phys = make_physics(sigma=0.005, m_rho=1000.0, m_nu=40.0, dt=0.025)
        L = 2048.0
        drops = [(L / 6, 0.0, 80.0), (L / 2, 0.0, 80.0), (5 * L / 6, 0.0, 80.0)]
        th = lambda x: np.where(x < L / 3, 45.0, np.where(x < 2 * L / 3, 90.0, 135.0))
        om = wetting_from_angles(mesh, th)
        return Workload("3-droplets-2048x1024-graded-rough", mesh, phys, droplet_field(mesh, drops, phys.xi), om,
                        2000, drops)
    if cfg == 4:
        mesh = split_grid_mesh(256.0, uniform_rows(128.0, 129), 256, seed=[4])
        phys = make_physics(sigma=0.01, m_rho=10.0, m_nu=1.0, dt=0.1)
        drops = [(128.0, 0.0, 32.0)]
        th = lambda x: 90.0 + 40.0 * fourier_field(x, 256.0, [4])
        om = wetting_from_angles(mesh, th)
        return Workload("adjoint-256x128", mesh, phys, droplet_field(mesh, drops, phys.xi), om, 500, drops,
                        extra={"ckpt_every": 50})
    if cfg == 5:
        mesh = split_grid_mesh(1024.0, graded_rows(512.0, 1.3), 1024, seed=[5])
        phys = make_physics(sigma=0.01, m_rho=10.0, m_nu=1.0, dt=0.025)
        drops = [(512.0, 0.0, 64.0)]
        th = lambda x: 90.0 + 40.0 * fourier_field(x, 1024.0, [5])
        om = wetting_from_angles(mesh, th)
        r = np.random.default_rng([5, 4])
        shift, scale = r.uniform(-32.0, 32.0), r.uniform(0.9, 1.1)
        target = droplet_field(mesh, [(512.0 + shift, 0.0, 64.0 * scale)], phys.xi)
        return Workload("adjoint-1024x512-graded", mesh, phys, droplet_field(mesh, drops, phys.xi), om, 2000, drops,
                        extra={"ckpt_every": 100, "C_target": target})
    raise ValueError(f"no workload {cfg}")


def free_droplet(level: int, t_end: float = 8000.0) -> Workload:
    """Static droplet for the parasitic-current comparison (the 2-D analogue of
    the table of Sec. III.A): density ratio 2, equal kinematic viscosities
    (1/30 in both phases), radius 16 centred in a 64 x 64 box (x-periodic,
    neutral walls 16 units from the interface), jittered split mesh with
    spacing h = 2^-level (level 0, 1, 2: 4,160 / 16,512 / 65,792 nodes).
    Space and time are refined together, dt = 0.1 h, and the run covers the
    same physical time t_end at every level."""
    n = 64 * 2 ** level
    mesh = split_grid_mesh(64.0, uniform_rows(64.0, n + 1), n, seed=[10 + level])
    dt = 0.1 / 2 ** level
    nu = 0.1 / 3.0
    phys = Physics(sigma=0.01, xi=4.0, mobility=0.02, rho_l=1.0, rho_v=0.5, nu_l=nu, nu_v=nu, dt=dt)
    drops = [(32.0, 32.0, 16.0)]
    om = wetting_from_angles(mesh, 90.0)
    return Workload(f"free-droplet-64x64-level{level}", mesh, phys, droplet_field(mesh, drops, phys.xi),
                    om, int(round(t_end / dt)), drops)


def wetting_drop(theta_deg: float, m_rho: float = 10.0, m_nu: float = 1.0, refine: int = 2, xi: float = 4.0,
                 radius: float = 20.0, sigma: float = 0.01, mobility: float = 0.2, dt: float | None = None,
                 t_end: float = 8000.0, box: float = 6.4) -> Workload:
    """Sessile droplet for the equilibrium contact angle against the imposed
    wetting potential (the 2-D analogue of the angle sweep of Sec. III.B):
    a semicircular droplet of the given radius on the bottom wall of a
    box R x box R / 2 x-periodic box (box = 6.4 by default; wider for small
    angles, whose caps spread beyond it), wetting potential
    Omega_c = -cos(theta) on the bottom wall, neutral top wall.  Jittered
    split mesh with spacing h = 1 / refine; kinematic viscosity 1/30 in the
    liquid and m_nu / 30 in the vapour whatever the spacing; dt = 0.1 / refine
    unless given.  The explicit composition update needs dt below about
    h^4 / (32 M kappa)."""
    L = box * radius
    n = int(round(refine * L))
    mesh = split_grid_mesh(L, uniform_rows(3.2 * radius, int(round(refine * 3.2 * radius)) + 1), n, seed=[20])
    dt = 0.1 / refine if dt is None else dt
    nu = 0.1 / 3.0
    phys = Physics(sigma=sigma, xi=xi, mobility=mobility, rho_l=1.0, rho_v=1.0 / m_rho, nu_l=nu, nu_v=nu * m_nu,
                   dt=dt)
    drops = [(L / 2, 0.0, radius)]
    om = wetting_from_angles(mesh, theta_deg)
    return Workload(f"wetting-drop-theta{theta_deg:g}-h{1.0 / refine:g}-xi{xi:g}-box{box:g}", mesh, phys,
                    droplet_field(mesh, drops, xi), om, int(round(t_end / dt)), drops,
                    extra={"theta": theta_deg, "m_rho": m_rho, "m_nu": m_nu})


def capillary_channel(theta_deg: float, width: float = 10.0, length: float = 100.0, refine: int = 2,
                      xi: float = 4.0, sigma: float = 0.02, m_rho: float = 10.0, m_nu: float = 1.0,
                      mobility: float = 0.2, l0: float | None = None, t_end: float = 10000.0) -> Workload:
    """Capillary intrusion (the 2-D analogue of the capillary-tube experiment of
    Sec. III.C): a channel of the given width and length between two solid
    blocks (`channel_mesh`), wetting potential Omega_c = -cos(theta) on the
    channel walls, neutral box walls and block faces.  The box is 4 widths
    high; the reservoir (8 widths long, joined through the x period) holds a
    liquid slab of length 4 widths that reaches l0 (default one width) into
    the channel, vapour elsewhere; flat tanh interfaces of width xi.
    Spacing h = 1 / refine, dt = 0.1 / refine, nu_l = 1/30."""
    H = width
    ly = 4.0 * H
    y0, y1 = 1.5 * H, 2.5 * H
    slab = 4.0 * H
    x0 = slab + 2.0 * H
    x1 = x0 + length
    lx = x1 + 2.0 * H
    l0 = H if l0 is None else l0
    h = 1.0 / refine
    mesh = channel_mesh(lx, ly, h, x0, x1, y0, y1, seed=[30])
    dt = 0.1 / refine
    nu = 0.1 / 3.0
    phys = Physics(sigma=sigma, xi=xi, mobility=mobility, rho_l=1.0, rho_v=1.0 / m_rho, nu_l=nu, nu_v=nu * m_nu,
                   dt=dt)
    om = np.zeros(mesh.n_nodes)
    om[mesh.wall_nodes(4)] = -np.cos(np.radians(theta_deg))
    # corner nodes shared by a channel wall and a block face keep the channel value
    x = mesh.xy[:, 0]
    d = np.minimum(x - (x0 - slab), (x0 + l0) - x)
    C0 = 0.5 + 0.5 * np.tanh(2.0 * d / xi)
    return Workload(f"capillary-channel-theta{theta_deg:g}-H{H:g}-L{length:g}", mesh, phys, C0, om,
                    int(round(t_end / dt)), [],
                    extra={"theta": theta_deg, "x0": x0, "x1": x1, "y0": y0, "y1": y1, "l0": l0, "width": H,
                           "length": length})
