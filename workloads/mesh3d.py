"""Seeded synthetic tetrahedral meshes for the 3-D workloads (D3Q19 on linear
tetrahedra, the paper's own setting).

Geometry only: node coordinates, tetrahedron connectivity, the wall-face list
and the periods; no lattice Boltzmann or finite element arithmetic.

Construction (Kuhn-split box):
  * an nx x ny x nz-cell box, x and y periodic (node column nx is node column
    0, and likewise in y), solid walls at z = 0 and z = lz;
  * nodes off the walls are jittered independently in x, y and z by
    U(-j, j) times the local spacing;
  * each cell is split into the six tetrahedra of the Kuhn (Freudenthal)
    subdivision, paths from corner (0,0,0) to (1,1,1) along the three axes
    in each order; every cell is split the same way, so faces match across
    cells.
Tetrahedra are oriented with positive volume after the periodic unwrap
(minimum image of each vertex relative to vertex 0).
"""
from __future__ import annotations

from dataclasses import dataclass
from itertools import permutations

import numpy as np


@dataclass
class TetMesh:
    xyz: np.ndarray          # (N, 3) float64
    tet: np.ndarray          # (E, 4) int32, positive volume after unwrap
    wall_faces: np.ndarray   # (W, 3) int32 node triples on solid walls
    wall_side: np.ndarray    # (W,) int8: 0 bottom (z = 0), 1 top (z = lz)
    period: tuple            # (period_x, period_y); 0 = not periodic
    shape: tuple             # (nx, ny, nz) cells

    @property
    def n_nodes(self) -> int:
        return int(self.xyz.shape[0])

    @property
    def n_tets(self) -> int:
        return int(self.tet.shape[0])

    def wall_nodes(self, side: int | None = None) -> np.ndarray:
        f = self.wall_faces if side is None else self.wall_faces[self.wall_side == side]
        return np.unique(f.ravel())


def unwrap_tet_xyz(xyz: np.ndarray, tet: np.ndarray, period) -> np.ndarray:
    """(E, 4, 3) vertex coordinates, x and y shifted to the minimum image of vertex 0."""
    p = xyz[tet].copy()
    for d, L in enumerate(period):
        if L > 0:
            for k in (1, 2, 3):
                p[:, k, d] -= L * np.round((p[:, k, d] - p[:, 0, d]) / L)
    return p


def signed_volumes(p: np.ndarray) -> np.ndarray:
    a, b, c = p[:, 1] - p[:, 0], p[:, 2] - p[:, 0], p[:, 3] - p[:, 0]
    return np.einsum("ij,ij->i", a, np.cross(b, c)) / 6.0


def tet_box_mesh(lx: float, ly: float, lz: float, nx: int, ny: int, nz: int, seed, *, jitter: float = 0.2,
                 z_rows: np.ndarray | None = None) -> TetMesh:
    """Jittered Kuhn-split box, periodic in x and y, walls at z = 0 and z = lz.
    z_rows (nz + 1 increasing values from 0 to lz) overrides uniform layers."""
    seed = list(np.atleast_1d(seed).astype(int))
    hx, hy = lx / nx, ly / ny
    zs = np.linspace(0.0, lz, nz + 1) if z_rows is None else np.asarray(z_rows, dtype=np.float64)
    gap = np.diff(zs)
    hz = np.empty(nz + 1)
    hz[0], hz[-1] = gap[0], gap[-1]
    hz[1:-1] = np.minimum(gap[:-1], gap[1:])
    I, J, K = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz + 1), indexing="ij")
    X, Y, Z = I * hx, J * hy, zs[K]
    if jitter > 0:
        inner = (K > 0) & (K < nz)
        r = [np.random.default_rng(seed + [d]).uniform(-jitter, jitter, X.shape) for d in range(3)]
        X = X + np.where(inner, r[0] * hx, 0.0)
        Y = Y + np.where(inner, r[1] * hy, 0.0)
        Z = Z + np.where(inner, r[2] * hz[K], 0.0)

    def node(i, j, k):
        return ((i % nx) * ny + (j % ny)) * (nz + 1) + k

    xyz = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    ci, cj, ck = (a.ravel() for a in np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij"))
    tets = []
    for perm in permutations(range(3)):
        corner = np.zeros(3, dtype=int)
        verts = [node(ci, cj, ck)]
        for axis in perm:
            corner[axis] += 1
            verts.append(node(ci + corner[0], cj + corner[1], ck + corner[2]))
        tets.append(np.stack(verts, axis=1))
    tet = np.concatenate(tets).astype(np.int32)
    period = (float(lx), float(ly))
    vol = signed_volumes(unwrap_tet_xyz(xyz, tet, period))
    flip = vol < 0
    tet[flip, 2], tet[flip, 3] = tet[flip, 3].copy(), tet[flip, 2].copy()
    if not np.all(signed_volumes(unwrap_tet_xyz(xyz, tet, period)) > 0):
        raise RuntimeError("tet_box_mesh produced a degenerate tetrahedron")
    # boundary faces: faces of exactly one tetrahedron
    faces = np.concatenate([tet[:, [1, 2, 3]], tet[:, [0, 3, 2]], tet[:, [0, 1, 3]], tet[:, [0, 2, 1]]])
    key = np.sort(faces, axis=1).astype(np.int64)
    n = np.int64(xyz.shape[0])
    if float(n) ** 3 < 2.0 ** 62:  # one int64 per sorted triple
        _, inv, cnt = np.unique((key[:, 0] * n + key[:, 1]) * n + key[:, 2], return_inverse=True,
                                return_counts=True)
    else:
        _, inv, cnt = np.unique(key, axis=0, return_inverse=True, return_counts=True)
    bnd = faces[cnt[inv.ravel()] == 1]
    zf = xyz[bnd, 2]
    side = np.full(len(bnd), -1, np.int8)
    side[np.all(zf == 0.0, axis=1)] = 0
    side[np.all(zf == lz, axis=1)] = 1
    if np.any(side < 0):
        raise RuntimeError("tet_box_mesh: boundary face off the walls")
    return TetMesh(xyz=xyz, tet=tet, wall_faces=bnd.astype(np.int32), wall_side=side, period=period,
                   shape=(nx, ny, nz))


def droplet_field_3d(mesh: TetMesh, droplets, xi: float) -> np.ndarray:
    """C = 1/2 + 1/2 tanh(2 (R - |x - x_c|) / xi) around each centre (minimum
    image in the periodic directions); several droplets combine by maximum."""
    C = np.zeros(mesh.n_nodes)
    for (xc, yc, zc, R) in droplets:
        d2 = (mesh.xyz[:, 2] - zc) ** 2
        for dim, (c, L) in enumerate(((xc, mesh.period[0]), (yc, mesh.period[1]))):
            dd = mesh.xyz[:, dim] - c
            if L > 0:
                dd -= L * np.round(dd / L)
            d2 = d2 + dd * dd
        C = np.maximum(C, 0.5 + 0.5 * np.tanh(2.0 * (R - np.sqrt(d2)) / xi))
    return C


def wetting_from_angles_3d(mesh: TetMesh, theta_bottom_deg, theta_top_deg=90.0) -> np.ndarray:
    """Per-node Omega_c = -cos(theta) on the bottom and top walls (Young)."""
    om = np.zeros(mesh.n_nodes)
    for side, th in ((0, theta_bottom_deg), (1, theta_top_deg)):
        nodes = mesh.wall_nodes(side)
        om[nodes] = -np.cos(np.deg2rad(float(th)))
    return om


def graded_z_rows(fine: float, fine_top: float, growth: float, coarse: float, nz: int) -> np.ndarray:
    """nz + 1 layer heights from z = 0: spacing `fine` up to z = fine_top, then
    growing by `growth` per layer up to `coarse`, then constant."""
    z = [0.0]
    h = fine
    while len(z) < nz + 1:
        if z[-1] + 1e-12 >= fine_top:
            h = min(h * growth, coarse)
        z.append(z[-1] + h)
    return np.asarray(z)


def sessile_drop_3d(nx: int = 128, ny: int = 128, nz: int = 90, R: float = 32.0, theta: float = 150.0,
                    m_rho: float = 10.0, m_nu: float = 1.0, sigma: float = 0.0025, seed: int = 7):
    """The 3-D droplet of the paper's equilibrium-shape study (Sec. III): a
    hemisphere of radius R resting on the bottom wall of a box whose layers
    are refined toward that wall, wetting potential of theta_eq on the bottom,
    90 deg on the top.  Defaults: 128 x 128 unit columns, 90 layers of 0.5 up
    to z = 16 growing by 6 % to 1.25 (top at z ~ 82); 1,490,944 nodes
    (the paper's mesh holds 1.5e6), 8,847,360 tetrahedra; xi = 4, sigma = 0.0025,
    mobility 0.02, dt = 0.05, tau_l = 1, densities and viscosities by
    M_rho, M_nu.  Returns (name, mesh, physics, C0, Omega_c, droplets)."""
    from .configs import make_physics
    z_rows = graded_z_rows(0.5, 16.0, 1.06, 1.25, nz)
    mesh = tet_box_mesh(float(nx), float(ny), float(z_rows[-1]), nx, ny, nz, seed=[seed], z_rows=z_rows)
    phys = make_physics(sigma=sigma, m_rho=m_rho, m_nu=m_nu, dt=0.05)
    drops = [(0.5 * nx, 0.5 * ny, 0.0, R)]
    C0 = droplet_field_3d(mesh, drops, phys.xi)
    om = wetting_from_angles_3d(mesh, theta, 90.0)
    name = f"sessile3d-{nx}x{ny}x{nz}-R{R:g}-theta{theta:g}"
    return name, mesh, phys, C0, om, drops
