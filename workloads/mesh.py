"""Seeded synthetic triangle meshes for the droplet-on-wall workloads.

This module generates geometry only: node coordinates, triangle connectivity,
the wall-edge list and the x period.  It holds none of the lattice Boltzmann
or finite element arithmetic; both the CPU oracle and the GPU library consume
its output independently.

Construction (split-quad grid):
  * an (nx) x (ny) point grid (x periodic: column nx is identified with
    column 0), or an (nx+1) x (ny) grid with walls on all four sides;
  * interior points (not on a wall row, not on the seam column) are jittered
    independently in x and y by U(-j, j) times the local spacing;
  * each quad is split along a diagonal chosen by a fair seeded coin;
  * optionally a sinusoidal roughness is sheared into the bottom wall.

Node numbering is row-major: node (i, j) -> j * ncols + i.  Triangles are
counter-clockwise after the periodic unwrap (minimum image in x).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Mesh:
    xy: np.ndarray            # (N, 2) float64 node coordinates
    tri: np.ndarray           # (E, 3) int32, counter-clockwise after unwrap
    wall_edges: np.ndarray    # (W, 2) int32 node pairs on solid walls
    period_x: float           # x period (0.0 = not periodic)
    ncols: int                # nodes per row
    nrows: int                # rows
    wall_side: np.ndarray = field(default=None)  # (W,) int8: 0 bottom, 1 top, 2 left, 3 right

    @property
    def n_nodes(self) -> int:
        return int(self.xy.shape[0])

    @property
    def n_tris(self) -> int:
        return int(self.tri.shape[0])

    def wall_nodes(self, side: int | None = None) -> np.ndarray:
        e = self.wall_edges if side is None else self.wall_edges[self.wall_side == side]
        return np.unique(e.ravel())


def uniform_rows(ly: float, nrows: int) -> np.ndarray:
    """Row y-coordinates of a uniform grid with nrows rows spanning [0, ly]."""
    return np.linspace(0.0, ly, nrows)


def graded_rows(ly: float, h_bulk: float, h_fine: float = 0.25, y_fine: float = 32.0,
                growth: float = 1.05) -> np.ndarray:
    """Wall-graded rows: spacing h_fine up to y_fine, then geometric growth by
    `growth` per row up to h_bulk, then h_bulk up to the top wall.  The last
    row is snapped onto y = ly (it replaces a row closer than half a spacing)."""
    ys = [0.0]
    while ys[-1] < y_fine - 1e-12:
        ys.append(ys[-1] + h_fine)
    s = h_fine
    while True:
        s = min(s * growth, h_bulk)
        y = ys[-1] + s
        if y >= ly - 0.5 * s:
            ys.append(float(ly))
            break
        ys.append(y)
    return np.asarray(ys, dtype=np.float64)


def unwrap_tri_xy(xy: np.ndarray, tri: np.ndarray, period_x: float) -> np.ndarray:
    """(E, 3, 2) vertex coordinates with x shifted to the minimum image of vertex 0."""
    p = xy[tri].copy()
    if period_x > 0:
        for k in (1, 2):
            dx = p[:, k, 0] - p[:, 0, 0]
            p[:, k, 0] -= period_x * np.round(dx / period_x)
    return p


def split_grid_mesh(lx: float, rows: np.ndarray, ncols: int, seed, *, jitter: float = 0.2,
                    periodic: bool = True, rough_amp: float = 0.0, rough_period: float = 64.0,
                    rough_decay: float = 64.0, diag: str = "random") -> Mesh:
    """Jittered split-quad triangle mesh.

    lx      domain length in x; columns are uniformly spaced by lx / ncols
    rows    (nrows,) increasing y coordinates; rows[0] = bottom wall, rows[-1] = top wall
    seed    anything accepted by numpy.random.default_rng; sub-streams are
            default_rng([*seed, k]) with k = 0 (x jitter), 1 (y jitter), 2 (diagonals)
    diag    "random" (fair coin per quad), "up" (all (i,j)-(i+1,j+1)) or "down"
    """
    seed = list(np.atleast_1d(seed).astype(int))
    rows = np.asarray(rows, dtype=np.float64)
    nrows = rows.size
    hx = lx / ncols
    npts_x = ncols if periodic else ncols + 1
    xs = np.arange(npts_x, dtype=np.float64) * hx
    X, Y = np.meshgrid(xs, rows)  # (nrows, npts_x)

    # local y spacing: smaller of the two neighbouring row gaps
    gap = np.diff(rows)
    hy = np.empty(nrows)
    hy[0], hy[-1] = gap[0], gap[-1]
    hy[1:-1] = np.minimum(gap[:-1], gap[1:])

    interior = np.zeros_like(X, dtype=bool)
    interior[1:-1, 1:(npts_x if periodic else npts_x - 1)] = True
    if jitter > 0:
        rx = np.random.default_rng(seed + [0]).uniform(-jitter, jitter, X.shape)
        ry = np.random.default_rng(seed + [1]).uniform(-jitter, jitter, X.shape)
        X = X + np.where(interior, rx * hx, 0.0)
        Y = Y + np.where(interior, ry * hy[:, None], 0.0)
    if rough_amp != 0.0:
        Y = Y + rough_amp * np.sin(2.0 * np.pi * X / rough_period) * np.maximum(0.0, 1.0 - Y / rough_decay)

    xy = np.stack([X.ravel(), Y.ravel()], axis=1)

    nq = ncols  # quads per row
    if diag == "random":
        flip = np.random.default_rng(seed + [2]).random((nrows - 1, nq)) < 0.5
    elif diag == "up":
        flip = np.zeros((nrows - 1, nq), dtype=bool)
    elif diag == "down":
        flip = np.ones((nrows - 1, nq), dtype=bool)
    else:
        raise ValueError(diag)

    j, i = np.meshgrid(np.arange(nrows - 1), np.arange(nq), indexing="ij")
    i1 = (i + 1) % npts_x if periodic else i + 1
    n00 = j * npts_x + i
    n10 = j * npts_x + i1
    n01 = (j + 1) * npts_x + i
    n11 = (j + 1) * npts_x + i1
    # diagonal (0,0)-(1,1): [00,10,11], [00,11,01]; diagonal (1,0)-(0,1): [00,10,01], [10,11,01]
    t_a = np.where(flip[..., None], np.stack([n00, n10, n01], -1), np.stack([n00, n10, n11], -1))
    t_b = np.where(flip[..., None], np.stack([n10, n11, n01], -1), np.stack([n00, n11, n01], -1))
    tri = np.stack([t_a, t_b], axis=2).reshape(-1, 3).astype(np.int32)

    walls, side = [], []
    bi = np.arange(nq)
    bi1 = (bi + 1) % npts_x if periodic else bi + 1
    walls.append(np.stack([bi, bi1], 1)); side.append(np.zeros(nq, np.int8))
    top = (nrows - 1) * npts_x
    walls.append(np.stack([top + bi, top + bi1], 1)); side.append(np.ones(nq, np.int8))
    if not periodic:
        jj = np.arange(nrows - 1)
        walls.append(np.stack([jj * npts_x, (jj + 1) * npts_x], 1)); side.append(np.full(nrows - 1, 2, np.int8))
        walls.append(np.stack([jj * npts_x + ncols, (jj + 1) * npts_x + ncols], 1)); side.append(np.full(nrows - 1, 3, np.int8))
    wall_edges = np.concatenate(walls).astype(np.int32)
    wall_side = np.concatenate(side)

    mesh = Mesh(xy=xy, tri=tri, wall_edges=wall_edges, period_x=float(lx) if periodic else 0.0,
                ncols=npts_x, nrows=nrows, wall_side=wall_side)
    p = unwrap_tri_xy(xy, tri, mesh.period_x)
    area2 = (p[:, 1, 0] - p[:, 0, 0]) * (p[:, 2, 1] - p[:, 0, 1]) - (p[:, 2, 0] - p[:, 0, 0]) * (p[:, 1, 1] - p[:, 0, 1])
    if not np.all(area2 > 0):
        raise RuntimeError("mesh generator produced a non-positive triangle")
    return mesh


def channel_mesh(lx: float, ly: float, h: float, x0: float, x1: float, y0: float, y1: float, seed, *,
                 jitter: float = 0.2) -> Mesh:
    """x-periodic box [0, lx) x [0, ly] meshed as a split-quad grid of spacing
    h, with two solid blocks removed: x0 <= x <= x1 below y0 and above y1.
    Between the blocks runs a channel of width y1 - y0 and length x1 - x0
    that joins the two sides of the box (one reservoir, through the period).

    Every boundary edge is a wall edge.  wall_side: 0 bottom and 1 top of the
    box, 4 the channel walls (y = y0 or y1), 5 the block end faces (x = x0 or
    x1).  Nodes that lie on no wall are jittered by U(-jitter, jitter) h in x
    and y; wall nodes stay on the grid lines, so the walls are straight.  The
    block edges must lie on grid lines (multiples of h)."""
    seed = list(np.atleast_1d(seed).astype(int))
    ncols, nrows = int(round(lx / h)), int(round(ly / h)) + 1
    for v in (x0, x1, y0, y1):
        if abs(v / h - round(v / h)) > 1e-9:
            raise ValueError("channel_mesh: block edges must lie on grid lines")
    if not (0.0 < x0 < x1 < lx and 0.0 < y0 < y1 < ly):
        raise ValueError("channel_mesh: blocks must lie strictly inside the box")
    X, Y = np.meshgrid(np.arange(ncols) * h, np.arange(nrows) * h)
    flip = np.random.default_rng(seed + [2]).random((nrows - 1, ncols)) < 0.5
    j, i = np.meshgrid(np.arange(nrows - 1), np.arange(ncols), indexing="ij")
    i1 = (i + 1) % ncols
    n00, n10 = j * ncols + i, j * ncols + i1
    n01, n11 = (j + 1) * ncols + i, (j + 1) * ncols + i1
    # the quad (i, j) spans [i h, (i+1) h] x [j h, (j+1) h]; it is solid when its centre is in a block
    cx, cy = (i + 0.5) * h, (j + 0.5) * h
    fluid = ~((cx > x0) & (cx < x1) & ((cy < y0) | (cy > y1)))
    t_a = np.where(flip[..., None], np.stack([n00, n10, n01], -1), np.stack([n00, n10, n11], -1))
    t_b = np.where(flip[..., None], np.stack([n10, n11, n01], -1), np.stack([n00, n11, n01], -1))
    tri = np.stack([t_a, t_b], axis=2)[fluid].reshape(-1, 3)
    used = np.unique(tri)
    remap = np.full(nrows * ncols, -1, np.int64)
    remap[used] = np.arange(used.size)
    tri = remap[tri].astype(np.int32)
    xy = np.stack([X.ravel(), Y.ravel()], axis=1)[used]

    # boundary edges: edges of exactly one triangle
    e = np.concatenate([tri[:, [0, 1]], tri[:, [1, 2]], tri[:, [2, 0]]])
    key = np.sort(e, axis=1)
    uniq, inv, cnt = np.unique(key, axis=0, return_inverse=True, return_counts=True)
    bnd = cnt[inv.ravel()] == 1
    walls = e[bnd].astype(np.int32)          # oriented as in their triangle (fluid on the left)
    pa, pb = xy[walls[:, 0]], xy[walls[:, 1]]
    tol = 1e-9 * h
    side = np.full(len(walls), -1, np.int8)
    side[(np.abs(pa[:, 1]) < tol) & (np.abs(pb[:, 1]) < tol)] = 0
    side[(np.abs(pa[:, 1] - ly) < tol) & (np.abs(pb[:, 1] - ly) < tol)] = 1
    horiz = np.abs(pa[:, 1] - pb[:, 1]) < tol
    on_ch = horiz & ((np.abs(pa[:, 1] - y0) < tol) | (np.abs(pa[:, 1] - y1) < tol))
    side[on_ch] = 4
    vert = np.abs(pa[:, 0] - pb[:, 0]) < tol
    side[vert & ((np.abs(pa[:, 0] - x0) < tol) | (np.abs(pa[:, 0] - x1) < tol))] = 5
    if np.any(side < 0):
        raise RuntimeError("channel_mesh: unclassified boundary edge")

    on_wall = np.zeros(len(xy), bool)
    on_wall[walls.ravel()] = True
    if jitter > 0:
        r = np.random.default_rng(seed + [0]).uniform(-jitter, jitter, (nrows * ncols, 2))[used]
        xy = xy + np.where(on_wall[:, None], 0.0, r * h)
    mesh = Mesh(xy=xy, tri=tri, wall_edges=walls, period_x=float(lx), ncols=ncols, nrows=nrows, wall_side=side)
    p = unwrap_tri_xy(xy, tri, mesh.period_x)
    area2 = (p[:, 1, 0] - p[:, 0, 0]) * (p[:, 2, 1] - p[:, 0, 1]) - (p[:, 2, 0] - p[:, 0, 0]) * (p[:, 1, 1] - p[:, 0, 1])
    if not np.all(area2 > 0):
        raise RuntimeError("mesh generator produced a non-positive triangle")
    return mesh
