"""Host post-processing of fields read back from the library (Sec. III.B):
the equilibrium contact angle of a droplet on a flat wall measured on the
C = 0.5 contour from the droplet height h and base width b."""
from __future__ import annotations

import numpy as np


def contact_angle(xy, tri, bottom_nodes, C, period_x=0.0, level=0.5, x_window=None):
    """Contact angle (degrees), height and base of the droplet whose contour
    crosses the bottom wall y = 0 twice (inside x_window = (x0, x1) if given).

    b: distance between the two points where the P1 interpolant of C on the
    wall edges crosses `level`; h: highest point of the level line over the
    element edges (within the window).  The angle follows from the circular
    cap relation tan(theta / 2) = 2 h / b (the formula printed with the
    measurement returns pi - theta for an exact cap)."""
    xy = np.asarray(xy, dtype=np.float64)
    C = np.asarray(C, dtype=np.float64)
    nodes = np.asarray(bottom_nodes)
    nodes = nodes[np.argsort(xy[nodes, 0])]
    xw, cw = xy[nodes, 0], C[nodes]
    segs = [(k, k + 1) for k in range(len(nodes) - 1)]
    if period_x > 0:
        segs.append((len(nodes) - 1, 0))
    cuts = []
    for a, b in segs:
        if (cw[a] >= level) == (cw[b] >= level):
            continue
        xa, xb = xw[a], xw[b] + (period_x if b < a else 0.0)
        s = (level - cw[a]) / (cw[b] - cw[a])
        xc = xa + s * (xb - xa)
        if period_x > 0:
            xc %= period_x
        if x_window is None or x_window[0] <= xc <= x_window[1]:
            cuts.append(xc)
    if len(cuts) != 2:
        raise ValueError(f"contour crosses the wall {len(cuts)} times inside the window")
    x0, x1 = sorted(cuts)
    base = x1 - x0
    tri = np.asarray(tri)
    height = 0.0
    for p, q in ((0, 1), (1, 2), (2, 0)):
        i, j = tri[:, p], tri[:, q]
        ci, cj = C[i], C[j]
        cross = (ci >= level) != (cj >= level)
        i, j, ci, cj = i[cross], j[cross], ci[cross], cj[cross]
        s = (level - ci) / (cj - ci)
        y = xy[i, 1] + s * (xy[j, 1] - xy[i, 1])
        x = xy[i, 0]
        keep = (x >= x0 - 1.0) & (x <= x1 + 1.0)
        if np.any(keep):
            height = max(height, float(y[keep].max()))
    return float(np.degrees(2.0 * np.arctan2(2.0 * height, base))), height, base


def contour_points(xy, tri, C, period_x=0.0, level=0.5, x_center=None):
    """Points where the P1 interpolant of C crosses `level` on the element
    edges (one per crossing edge and element side), x unwrapped to the minimum
    image of x_center when the mesh is x-periodic."""
    xy = np.asarray(xy, dtype=np.float64)
    C = np.asarray(C, dtype=np.float64)
    tri = np.asarray(tri)
    pts = []
    for p, q in ((0, 1), (1, 2), (2, 0)):
        i, j = tri[:, p], tri[:, q]
        ci, cj = C[i], C[j]
        cross = (ci >= level) != (cj >= level)
        i, j, ci, cj = i[cross], j[cross], ci[cross], cj[cross]
        s = (level - ci) / (cj - ci)
        xi_, xj_ = xy[i, 0].copy(), xy[j, 0].copy()
        if period_x > 0:
            xj_ -= period_x * np.round((xj_ - xi_) / period_x)
        x = xi_ + s * (xj_ - xi_)
        y = xy[i, 1] + s * (xy[j, 1] - xy[i, 1])
        if period_x > 0 and x_center is not None:
            x -= period_x * np.round((x - x_center) / period_x)
        pts.append(np.stack([x, y], 1))
    pts = np.concatenate(pts)
    # an edge shared by two elements gives the same point twice
    return np.unique(np.round(pts, 12), axis=0)


def cap_fit_angle(xy, tri, C, period_x=0.0, level=0.5, x_window=None, y_min=0.0, y_wall=0.0):
    """Apparent contact angle (degrees) of a droplet from a circle fitted to its
    C = level contour, for walls where the height/base measurement does not
    apply (a rough wall: the contour's wall crossings sit on the roughness).

    The contour points with y > y_min (above the roughness) inside x_window =
    (x0, x1) are fitted by least squares with x^2 + y^2 + D x + E y + F = 0
    (algebraic circle fit); the angle is where that circle meets the mean wall
    line y = y_wall, measured inside the liquid: cos(theta) = -(y_c - y_wall)/r
    for centre (x_c, y_c) and radius r.  Returns (theta, x_c, y_c, r)."""
    xc_guess = None if x_window is None else 0.5 * (x_window[0] + x_window[1])
    pts = contour_points(xy, tri, C, period_x, level, xc_guess)
    sel = pts[:, 1] > y_min
    if x_window is not None:
        sel &= (pts[:, 0] >= x_window[0]) & (pts[:, 0] <= x_window[1])
    p = pts[sel]
    if p.shape[0] < 8:
        raise ValueError(f"only {p.shape[0]} contour points above y_min inside the window")
    x, y = p[:, 0], p[:, 1]
    A = np.stack([x, y, np.ones_like(x)], 1)
    D, E, F = np.linalg.lstsq(A, -(x * x + y * y), rcond=None)[0]
    xc, yc = -0.5 * D, -0.5 * E
    r = float(np.sqrt(xc * xc + yc * yc - F))
    cos_t = np.clip(-(yc - y_wall) / r, -1.0, 1.0)
    return float(np.degrees(np.arccos(cos_t))), float(xc), float(yc), r
