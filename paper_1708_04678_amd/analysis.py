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
