"""Losses of the adjoint workloads, as functions of the composition field
(numpy; shared by the GPU tests and the scripts that write stored reference
values).  No FE-LBM arithmetic here."""
import numpy as np


def wetted_centroid_loss(mesh, m, C):
    """Loss of the 256 x 128 adjoint workload: the droplet centroid x plus the
    wetted length squared, x_c + L_w^2 with x_c = sum m x C / sum m C and
    L_w = int_bottom C ds (trapezoid on the bottom wall edges).  Returns L and
    dL/dC.  Works for complex C (complex-step derivatives)."""
    x = mesh.xy[:, 0]
    M0, M1 = np.sum(m * C), np.sum(m * x * C)
    xc = M1 / M0
    we = mesh.wall_edges[mesh.wall_side == 0]
    dx = mesh.xy[we[:, 1], 0] - mesh.xy[we[:, 0], 0]
    dx -= mesh.period_x * np.round(dx / mesh.period_x)
    L_w = np.sum(np.abs(dx) * 0.5 * (C[we[:, 0]] + C[we[:, 1]]))
    dL = m * x / M0 - M1 * m / M0 ** 2
    dLw = np.zeros(C.shape, dtype=C.dtype)
    np.add.at(dLw, we[:, 0], 0.5 * np.abs(dx))
    np.add.at(dLw, we[:, 1], 0.5 * np.abs(dx))
    return xc + L_w ** 2, dL + 2.0 * L_w * dLw


def adjoint_probe_nodes(mesh):
    """The 8 seeded bottom-wall nodes at which the 256 x 128 adjoint workload's
    gradient is checked."""
    bottom = mesh.wall_nodes(0)
    return np.random.default_rng([4, 5]).choice(bottom, 8, replace=False)
