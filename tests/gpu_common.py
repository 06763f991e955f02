"""Shared helpers of the GPU tests: build a library context from a workload
and lay oracle arrays out like the library's [18][N] populations."""
import sys

import numpy as np

import paper_1708_04678_amd as felbm


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def make_ctx(mesh, phys, omega_c, precision="fp64", sweeps=32, **extra):
    ctx = felbm.Context(sigma=phys.sigma, xi=phys.xi, mobility=phys.mobility, rho_l=phys.rho_l, rho_v=phys.rho_v,
                        nu_l=phys.nu_l, nu_v=phys.nu_v, dt=phys.dt, precision=precision, solver_sweeps=sweeps, **extra)
    ctx.upload_mesh(mesh.xy, mesh.tri, mesh.wall_edges, mesh.period_x)
    ctx.set_wetting(omega_c)
    return ctx


def stack(g, h):
    """Oracle (N, 9) g and h -> library layout (18, N)."""
    return np.concatenate([np.asarray(g).T, np.asarray(h).T], axis=0)


def rel(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / max(np.abs(np.asarray(b)).max(), 1e-300))
