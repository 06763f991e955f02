"""Parity at the full size of the three-droplet workload (2,140,160 nodes,
4,276,224 triangles, graded rough wall, density ratio 1000), in the launch
configuration the benchmark times: one step of the GPU path, FP64 with 26
sweeps and FP32 with 11, against one step of the FP64 oracle (assembled
matrices, PCG to 1e-13) on the same mesh and initial state, every output
compared.  The oracle needs about a minute and 10 GB of host memory here.

Tolerances.  FP64: 26 Chebyshev sweeps on [1/4, 1] leave at most
2 * 3^-26 ~ 8e-13 of the increment, which is a small fraction of the
populations, plus rounding; held to 1e-12 of max |psi|.  FP32: unit roundoff
6e-8 over a few hundred operations plus the 12-sweep truncation
2 * 3^-12 ~ 4e-6 of the increment; held to 1e-5 of max |psi|, and the FP64
composition C to 1e-6 absolute.  Over 200 steps at this size both precisions
keep the total mass to 1e-10 relative and repeat bitwise.
"""
import numpy as np
import pytest

from gpu_common import log, make_ctx, rel, stack
from oracle import Oracle
from workloads import config

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def full_ref():
    w = config(3)
    log(f"full-size workload: {w.mesh.n_nodes} nodes, {w.mesh.n_tris} triangles; oracle step (about a minute)")
    o = Oracle(w.mesh, w.phys, w.omega_c)
    g, h = o.init_state(w.C0)
    g1, h1 = o.step(g, h)
    return w, stack(g1, h1), h1.sum(1)


@pytest.mark.parametrize("precision,sweeps,tol_pop,tol_C", [("fp64", 26, 1e-12, 1e-12), ("fp32", 11, 1e-5, 1e-6)])
def test_full_size_one_step_matches_oracle(full_ref, precision, sweeps, tol_pop, tol_C):
    w, P1, C1 = full_ref
    log(f"full-size one step, {precision}, {sweeps} sweeps")
    ctx = make_ctx(w.mesh, w.phys, w.omega_c, precision=precision, sweeps=sweeps)
    ctx.init(w.C0)
    ctx.step(1)
    pops = rel(ctx.read_populations(), P1)
    cerr = float(np.abs(ctx.read("C") - C1).max())
    log(f"  pops rel {pops:.3e}  C abs {cerr:.3e}")
    assert pops < tol_pop
    assert cerr < tol_C
    ctx.close()


@pytest.mark.parametrize("precision,sweeps", [("fp64", 26), ("fp32", 11)])
def test_full_size_mass_and_determinism(precision, sweeps):
    w = config(3)
    log(f"full-size 200 steps, {precision}: mass drift and bitwise repeat")
    runs = []
    for _ in range(2):
        ctx = make_ctx(w.mesh, w.phys, w.omega_c, precision=precision, sweeps=sweeps)
        ctx.init(w.C0)
        m0 = ctx.diagnostics()["mass"]
        ctx.step(200)
        d = ctx.diagnostics()
        runs.append(ctx.read_populations())
        log(f"  mass drift {abs(d['mass'] - m0) / m0:.3e}  max|u| {d['max_u']:.6e}")
        assert abs(d["mass"] - m0) / m0 < 1e-10
        assert np.isfinite(runs[-1]).all()
        ctx.close()
    assert np.array_equal(runs[0], runs[1])
