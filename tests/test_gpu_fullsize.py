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


def test_fp32_vs_fp64_at_the_workload_horizon():
    """The precision form at the workload's stated 2,000 steps: FP32 (K = 11)
    and FP64 (K = 26) from the same initial state.  Bars from the precision
    form's targets: max|u| (the spurious-current magnitude) within 5 %, each
    droplet's apparent contact angle (circle fit above the roughness against
    the mean wall line) within 0.5 deg, relative mass drift below 1e-10 in
    both; the band KE of the first droplet is reported."""
    from paper_1708_04678_amd.analysis import cap_fit_angle
    w = config(3)
    res = {}
    for prec, K in (("fp32", 11), ("fp64", 26)):
        log(f"workload horizon: {w.steps} steps, {prec}, K = {K}")
        ctx = make_ctx(w.mesh, w.phys, w.omega_c, precision=prec, sweeps=K)
        xc, yc, R = w.droplets[0]
        ctx.set_band(xc, yc, R, w.phys.xi)
        ctx.init(w.C0)
        m0 = ctx.diagnostics()["mass"]
        ctx.step(w.steps)
        d = ctx.diagnostics()
        C = ctx.read("C")
        ang = [cap_fit_angle(w.mesh.xy, w.mesh.tri, C, w.mesh.period_x, x_window=(x - 2 * r, x + 2 * r), y_min=10.0)[0]
               for (x, _, r) in w.droplets]
        drift = abs(d["mass"] - m0) / m0
        log(f"  max|u| {d['max_u']:.6e}  band KE {d['band_ke']:.6e}  mass drift {drift:.2e}  angles "
            + ", ".join(f"{a:.4f}" for a in ang))
        assert drift < 1e-10
        res[prec] = (d, ang)
        ctx.close()
    (d32, a32), (d64, a64) = res["fp32"], res["fp64"]
    assert abs(d32["max_u"] - d64["max_u"]) <= 0.05 * d64["max_u"]
    assert max(abs(a - b) for a, b in zip(a32, a64)) < 0.5
    log(f"  max|u| rel diff {abs(d32['max_u'] - d64['max_u']) / d64['max_u']:.2e}, band KE rel diff "
        f"{abs(d32['band_ke'] - d64['band_ke']) / d64['band_ke']:.2e}")


@pytest.fixture(scope="module")
def sessile3d():
    from workloads.mesh3d import sessile_drop_3d
    return sessile_drop_3d()


def test_3d_full_size_fields_match_oracle(sessile3d):
    """The 3-D droplet at the paper's mesh size (1,490,944 nodes, 8,847,360
    tetrahedra, layers refined toward the wall), FP64: every field of the
    initial state (moments, the patch Laplacian of C with the wetting flux,
    mu, the element Laplacian of mu) against the oracle's field chain on the
    whole mesh (geometry only; its assembled matrices at this size need
    30 GB), to 1e-13 of each field's largest value."""
    from oracle import felbm3d_oracle as fo3
    from test_gpu_3d import FIELD_NAMES, make_ctx3, oracle_fields
    name, mesh, phys, C0, om, _ = sessile3d
    log(f"3-D full size {name}: {mesh.n_nodes} nodes, {mesh.n_tets} tets; oracle fields")
    o = fo3.Oracle3D(mesh, phys, om, with_matrices=False)
    g, h = o.init_state(C0)
    ref = oracle_fields(o, g, h)
    ctx = make_ctx3(mesh, phys, om, sweeps=30)
    ctx.init(C0)
    for fname in FIELD_NAMES:
        err = rel(ctx.read(fname), ref[fname])
        log(f"  {fname}: max rel diff {err:.3e}")
        assert err < 1e-13, fname
    ctx.close()


@pytest.mark.parametrize("precision,sweeps,bar", [("fp64", 30, 1e-12), ("fp32", 13, 1e-10)])
def test_3d_full_size_mass_and_determinism(sessile3d, precision, sweeps, bar):
    """100 steps of the 3-D droplet at full size in the benchmark's launch
    configuration: the lumped mass of C stays to rounding (FP32: the FP64
    composition transport, bar 1e-10), the state stays finite with no
    velocity at wall nodes, and two runs agree bitwise."""
    from test_gpu_3d import make_ctx3
    name, mesh, phys, C0, om, _ = sessile3d
    log(f"3-D full size, 100 steps, {precision} K = {sweeps}: mass and bitwise repeat")
    runs = []
    walls = mesh.wall_nodes()
    for _ in range(2):
        ctx = make_ctx3(mesh, phys, om, precision=precision, sweeps=sweeps)
        ctx.init(C0)
        m0 = ctx.diagnostics()["mass"]
        ctx.step(100)
        d = ctx.diagnostics()
        drift = abs(d["mass"] - m0) / m0
        log(f"  mass drift {drift:.3e}  max|u| {d['max_u']:.6e}")
        assert drift < bar and d["nonfinite"] == 0
        for comp in ("UX", "UY", "UZ"):
            assert np.abs(ctx.read(comp)[walls]).max() < 1e-6 * max(d["max_u"], 1e-30)
        runs.append(ctx.read_populations())
        ctx.close()
    assert np.array_equal(runs[0], runs[1])
