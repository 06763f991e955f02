"""GPU (HIP, through the C ABI) versus the FP64 CPU oracle, element by element.

Tolerances.  In FP64 both sides evaluate the same formulas in a different
order (gathers vs assembled sparse products, Chebyshev sweeps vs PCG), so
they differ by rounding (~1e-16 relative per operation, a few hundred
operations deep) plus the solver truncation: K = 32 Chebyshev sweeps on the
spectrum [1/4, 1] leave a relative error <= 2 * 3^-32 ~ 1e-15 in the
increment, and the oracle's PCG stops at 1e-13 relative residual (~1e-13 of
the increment, which is itself ~1e-2 of the populations).  One step is
therefore held to 1e-13 of max |psi|; the dissipative step does not amplify
differences, so 10 and 200 steps are held to 1e-12 and 1e-11.
"""
import numpy as np
import pytest

from gpu_common import log, make_ctx, rel, stack
from oracle import Oracle
from oracle import felbm_oracle as fo
from workloads import (channel_mesh, config, droplet_field, make_physics, split_grid_mesh, uniform_rows,
                       wetting_from_angles)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cfg1_theta60():
    w = config(1)
    om = wetting_from_angles(w.mesh, 60.0)
    o = Oracle(w.mesh, w.phys, om)
    return w, om, o


def test_fields_after_init_match_oracle(cfg1_theta60):
    w, om, o = cfg1_theta60
    log("fields after init, workload 1, theta 60, fp64")
    ctx = make_ctx(w.mesh, w.phys, om)
    ctx.init(w.C0)
    g, h = o.init_state(w.C0)
    assert rel(ctx.read_populations(), stack(g, h)) < 1e-15
    f = o.fields(g, h)
    assert rel(ctx.read("C"), f["C"]) < 1e-14
    assert rel(ctx.read("RHO"), f["rho"]) < 1e-14
    assert np.abs(ctx.read("P") - f["p"]).max() < 1e-16
    assert rel(ctx.read("LAPC"), f["lapC"]) < 1e-12
    assert rel(ctx.read("MU"), f["mu"]) < 1e-12
    assert rel(ctx.read("LAPMU"), f["lapmu"]) < 1e-11
    ctx.close()


def test_step_intermediates_match_oracle(cfg1_theta60):
    w, om, o = cfg1_theta60
    log("step intermediates after 5 steps, workload 1, fp64")
    ctx = make_ctx(w.mesh, w.phys, om)
    ctx.init(w.C0)
    ctx.step(5)
    g, h = o.init_state(w.C0)
    g, h = o.run(g, h, 5)
    hat, rhs, delta = ctx.step_debug()
    _, _, f = o.step(g, h, return_fields=True)
    assert rel(hat, stack(f["g_hat"], f["h_hat"])) < 1e-14
    m = o.mat.lumped
    b_over_m = stack(f["b_g"] / m[:, None], f["b_h"] / m[:, None])
    assert np.abs(rhs - b_over_m).max() < 1e-12 * np.abs(b_over_m).max()
    d_ref = stack(f["d_g"], f["d_h"])
    interior = ~o.geo.is_wall_node
    assert np.abs(delta[:, interior] - d_ref[:, interior]).max() < 1e-11 * np.abs(d_ref).max()
    ctx.close()


@pytest.mark.parametrize("steps,tol", [(1, 1e-13), (10, 1e-12), (200, 1e-11)])
def test_full_step_parity_fp64(cfg1_theta60, steps, tol):
    w, om, o = cfg1_theta60
    log(f"full-step parity, workload 1 (2112 nodes), theta 60, fp64, {steps} steps")
    ctx = make_ctx(w.mesh, w.phys, om)
    ctx.init(w.C0)
    ctx.step(steps)
    g, h = o.init_state(w.C0)
    g, h = o.run(g, h, steps)
    err = rel(ctx.read_populations(), stack(g, h))
    log(f"  max rel diff {err:.3e}")
    assert err < tol
    ctx.close()


def test_global_gather_kernels(cfg1_theta60):
    """The global-gather kernels (sliced-ELL sweep, node gather of the
    right-hand side from global memory), used for meshes whose tiles do not
    fit the LDS layout, against the oracle (FP64) and against the tiled
    kernels (FP32: same formulas, different summation order)."""
    w, om, o = cfg1_theta60
    log("global-gather kernels, workload 1, fp64 10 steps vs oracle")
    ctx = make_ctx(w.mesh, w.phys, om, kernels="global")
    ctx.init(w.C0)
    ctx.step(10)
    g, h = o.init_state(w.C0)
    g, h = o.run(g, h, 10)
    assert rel(ctx.read_populations(), stack(g, h)) < 1e-12
    ctx.close()
    log("global-gather kernels, fp32 200 steps vs the tiled kernels")
    outs = []
    for kern in ("global", "auto"):
        ctx = make_ctx(w.mesh, w.phys, om, precision="fp32", sweeps=16, kernels=kern)
        ctx.init(w.C0)
        m0 = ctx.diagnostics()["mass"]
        ctx.step(200)
        assert abs(ctx.diagnostics()["mass"] - m0) / m0 < 1e-10
        outs.append(ctx.read_populations())
        ctx.close()
    assert rel(outs[0], outs[1]) < 1e-5


def test_ragged_and_closed_meshes():
    # N not a multiple of 64, walls on all four sides, two droplets
    for periodic, nx, ny in ((True, 37, 13), (False, 29, 11)):
        log(f"ragged mesh parity periodic={periodic} {nx}x{ny}")
        mesh = split_grid_mesh(float(nx), uniform_rows(float(ny - 1), ny), nx, seed=[nx], periodic=periodic)
        phys = make_physics(sigma=0.01, m_rho=5.0, m_nu=2.0, dt=0.1)
        om = wetting_from_angles(mesh, 70.0, 110.0)
        C0 = droplet_field(mesh, [(nx / 3, 0.0, 4.0), (2 * nx / 3, ny - 1.0, 3.5)], phys.xi)
        ctx = make_ctx(mesh, phys, om)
        ctx.init(C0)
        ctx.step(7)
        o = Oracle(mesh, phys, om)
        g, h = o.init_state(C0)
        g, h = o.run(g, h, 7)
        assert mesh.n_nodes % 64 != 0
        assert rel(ctx.read_populations(), stack(g, h)) < 1e-12
        ctx.close()


def test_channel_mesh_with_internal_walls():
    """A mesh with two holes (solid blocks leaving a channel between them,
    40 x 16 box, 500 nodes): wall edges on the block faces and channel walls,
    wall nodes at re-entrant corners, wetting (theta = 60 deg) on the channel
    walls only, a liquid slab reaching into the channel.  FP64 against the
    oracle after 20 steps; FP32 precision form against the oracle on the
    populations and the mass."""
    mesh = channel_mesh(40.0, 16.0, 1.0, 12.0, 28.0, 6.0, 10.0, seed=[7])
    phys = make_physics(sigma=0.01, m_rho=10.0, m_nu=1.0, dt=0.1)
    om = np.zeros(mesh.n_nodes)
    om[mesh.wall_nodes(4)] = -0.5
    x = mesh.xy[:, 0]
    C0 = 0.5 + 0.5 * np.tanh(2.0 * np.minimum(x - 4.0, 16.0 - x) / phys.xi)
    o = Oracle(mesh, phys, om)
    g, h = o.init_state(C0)
    g, h = o.run(g, h, 20)
    ref = stack(g, h)
    for prec, sweeps, bar in (("fp64", 32, 1e-12), ("fp32", 16, 1e-5)):
        log(f"channel mesh with internal walls ({mesh.n_nodes} nodes), {prec}, 20 steps")
        ctx = make_ctx(mesh, phys, om, precision=prec, sweeps=sweeps)
        ctx.init(C0)
        m0 = ctx.diagnostics()["mass"]
        ctx.step(20)
        err = rel(ctx.read_populations(), ref)
        drift = abs(ctx.diagnostics()["mass"] - m0) / m0
        log(f"  max rel diff {err:.3e}  mass drift {drift:.2e}")
        assert err < bar
        assert drift < 1e-10
        ctx.close()


def test_degenerate_single_phase_states(cfg1_theta60):
    """Uniform composition, where every interface force vanishes: a pure
    liquid (C = 1) carrying a shear wave u_x = U sin(pi y / L_y) against the
    oracle after 20 steps (FP64 1e-12, FP32 1e-5), and a pure vapour (C = 0)
    at rest, which must stay at rest exactly (the equilibrium is a fixed point
    of collision and streaming, and the wall operator keeps it)."""
    w, om, o = cfg1_theta60
    y = w.mesh.xy[:, 1]
    Ly = y.max()
    u0 = np.zeros((w.mesh.n_nodes, 2))
    u0[:, 0] = 1e-3 * np.sin(np.pi * y / Ly)
    ones = np.ones(w.mesh.n_nodes)
    g, h = o.init_state(ones, u0)
    g, h = o.run(g, h, 20)
    ref = stack(g, h)
    for prec, sweeps, bar in (("fp64", 32, 1e-12), ("fp32", 16, 1e-5)):
        log(f"pure liquid with a shear wave, {prec}, 20 steps")
        ctx = make_ctx(w.mesh, w.phys, om, precision=prec, sweeps=sweeps)
        ctx.init(ones, u0)
        ctx.step(20)
        err = rel(ctx.read_populations(), ref)
        log(f"  max rel diff {err:.3e}")
        assert err < bar
        ctx.close()
        log(f"pure vapour at rest, {prec}, 20 steps")
        ctx = make_ctx(w.mesh, w.phys, om, precision=prec, sweeps=sweeps)
        ctx.init(np.zeros(w.mesh.n_nodes))
        ctx.step(20)
        d = ctx.diagnostics()
        log(f"  max|u| {d['max_u']:.3e}  mean KE {d['mean_ke']:.3e}")
        assert d["max_u"] == 0.0 and d["mean_ke"] == 0.0
        ctx.close()


@pytest.mark.parametrize("K", [0, 1, 2, 5])
def test_short_solver_polynomials(K):
    """K Chebyshev sweeps: the increment's error against the exact solve obeys
    the Chebyshev bound 2/T_K(5/3) relative to the lumped-solve error."""
    w = config(1)
    om = wetting_from_angles(w.mesh, 60.0)
    log(f"solver sweeps K={K}")
    ctx = make_ctx(w.mesh, w.phys, om, sweeps=K)
    ctx.init(w.C0)
    ctx.step(3)
    hat, rhs, delta = ctx.step_debug()
    o = Oracle(w.mesh, w.phys, om)
    m = o.mat.lumped
    interior = ~o.geo.is_wall_node
    bound = 1.0 / np.cosh(K * np.arccosh(5.0 / 3.0)) * 2.0
    for a in (0, 5, 9, 14):
        b = rhs[a] * m
        exact, _ = fo.pcg(o.mat.M11, m, b, tol=1e-15)
        e0 = rhs[a] - exact
        eK = delta[a] - exact
        # M11-weighted (energy) norms over interior nodes approximate the A-norm bound
        n0 = np.sqrt(np.sum(m[interior] * e0[interior] ** 2))
        nK = np.sqrt(np.sum(m[interior] * eK[interior] ** 2))
        assert nK <= 2.0 * bound * n0 + 1e-15 * np.abs(exact).max()
    ctx.close()


def test_mass_conserved_fp64_and_fp32():
    w = config(1)
    om = wetting_from_angles(w.mesh, 60.0)
    for prec, sweeps, bar in (("fp64", 32, 1e-13), ("fp32", 16, 1e-10)):
        log(f"mass conservation 200 steps {prec}")
        ctx = make_ctx(w.mesh, w.phys, om, precision=prec, sweeps=sweeps)
        ctx.init(w.C0)
        m0 = ctx.diagnostics()["mass"]
        ctx.step(200)
        m1 = ctx.diagnostics()["mass"]
        log(f"  drift {abs(m1 - m0) / m0:.3e}")
        assert abs(m1 - m0) / m0 < bar
        ctx.close()


def test_fp32_precision_form_vs_fp64_oracle(cfg1_theta60):
    """FP32 populations and arithmetic (FP64 mu chain, reductions and
    composition) against the FP64 oracle after 200 steps, on the bars the
    precision form is held to: spurious-current maximum within 5%, mass drift
    below 1e-10 relative; the populations themselves differ at FP32 rounding
    level (unit roundoff 6e-8, a few hundred operations per step)."""
    w, om, o = cfg1_theta60
    log("fp32 precision form vs fp64 oracle, workload 1, 200 steps")
    ctx = make_ctx(w.mesh, w.phys, om, precision="fp32", sweeps=16)
    ctx.init(w.C0)
    m0 = ctx.diagnostics()["mass"]
    ctx.step(200)
    d = ctx.diagnostics()
    g, h = o.init_state(w.C0)
    g, h = o.run(g, h, 200)
    r = o.diagnostics(g, h)
    pops = rel(ctx.read_populations(), stack(g, h))
    cerr = np.abs(ctx.read("C") - h.sum(1)).max()
    log(f"  pops rel {pops:.2e}  C abs {cerr:.2e}  max_u {d['max_u']:.6e} vs {r['max_u']:.6e}  "
        f"mass drift {abs(d['mass'] - m0) / m0:.2e}")
    assert pops < 1e-5
    assert cerr < 1e-5
    assert abs(d["max_u"] - r["max_u"]) / r["max_u"] < 0.05
    assert abs(d["mass"] - m0) / m0 < 1e-10
    assert abs(d["mass"] - r["mass"]) / r["mass"] < 1e-10
    ctx.close()


def test_deterministic_and_checkpoint_resume():
    w = config(1)
    om = wetting_from_angles(w.mesh, 60.0)
    for prec in ("fp64", "fp32"):
        log(f"determinism and save/load {prec}")
        a = make_ctx(w.mesh, w.phys, om, precision=prec, sweeps=16)
        a.init(w.C0)
        a.step(20)
        ref = a.read_populations()
        b = make_ctx(w.mesh, w.phys, om, precision=prec, sweeps=16)
        b.init(w.C0)
        b.step(10)
        blob = b.save_state()
        b.step(3)
        b.load_state(blob)
        b.step(10)
        assert np.array_equal(b.read_populations(), ref)
        assert b.diagnostics()["step"] == 20
        a.close()
        b.close()


def test_diagnostics_match_oracle(cfg1_theta60):
    w, om, o = cfg1_theta60
    log("diagnostics vs oracle")
    ctx = make_ctx(w.mesh, w.phys, om)
    ctx.set_band(32.0, 0.0, 12.0, 4.0)
    ctx.init(w.C0)
    ctx.step(20)
    g, h = o.init_state(w.C0)
    g, h = o.run(g, h, 20)
    d = ctx.diagnostics()
    r = o.diagnostics(g, h, band=(32.0, 0.0, 12.0, 4.0))
    assert abs(d["mass"] - r["mass"]) < 1e-12 * r["mass"]
    assert abs(d["mean_ke"] - r["mean_ke"]) < 1e-9 * r["mean_ke"]
    assert abs(d["max_u"] - r["max_u"]) < 1e-9 * r["max_u"]
    assert abs(d["band_ke"] - r["band_ke"]) < 1e-9 * r["band_ke"]
    hist = ctx.history()
    assert [x["step"] for x in hist] == list(range(20))
    ctx.close()


def test_nonfinite_state_is_reported():
    w = config(1)
    log("non-finite detection")
    ctx = make_ctx(w.mesh, w.phys, w.omega_c)
    ctx.init(w.C0)
    blob = bytearray(ctx.save_state())
    # header is 40 bytes; poison one population value of internal node 100 (fp64)
    off = 40 + 8 * 100
    blob[off:off + 8] = np.array([np.nan]).tobytes()
    ctx.load_state(bytes(blob))
    import paper_1708_04678_amd as felbm
    with pytest.raises(felbm.FelbmError) as ei:
        ctx.step(2)
    assert ei.value.name == "ENONFINITE"
    ctx.close()


def test_api_state_errors():
    import paper_1708_04678_amd as felbm
    w = config(1)
    ctx = felbm.Context(sigma=0.01, xi=4.0, mobility=0.02, rho_l=1.0, rho_v=0.1, nu_l=0.1 / 3, nu_v=0.1 / 3, dt=0.1)
    with pytest.raises(felbm.FelbmError) as ei:
        ctx.step(1)
    assert ei.value.name == "ESTATE"
    ctx.upload_mesh(w.mesh.xy, w.mesh.tri, w.mesh.wall_edges, w.mesh.period_x)
    with pytest.raises(felbm.FelbmError):
        ctx.upload_mesh(w.mesh.xy, w.mesh.tri, w.mesh.wall_edges, w.mesh.period_x)
    with pytest.raises(felbm.FelbmError) as ei:
        ctx.read("C")
    assert ei.value.name == "ESTATE"
    bad = w.C0.copy()
    bad[3] = np.inf
    with pytest.raises(felbm.FelbmError) as ei:
        ctx.init(bad)
    assert ei.value.name == "EINVAL"
    ctx.close()


@pytest.mark.parametrize("prec,kernels", [("fp64", "auto"), ("fp32", "auto"), ("fp32", "global")])
def test_residual_sampling_is_bitwise_neutral_and_bounded(cfg1_theta60, prec, kernels):
    """A step whose solve residual is sampled gives bitwise the same state as an
    unsampled one, and the sampled relative residual ||A x_K - f||_m / ||f||_m
    obeys the Chebyshev bound (3/4) / T_K(5/3) of the K-sweep iterate from
    x_0 = f on the spectrum [1/4, 1] (A = diag(m)^-1 M11 is self-adjoint in the
    m inner product), up to the working precision's rounding floor."""
    w, om, _ = cfg1_theta60
    floor = 1e-13 if prec == "fp64" else 2e-6
    for K in (0, 1, 2, 5, 11):
        log(f"residual sampling {prec} {kernels} K={K}")
        outs = []
        for every in (0, 1):
            ctx = make_ctx(w.mesh, w.phys, om, precision=prec, sweeps=K, kernels=kernels)
            ctx.set_residual_sampling(every)
            ctx.init(w.C0)
            ctx.step(4)
            d = ctx.diagnostics()
            outs.append((ctx.read_populations(), ctx.read("C"), d))
            ctx.close()
        assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])
        d0, d1 = outs[0][2], outs[1][2]
        assert d0["solver_residual"] == -1.0 and d0["residual_step"] == -1 and d0["solver_sweeps"] == K
        res = d1["solver_residual"]
        bound = 0.75 / np.cosh(K * np.log(3.0))
        log(f"  residual {res:.3e} bound {bound:.3e} (step {d1['residual_step']})")
        assert d1["residual_step"] == 3
        assert 0.0 < res <= 1.001 * bound + floor


def test_residual_at_full_sweep_counts():
    """At the bench's sweep counts the sampled residual reaches the rounding
    floor of each precision (K = 26 in FP64, K = 11 in FP32 at the Chebyshev
    bound 2e-6)."""
    w = config(2)
    om = wetting_from_angles(w.mesh, 60.0)
    for prec, K, bar in (("fp64", 26, 1e-12), ("fp32", 11, 2e-5)):
        log(f"residual at K={K} {prec}, workload 2")
        ctx = make_ctx(w.mesh, w.phys, om, precision=prec, sweeps=K)
        ctx.set_residual_sampling(5)
        ctx.init(w.C0)
        ctx.step(11)
        d = ctx.diagnostics()
        log(f"  residual {d['solver_residual']:.3e} at step {d['residual_step']}")
        assert d["residual_step"] == 10 and 0.0 < d["solver_residual"] < bar
        ctx.close()
