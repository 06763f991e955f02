"""The nodal-force comparison scheme (P1 forces, readings N1-N4 of the
oracle) on the GPU, FP64, against the oracle's nodal scheme element by
element; tolerances as for the mixed scheme (same solver truncation and
rounding depth)."""
import pytest

from gpu_common import log, make_ctx, rel, stack
from oracle import Oracle
from workloads import config, droplet_field, make_physics, split_grid_mesh, uniform_rows, wetting_from_angles

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("steps,tol", [(1, 1e-13), (10, 1e-12)])
def test_nodal_scheme_matches_oracle(steps, tol):
    w = config(1)
    om = wetting_from_angles(w.mesh, 60.0)
    log(f"nodal force scheme, workload 1, fp64, {steps} steps")
    ctx = make_ctx(w.mesh, w.phys, om, force_scheme="nodal")
    ctx.init(w.C0)
    ctx.step(steps)
    o = Oracle(w.mesh, w.phys, om, force_scheme="nodal")
    g, h = o.init_state(w.C0)
    g, h = o.run(g, h, steps)
    err = rel(ctx.read_populations(), stack(g, h))
    log(f"  max rel diff {err:.3e}")
    assert err < tol
    ctx.close()


def test_nodal_scheme_ragged_walls_and_mass():
    mesh = split_grid_mesh(29.0, uniform_rows(10.0, 11), 29, seed=[29], periodic=False)
    phys = make_physics(sigma=0.01, m_rho=5.0, m_nu=2.0, dt=0.1)
    om = wetting_from_angles(mesh, 70.0, 110.0)
    C0 = droplet_field(mesh, [(10.0, 0.0, 4.0)], phys.xi)
    log("nodal force scheme, closed ragged mesh, 7 steps and 100-step mass")
    ctx = make_ctx(mesh, phys, om, force_scheme="nodal")
    ctx.init(C0)
    m0 = ctx.diagnostics()["mass"]
    ctx.step(7)
    o = Oracle(mesh, phys, om, force_scheme="nodal")
    g, h = o.init_state(C0)
    g, h = o.run(g, h, 7)
    assert rel(ctx.read_populations(), stack(g, h)) < 1e-12
    ctx.step(93)
    assert abs(ctx.diagnostics()["mass"] - m0) / m0 < 1e-13
    ctx.close()


def test_nodal_scheme_rejects_adjoint():
    import paper_1708_04678_amd as felbm
    w = config(1)
    ctx = make_ctx(w.mesh, w.phys, wetting_from_angles(w.mesh, 90.0), force_scheme="nodal")
    ctx.init(w.C0)
    with pytest.raises(felbm.FelbmError):
        ctx.forward_ckpt(4, 2)
    ctx.close()


# ---------------------------------------------------------------------------
# nodal forces integrated in the collision step (readings NC1-NC5)
# ---------------------------------------------------------------------------
def test_collision_step_scheme_initial_state_matches_oracle():
    """psi_bar^0 = psi_eq - dt/2 F from the given fields (NC5), with a nonzero
    initial velocity and pressure."""
    import numpy as np
    w = config(1)
    om = wetting_from_angles(w.mesh, 60.0)
    rng = np.random.default_rng(3)
    u = rng.normal(0, 1e-3, (w.mesh.n_nodes, 2))
    p = rng.normal(0, 1e-4, w.mesh.n_nodes)
    log("collision-step nodal scheme: initial state, workload 1")
    ctx = make_ctx(w.mesh, w.phys, om, force_scheme="nodal_collide")
    ctx.init(w.C0, u=u, p=p)
    o = Oracle(w.mesh, w.phys, om, force_scheme="nodal_collide")
    g, h = o.init_state(w.C0, u=u, p=p)
    err = rel(ctx.read_populations(), stack(g, h))
    log(f"  max rel diff {err:.3e}")
    assert err < 1e-14
    ctx.close()


@pytest.mark.parametrize("steps,tol", [(1, 1e-13), (10, 1e-12), (100, 1e-11)])
def test_collision_step_scheme_matches_oracle(steps, tol):
    import numpy as np
    w = config(1)
    om = wetting_from_angles(w.mesh, 60.0)
    log(f"collision-step nodal scheme, workload 1, fp64, {steps} steps")
    ctx = make_ctx(w.mesh, w.phys, om, force_scheme="nodal_collide")
    ctx.set_band(32.0, 0.0, 12.0, 4.0)
    ctx.init(w.C0)
    ctx.step(steps)
    o = Oracle(w.mesh, w.phys, om, force_scheme="nodal_collide")
    g, h = o.init_state(w.C0)
    g, h = o.run(g, h, steps)
    err = rel(ctx.read_populations(), stack(g, h))
    log(f"  populations max rel diff {err:.3e}")
    assert err < tol
    # fields with the half-force moments (NC3) and the reductions of them
    f = o.fields(g, h)
    assert rel(ctx.read("UX"), f["u"][:, 0]) < 100 * tol
    assert rel(ctx.read("P"), f["p"]) < 100 * tol
    assert rel(ctx.read("MU"), f["mu"]) < 100 * tol
    d, dref = ctx.diagnostics(), o.diagnostics(g, h, band=(32.0, 0.0, 12.0, 4.0))
    log(f"  max|u| {d['max_u']:.6e} / {dref['max_u']:.6e}, band KE {d['band_ke']:.6e} / {dref['band_ke']:.6e}")
    assert abs(d["max_u"] - dref["max_u"]) <= 100 * tol * dref["max_u"]
    assert abs(d["band_ke"] - dref["band_ke"]) <= 100 * tol * dref["band_ke"]
    assert abs(d["mass"] - dref["mass"]) <= 1e-13 * dref["mass"]
    ctx.close()


def test_collision_step_scheme_ragged_walls_and_mass():
    mesh = split_grid_mesh(29.0, uniform_rows(10.0, 11), 29, seed=[29], periodic=False)
    phys = make_physics(sigma=0.01, m_rho=5.0, m_nu=2.0, dt=0.1)
    om = wetting_from_angles(mesh, 70.0, 110.0)
    C0 = droplet_field(mesh, [(10.0, 0.0, 4.0)], phys.xi)
    log("collision-step nodal scheme, closed ragged mesh, 7 steps and 100-step mass")
    ctx = make_ctx(mesh, phys, om, force_scheme="nodal_collide")
    ctx.init(C0)
    m0 = ctx.diagnostics()["mass"]
    ctx.step(7)
    o = Oracle(mesh, phys, om, force_scheme="nodal_collide")
    g, h = o.init_state(C0)
    g, h = o.run(g, h, 7)
    assert rel(ctx.read_populations(), stack(g, h)) < 1e-12
    ctx.step(93)
    assert abs(ctx.diagnostics()["mass"] - m0) / m0 < 1e-13
    ctx.close()


def test_collision_step_scheme_rejects_adjoint_and_noalloc():
    import paper_1708_04678_amd as felbm
    w = config(1)
    ctx = make_ctx(w.mesh, w.phys, wetting_from_angles(w.mesh, 90.0), force_scheme="nodal_collide")
    ctx.init(w.C0)
    with pytest.raises(felbm.FelbmError):
        ctx.forward_ckpt(4, 2)
    with pytest.raises(felbm.FelbmError):
        ctx.diagnostics_noalloc()
    ctx.close()
