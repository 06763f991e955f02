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
