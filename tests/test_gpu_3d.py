"""The 3-D library (D3Q19 on linear tetrahedra, include/felbm3d.h) on the GPU
against the 3-D CPU oracle, element by element on the same seeded inputs.

Bars as for the 2-D path: FP64 with K = 40 Chebyshev-step sweeps (the
Richardson error factor on [1/5, 1] after 40 sweeps is below 1e-15) against the
oracle's PCG to 1e-13; FP32 populations within 1e-5 of the largest after 10
steps (single-precision rounding at depth 10 x 40 sweeps)."""
import numpy as np
import pytest

import paper_1708_04678_amd as felbm
from gpu_common import log, rel
from oracle import felbm3d_oracle as fo3
from workloads import make_physics
from workloads.mesh3d import droplet_field_3d, tet_box_mesh, wetting_from_angles_3d

pytestmark = pytest.mark.gpu

FIELD_NAMES = ("C", "RHO", "P", "UX", "UY", "UZ", "MU", "LAPC", "LAPMU")


def make_ctx3(mesh, phys, omega_c, precision="fp64", sweeps=40):
    ctx = felbm.Context3D(sigma=phys.sigma, xi=phys.xi, mobility=phys.mobility, rho_l=phys.rho_l,
                          rho_v=phys.rho_v, nu_l=phys.nu_l, nu_v=phys.nu_v, dt=phys.dt, precision=precision,
                          solver_sweeps=sweeps)
    ctx.upload_mesh(mesh.xyz, mesh.tet, mesh.wall_faces, mesh.period)
    ctx.set_wetting(omega_c)
    return ctx


def stack3(g, h):
    """Oracle (N, 19) g and h -> library layout (38, N)."""
    return np.concatenate([np.asarray(g).T, np.asarray(h).T], axis=0)


def oracle_fields(o, g, h):
    f = o.fields(g, h)
    return {"C": f["C"], "RHO": f["rho"], "P": f["p"], "UX": f["u"][:, 0], "UY": f["u"][:, 1], "UZ": f["u"][:, 2],
            "MU": f["mu"], "LAPC": f["lapC"], "LAPMU": f["lapmu"]}


def sessile_case(nx=20, ny=16, nz=10, seed=5, theta=60.0, m_rho=10.0, z_rows=None, jitter=0.2):
    """A hemispherical drop on the bottom wall of a jittered periodic box
    (walls at z = 0 and z = nz); 3520 nodes and 19200 tetrahedra by default,
    so every kernel runs several blocks and a ragged last block."""
    mesh = tet_box_mesh(float(nx), float(ny), float(nz), nx, ny, nz, seed=[seed], jitter=jitter, z_rows=z_rows)
    phys = make_physics(sigma=0.01, m_rho=m_rho, m_nu=2.0, dt=0.1, xi=2.0)
    om = wetting_from_angles_3d(mesh, theta, 180.0 - theta)
    C0 = droplet_field_3d(mesh, [(0.45 * nx, 0.5 * ny, 0.0, 0.3 * min(nx, ny))], phys.xi)
    return mesh, phys, om, C0


def test_init_and_fields_match_oracle():
    mesh, phys, om, C0 = sessile_case()
    rng = np.random.default_rng(11)
    u0 = 0.01 * rng.standard_normal((mesh.n_nodes, 3))
    u0[mesh.wall_nodes()] = 0.0
    p0 = 1e-3 * rng.standard_normal(mesh.n_nodes)
    log(f"3-D init and fields, {mesh.n_nodes} nodes, {mesh.n_tets} tets, fp64")
    ctx = make_ctx3(mesh, phys, om)
    info = ctx.mesh_info()
    assert info["n_nodes"] == mesh.n_nodes and info["n_tets"] == mesh.n_tets
    assert info["n_wall_faces"] == len(mesh.wall_faces)
    ctx.init(C0, u0, p0)
    o = fo3.Oracle3D(mesh, phys, om)
    g, h = o.init_state(C0, u0, p0)
    assert rel(ctx.read_populations(), stack3(g, h)) < 1e-15
    ref = oracle_fields(o, g, h)
    for name in FIELD_NAMES:
        err = rel(ctx.read(name), ref[name])
        log(f"  {name}: max rel diff {err:.3e}")
        assert err < 1e-13, name
    ctx.close()


@pytest.mark.parametrize("steps,tol", [(1, 1e-13), (10, 1e-12)])
def test_steps_match_oracle_fp64(steps, tol):
    mesh, phys, om, C0 = sessile_case()
    log(f"3-D fp64, {steps} steps vs oracle")
    ctx = make_ctx3(mesh, phys, om)
    ctx.init(C0)
    ctx.step(steps)
    o = fo3.Oracle3D(mesh, phys, om)
    g, h = o.init_state(C0)
    g, h = o.run(g, h, steps)
    err = rel(ctx.read_populations(), stack3(g, h))
    log(f"  populations max rel diff {err:.3e}")
    assert err < tol
    ref = oracle_fields(o, g, h)
    for name in FIELD_NAMES:
        scale = max(np.abs(ref[name]).max(), 1e-300)
        err = float(np.abs(ctx.read(name) - ref[name]).max() / scale)
        assert err < 100 * tol, (name, err)
    d, od = ctx.diagnostics(), o.diagnostics(g, h)
    assert d["step"] == steps and d["nonfinite"] == 0 and d["solver_sweeps"] == 40
    for k in ("mass", "mean_ke", "max_u"):
        assert abs(d[k] - od[k]) <= 1e-12 * abs(od[k]) + 1e-300, k
    ctx.close()


def test_graded_closed_mesh_and_contrast_100():
    """Graded z layers (thin near the walls), larger jitter, density ratio
    100, contact angles 45 and 135 degrees: 5 steps against the oracle."""
    nz = 8
    s = np.linspace(0.0, 1.0, nz + 1)
    z_rows = 8.0 * (s - 0.15 * np.sin(2 * np.pi * s) / (2 * np.pi))
    mesh, phys, om, C0 = sessile_case(nx=13, ny=11, nz=nz, seed=9, theta=45.0, m_rho=100.0, z_rows=z_rows,
                                      jitter=0.25)
    log(f"3-D fp64 graded mesh, M_rho 100, {mesh.n_nodes} nodes, 5 steps")
    ctx = make_ctx3(mesh, phys, om)
    ctx.init(C0)
    ctx.step(5)
    o = fo3.Oracle3D(mesh, phys, om)
    g, h = o.init_state(C0)
    g, h = o.run(g, h, 5)
    err = rel(ctx.read_populations(), stack3(g, h))
    log(f"  populations max rel diff {err:.3e}")
    assert err < 1e-12
    ctx.close()


def test_fp32_against_fp64_oracle():
    mesh, phys, om, C0 = sessile_case()
    log("3-D fp32 10 steps vs fp64 oracle")
    ctx = make_ctx3(mesh, phys, om, precision="fp32", sweeps=16)
    ctx.init(C0)
    o = fo3.Oracle3D(mesh, phys, om)
    g, h = o.init_state(C0)
    assert rel(ctx.read_populations(), stack3(g, h)) < 1e-6
    ctx.step(10)
    g, h = o.run(g, h, 10)
    err = rel(ctx.read_populations(), stack3(g, h))
    log(f"  populations max rel diff {err:.3e}")
    assert err < 1e-5
    C_err = float(np.abs(ctx.read("C") - fo3.moments(g, h, o.prm)[0]).max())
    log(f"  C max abs diff {C_err:.3e}")
    assert C_err < 1e-5
    ctx.close()


def test_mass_conserved_over_200_steps():
    """The collision keeps sum_a h_a, the Richardson sweeps keep the lumped
    mass of the right-hand side at every sweep and the streaming term sums
    to zero over each element: the lumped mass of C stays at its initial
    value up to rounding.  FP64: 1e-13.  FP32: the composition is carried in
    FP64 beside the float populations (C = sum h + r) and its increment keeps
    the mass to FP64 rounding: 1e-12 over 200 steps."""
    mesh, phys, om, C0 = sessile_case()
    for prec, sweeps, bar in (("fp64", 40, 1e-13), ("fp32", 16, 1e-12)):
        log(f"3-D mass over 200 steps, {prec}")
        ctx = make_ctx3(mesh, phys, om, precision=prec, sweeps=sweeps)
        ctx.init(C0)
        m0 = ctx.diagnostics()["mass"]
        ctx.step(200)
        d = ctx.diagnostics()
        drift = abs(d["mass"] - m0) / m0
        log(f"  relative drift {drift:.3e}, max|u| {d['max_u']:.3e}")
        assert d["nonfinite"] == 0
        assert drift < bar
        ctx.close()


def test_rejects_bad_input():
    mesh, phys, om, C0 = sessile_case(nx=6, ny=6, nz=4)
    ctx = felbm.Context3D(sigma=phys.sigma, xi=phys.xi, mobility=phys.mobility, rho_l=phys.rho_l,
                          rho_v=phys.rho_v, nu_l=phys.nu_l, nu_v=phys.nu_v, dt=phys.dt)
    with pytest.raises(felbm.FelbmError):
        ctx.step(1)  # no mesh yet
    with pytest.raises(felbm.FelbmError):
        ctx.upload_mesh(mesh.xyz, mesh.tet, mesh.wall_faces[1:], mesh.period)  # a boundary face unlisted
    bad = mesh.tet.copy()
    bad[0, [2, 3]] = bad[0, [3, 2]]
    with pytest.raises(felbm.FelbmError):
        ctx.upload_mesh(mesh.xyz, bad, mesh.wall_faces, mesh.period)  # negative volume
    ctx.upload_mesh(mesh.xyz, mesh.tet, mesh.wall_faces, mesh.period)
    with pytest.raises(felbm.FelbmError):
        ctx.upload_mesh(mesh.xyz, mesh.tet, mesh.wall_faces, mesh.period)  # second upload
    ctx.set_wetting(om)
    ctx.init(C0)
    ctx.step(0)
    assert ctx.diagnostics()["step"] == 0
    with pytest.raises(felbm.FelbmError):
        ctx.read(99)
    ctx.close()
