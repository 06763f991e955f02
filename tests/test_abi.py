"""C ABI checks that need no GPU: the library loads, exports every symbol
include/felbm.h declares, and its host-side validation rejects bad input."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_1708_04678_amd as felbm
from workloads import capillary_channel, channel_mesh, split_grid_mesh, uniform_rows

INCLUDE = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")


def declared_functions():
    """Every function any header under include/ declares."""
    names = set()
    for h in sorted(os.listdir(INCLUDE)):
        if not h.endswith(".h"):
            continue
        text = re.sub(r"/\*.*?\*/", "", open(os.path.join(INCLUDE, h)).read(), flags=re.S)
        names |= set(re.findall(r"\b(felbm(?:3d)?_[a-z_0-9]+)\s*\(", text))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    lib = felbm.load_library()
    names = declared_functions()
    assert len(names) >= 35
    assert any(n.startswith("felbm3d_") for n in names)
    for n in names:
        assert hasattr(lib, n), n
        assert isinstance(getattr(lib, n), ctypes._CFuncPtr)


def test_binding_covers_every_declared_symbol():
    from paper_1708_04678_amd.felbm import _SIGNATURES
    assert set(declared_functions()) <= set(_SIGNATURES)


def _mesh():
    return split_grid_mesh(8.0, uniform_rows(4.0, 5), 8, seed=[1])


def test_validate_accepts_generated_meshes():
    m = _mesh()
    assert felbm.validate_mesh(m.xy, m.tri, m.wall_edges, m.period_x)[0] == 0
    closed = split_grid_mesh(8.0, uniform_rows(4.0, 5), 8, seed=[1], periodic=False)
    assert felbm.validate_mesh(closed.xy, closed.tri, closed.wall_edges, 0.0)[0] == 0


def test_validate_accepts_channel_meshes():
    """Meshes with holes: every boundary edge a wall edge, straight walls,
    at most two wall edges per node, wall sides classified."""
    m = channel_mesh(40.0, 16.0, 1.0, 12.0, 28.0, 6.0, 10.0, seed=[7])
    assert felbm.validate_mesh(m.xy, m.tri, m.wall_edges, m.period_x)[0] == 0
    assert np.bincount(m.wall_side, minlength=6).tolist() == [24, 24, 0, 0, 32, 24]
    ys = m.xy[m.wall_nodes(4), 1]
    assert np.all((ys == 6.0) | (ys == 10.0))
    assert np.bincount(m.wall_edges.ravel()).max() == 2
    w = capillary_channel(60.0)
    assert felbm.validate_mesh(w.mesh.xy, w.mesh.tri, w.mesh.wall_edges, w.mesh.period_x)[0] == 0
    assert np.count_nonzero(w.omega_c) == w.mesh.wall_nodes(4).size


@pytest.mark.parametrize("case", ["index", "clockwise", "repeat", "missing_wall", "interior_wall", "nan_xy",
                                  "not_periodic", "dup_wall"])
def test_validate_rejects_bad_meshes(case):
    m = _mesh()
    xy, tri, we, per = m.xy.copy(), m.tri.copy(), m.wall_edges.copy(), m.period_x
    if case == "index":
        tri[3, 1] = m.n_nodes
    elif case == "clockwise":
        tri[5] = tri[5][::-1]
    elif case == "repeat":
        tri[2, 2] = tri[2, 0]
    elif case == "missing_wall":
        we = we[1:]
    elif case == "interior_wall":
        we = np.vstack([we, tri[40, :2][None, :]])
    elif case == "nan_xy":
        xy[7, 0] = np.nan
    elif case == "not_periodic":
        per = 0.0
    elif case == "dup_wall":
        we = np.vstack([we, we[:1]])
    code, msg = felbm.validate_mesh(xy, tri, we, per)
    expected = -1 if case == "nan_xy" else -2
    assert code == expected, (case, code, msg)
    assert msg


@pytest.mark.parametrize("bad", [dict(xi=0.0), dict(dt=-1.0), dict(rho_v=0.0), dict(sigma=-1.0),
                                 dict(precision=7), dict(solver_sweeps=-1), dict(solver_sweeps=1000),
                                 dict(lambda_min=1.0, lambda_max=0.5), dict(nu_l=float("nan")), dict(kernels=5),
                                 dict(force_scheme=3), dict(force_scheme="nodal", precision="fp32")])
def test_create_rejects_bad_parameters(bad):
    kw = dict(sigma=0.01, xi=4.0, mobility=0.02, rho_l=1.0, rho_v=0.1, nu_l=0.1 / 3, nu_v=0.1 / 3, dt=0.1)
    kw.update(bad)
    with pytest.raises(felbm.FelbmError) as ei:
        felbm.Context(**kw)
    assert ei.value.name == "EINVAL"


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    import paper_1708_04678_amd.felbm as fb
    monkeypatch.setattr(fb, "_lib", None)
    monkeypatch.setattr(fb, "_LIB_PATH", str(tmp_path / "nope.so"))
    with pytest.raises(RuntimeError):
        fb.load_library()
