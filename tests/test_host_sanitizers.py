"""The host-side mesh preparation (validation, bisection ordering, adjacency,
mass matrix) built with AddressSanitizer and UBSan by g++ and run, in a child
process with the sanitizer runtimes preloaded, on valid meshes (periodic,
closed, with holes; caller order and bisection order) and on malformed
ones, which must be rejected with an error code and no sanitizer report."""
import os
import shutil
import subprocess
import sys
import textwrap

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)

CHILD = textwrap.dedent('''
    import ctypes as ct, sys
    import numpy as np
    sys.path.insert(0, ROOT)
    from workloads import capillary_channel, channel_mesh, config, split_grid_mesh, uniform_rows
    lib = ct.CDLL(LIB)
    D, I = ct.POINTER(ct.c_double), ct.POINTER(ct.c_int32)
    lib.asan_prep.argtypes = [ct.c_int64, D, ct.c_int64, I, ct.c_int64, I, ct.c_double, ct.c_int]
    def run(xy, tri, we, period, reorder=1):
        xy = np.ascontiguousarray(xy, np.float64)
        tri = np.ascontiguousarray(tri, np.int32).reshape(-1, 3)
        we = np.ascontiguousarray(we, np.int32).reshape(-1, 2)
        return lib.asan_prep(len(xy), xy.ctypes.data_as(D), len(tri), tri.ctypes.data_as(I), len(we),
                             we.ctypes.data_as(I), period, reorder)
    for m in (config(1).mesh, channel_mesh(40.0, 16.0, 1.0, 12.0, 28.0, 6.0, 10.0, seed=[7]),
              capillary_channel(60.0).mesh, split_grid_mesh(29.0, uniform_rows(10.0, 11), 29, seed=[3], periodic=False)):
        for ro in (0, 1):
            assert run(m.xy, m.tri, m.wall_edges, m.period_x, ro) == 0
    m = split_grid_mesh(8.0, uniform_rows(4.0, 5), 8, seed=[1])
    cases = []
    t = m.tri.copy(); t[3, 1] = 10 ** 6; cases.append((m.xy, t, m.wall_edges, m.period_x))
    t = m.tri.copy(); t[5] = t[5][::-1]; cases.append((m.xy, t, m.wall_edges, m.period_x))
    t = m.tri.copy(); t[2, 2] = t[2, 0]; cases.append((m.xy, t, m.wall_edges, m.period_x))
    cases.append((m.xy, m.tri, m.wall_edges[1:], m.period_x))
    cases.append((m.xy, m.tri, np.concatenate([m.wall_edges, [[m.tri[10, 0], m.tri[10, 1]]]]), m.period_x))
    xy = m.xy.copy(); xy[7, 0] = np.nan; cases.append((xy, m.tri, m.wall_edges, m.period_x))
    cases.append((m.xy, m.tri, m.wall_edges, 0.0))
    cases.append((m.xy, m.tri, np.concatenate([m.wall_edges, m.wall_edges[:1]]), m.period_x))
    w = m.wall_edges.copy(); w[0, 0] = -5; cases.append((m.xy, m.tri, w, m.period_x))
    cases.append((m.xy, m.tri[:0], m.wall_edges, m.period_x))
    for c in cases:
        assert run(*c) < 0
    print("ok")
''')


def test_mesh_prep_under_address_and_ub_sanitizers(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    rt = [subprocess.run([gxx, f"-print-file-name={n}"], capture_output=True, text=True).stdout.strip()
          for n in ("libasan.so", "libubsan.so")]
    if not all(os.path.isabs(p) and os.path.exists(p) for p in rt):
        pytest.skip("sanitizer runtimes not available")
    lib = str(tmp_path / "libprep_asan.so")
    subprocess.run([gxx, "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
                    "-fno-sanitize-recover=undefined", "-fPIC", "-shared", f"-I{ROOT}/include",
                    f"-I{ROOT}/paper_1708_04678_amd/csrc", f"{ROOT}/paper_1708_04678_amd/csrc/mesh_prep.cpp",
                    f"{HERE}/asan_mesh_prep_driver.cpp", "-o", lib], check=True)
    env = dict(os.environ, LD_PRELOAD=":".join(rt), ASAN_OPTIONS="detect_leaks=0:abort_on_error=0")
    code = f"ROOT = {ROOT!r}\nLIB = {lib!r}\n" + CHILD
    p = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env, timeout=300)
    report = p.stdout + p.stderr
    assert p.returncode == 0, report[-4000:]
    assert "AddressSanitizer" not in report and "runtime error" not in report, report[-4000:]
    assert p.stdout.strip().endswith("ok")
