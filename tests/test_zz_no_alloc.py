"""felbm_diagnostics_noalloc (fixed per-device scratch, no allocation) against
felbm_diagnostics through the C ABI: the same reductions, so every field must
agree bitwise.  Two calls in a row on two meshes, the second smaller, in both
precisions; the scratch keeps the previous call's contents between them."""
import numpy as np
import pytest

from gpu_common import log, make_ctx
from workloads import config, wetting_from_angles

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_noalloc_diagnostics_match_allocating_entry_point(prec):
    for cfg in (2, 1):   # 131,584 nodes, then 2,112
        w = config(cfg)
        om = wetting_from_angles(w.mesh, 60.0)
        log(f"no-alloc diagnostics, workload {cfg} ({w.mesh.n_nodes} nodes), {prec}")
        ctx = make_ctx(w.mesh, w.phys, om, precision=prec, sweeps=8)
        xc, yc, R = w.droplets[0]
        ctx.set_band(xc, yc, R, w.phys.xi)
        ctx.set_residual_sampling(2)
        ctx.init(w.C0)
        ctx.step(3)
        ref = ctx.diagnostics()
        got = ctx.diagnostics_noalloc()
        log(f"  mass {got['mass']!r} max_u {got['max_u']!r} band_ke {got['band_ke']!r}")
        assert got == ref
        assert got["band_nodes"] > 0 and got["max_u"] > 0 and got["residual_step"] == 2
        # a second call on the same state: the same record again
        assert ctx.diagnostics_noalloc() == ref
        ctx.step(1)
        assert ctx.diagnostics_noalloc() == ctx.diagnostics()
        ctx.close()
