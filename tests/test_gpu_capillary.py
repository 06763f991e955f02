"""Capillary intrusion into a 2-D channel between two wetting plates (the
2-D form of the capillary experiment of Sec. III.C) on a mesh with holes.

The liquid length l(t) (liquid volume in the channel over its width H)
follows Poiseuille flow driven by the capillary pressure 2 sigma cos(theta)/H:
(eta_l (l + l_e) + eta_v (L - l)) dl/dt = H sigma cos(theta) / 6, with a
constant extra length l_e for the entrance, the reservoir and the moving
contact lines.  Fitting K and l_e jointly for theta = 56 and 72 deg over
l from 20 to about 36 (half the channel by the law): the ratio of the two K
equals cos(56)/cos(72) within 2 % (the angle enters only through the
capillary pressure); each K is within 15 % of H sigma cos(theta) / 6 (the
fit measures 0.89-0.91 here and 0.935 over l up to 60, the start of the run
being slowed by the acceleration of the liquid); l_e agrees between the two
angles within 15 %; mass is conserved.
"""
import numpy as np
import pytest

from gpu_common import log, make_ctx
from workloads import capillary_channel

pytestmark = pytest.mark.gpu


def intrusion(theta, samples=16, fill=0.5):
    w = capillary_channel(theta)
    e, p = w.extra, w.phys
    H, L, l0 = e["width"], e["length"], e["l0"]
    eta_l, eta_v = p.rho_l * p.nu_l, p.rho_v * p.nu_v
    K = H * p.sigma * np.cos(np.radians(theta)) / 6.0
    lt = fill * L
    t_end = (0.5 * (eta_l - eta_v) * (lt * lt - l0 * l0) + eta_v * L * (lt - l0)) / K
    chunk = int(round(t_end / p.dt)) // samples
    log(f"capillary intrusion theta {theta:g}: {w.mesh.n_nodes} nodes, {chunk * samples} steps")
    ctx = make_ctx(w.mesh, w.phys, w.omega_c, precision="fp32", sweeps=11)
    ctx.init(w.C0)
    m = ctx.lumped_mass()
    m0 = ctx.diagnostics()["mass"]
    inside = (w.mesh.xy[:, 0] > e["x0"]) & (w.mesh.xy[:, 0] < e["x1"])
    t, ln = [], []
    for s in range(samples + 1):
        if s:
            ctx.step(chunk)
        t.append(s * chunk * p.dt)
        ln.append(float((m[inside] * ctx.read("C")[inside]).sum() / H))
    drift = abs(ctx.diagnostics()["mass"] - m0) / m0
    ctx.close()
    t, ln = np.array(t), np.array(ln)
    sel = ln > l0 + H
    I = 0.5 * (eta_l - eta_v) * ln * ln + eta_v * L * ln
    A = np.stack([t[sel], -ln[sel], np.ones(int(sel.sum()))], 1)
    K_fit, R0 = np.linalg.lstsq(A, I[sel], rcond=None)[0][:2]
    log(f"  l: {ln[0]:.2f} -> {ln[-1]:.2f}; K_fit / K {K_fit / K:.4f}; entrance length {R0 / eta_l:.2f}; "
        f"mass drift {drift:.1e}")
    assert np.all(np.diff(ln) > 0)
    return K_fit, K, R0 / eta_l, drift


def test_intrusion_rate_scales_with_cos_theta():
    K56, T56, le56, d56 = intrusion(56.0)
    K72, T72, le72, d72 = intrusion(72.0)
    assert abs((K56 / K72) / (T56 / T72) - 1.0) < 0.02
    assert abs(K56 / T56 - 1.0) < 0.15 and abs(K72 / T72 - 1.0) < 0.15
    assert abs(le56 - le72) / le72 < 0.15
    assert d56 < 1e-10 and d72 < 1e-10
