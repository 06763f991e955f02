#!/usr/bin/env python3
"""Throughput of the FE-LBM time step on one MI355X.

Workload (default): three droplets (R = 80, theta = 45/90/135 deg) on a
sinusoidally rough wall, 2048 x 1024 domain, wall-graded jittered split-quad
mesh (2,140,160 nodes, 4,276,224 triangles), density ratio 1000, viscosity
ratio 40.  A step is one pass of the whole hot path (moments, collision,
Laplacians, element forces, Galerkin right-hand side, mass-matrix solve, wall
operator, FP64 reductions) over all nodes; inputs are resident in HBM when the
timed region starts.

Printed: one JSON line with MNUPS (mesh nodes x steps / s / 1e6, each node
update advancing all 9 directions of both g and h) for the FP32 precision form
(FP64 chemical-potential chain, composition transport and reductions) at
K = 11 solve sweeps, and beside it:
  equal_error     FP32 and FP64 after the workload's 2000 steps against a
                  converged FP64 solve (K = 40): max|u| (the spurious-current
                  magnitude), band KE, max|C - C_ref|, mass drift and each
                  droplet's apparent contact angle; FP64 at K = 8..13, the
                  matched count being the fewest sweeps whose max|u| error is
                  at most FP32's; the speedup at that count is the headline
                  ratio;
  fp64_rounding_floor  FP64 at K = 26 (each precision at its own floor);
  roofline        the dominant kernel (the middle solve sweep) at the model's
                  266 B per node, over its HIP-event launch time;
  model_roofline  the whole step at the model's 2*18*4 + 100 + K (3*18*4 + 50)
                  B per node over the timed step;
  cpu_baseline    the CPU oracle timed on a bounded sample, one process and
                  one process per host CPU.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, AMD-published


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_sha():
    """Hash of the sources that set the traffic of the step kernels: the kernels,
    their launch code and the node ordering."""
    h = hashlib.sha256()
    for f in ("common.hpp", "kernels.hpp", "felbm.hip", "mesh_prep.cpp"):
        with open(os.path.join(ROOT, "paper_1708_04678_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def make_ctx(felbm, w, precision, sweeps, stream, force_scheme="mixed"):
    p = w.phys
    ctx = felbm.Context(sigma=p.sigma, xi=p.xi, mobility=p.mobility, rho_l=p.rho_l, rho_v=p.rho_v, nu_l=p.nu_l,
                        nu_v=p.nu_v, dt=p.dt, precision=precision, solver_sweeps=sweeps, force_scheme=force_scheme)
    ctx.bind_stream(stream)
    ctx.upload_mesh(w.mesh.xy, w.mesh.tri, w.mesh.wall_edges, w.mesh.period_x)
    ctx.set_wetting(w.omega_c)
    if w.droplets:
        xc, yc, R = w.droplets[0]
        ctx.set_band(xc, yc, R, w.phys.xi)
    ctx.init(w.C0)
    return ctx, ctx.diagnostics()


def timed_run(torch, ctx, warmup, steps):
    ctx.step(warmup)
    torch.cuda.synchronize()
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0.record()
    ctx.step_async(steps)
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1)
    ctx.step(0)
    return ms


def model_bytes(s, K):
    """Algorithmic HBM bytes per node of the step's model: read and write the 18
    populations (2 * 18 * s), the mesh data (about 100 B), and per solve sweep
    the gathered iterate read, the right-hand side read and the new iterate
    written (3 * 18 * s) plus about 50 B of matrix entries and indices."""
    return 2 * 18 * s + 100 + K * (3 * 18 * s + 50)


def sweep_model_bytes(s):
    return 3 * 18 * s + 50


def droplet_angles(w, ctx):
    """Apparent contact angle of each droplet of the workload from a circle fitted
    to its C = 0.5 contour above the wall roughness (analysis.cap_fit_angle),
    measured against the mean wall line y = 0."""
    from paper_1708_04678_amd.analysis import cap_fit_angle
    C = ctx.read("C")
    out = []
    for (xc, yc, R) in w.droplets:
        out.append(cap_fit_angle(w.mesh.xy, w.mesh.tri, C, w.mesh.period_x, x_window=(xc - 2 * R, xc + 2 * R),
                                 y_min=10.0)[0])
    return out, C


def precision_comparison(felbm, w, stream, sweeps32, k64_candidates, ref_sweeps=40, steps=None):
    """FP32 and FP64 against a converged FP64 solve after the workload's stated
    step count: max|u| (the spurious-current magnitude), band KE, mass drift,
    each droplet's apparent contact angle and max|C - C_ref|.  FP64 runs at each
    candidate sweep count; the matched count is the fewest sweeps whose max|u|
    error is at most FP32's."""
    import numpy as np
    steps = w.steps if steps is None else steps

    def run(prec, K):
        log(f"  {prec} K={K}: {steps} steps")
        ctx, d0 = make_ctx(felbm, w, prec, K, stream)
        ctx.step(steps)
        d = ctx.diagnostics()
        ang, C = droplet_angles(w, ctx)
        ctx.close()
        return {"d": d, "d0": d0, "angles": ang, "C": C}

    ref = run("fp64", ref_sweeps)

    def errors(r):
        return {"max_u": r["d"]["max_u"],
                "max_u_rel_err": abs(r["d"]["max_u"] - ref["d"]["max_u"]) / ref["d"]["max_u"],
                "band_ke_rel_err": abs(r["d"]["band_ke"] - ref["d"]["band_ke"]) / max(ref["d"]["band_ke"], 1e-300),
                "max_C_err": float(np.abs(r["C"] - ref["C"]).max()),
                "theta_deg": [round(a, 4) for a in r["angles"]],
                "theta_err_deg": [round(a - b, 5) for a, b in zip(r["angles"], ref["angles"])],
                "mass_drift": abs(r["d"]["mass"] - r["d0"]["mass"]) / r["d0"]["mass"]}

    e32 = errors(run("fp32", sweeps32))
    e32["K"] = sweeps32
    e64 = []
    for K in k64_candidates:
        e = errors(run("fp64", K))
        e["K"] = K
        e64.append(e)
    ok = [e for e in e64 if e["max_u_rel_err"] <= e32["max_u_rel_err"]]
    matched = min(ok, key=lambda e: e["K"]) if ok else max(e64, key=lambda e: e["K"])
    return {"steps": steps, "reference": {"precision": "fp64", "K": ref_sweeps, "max_u": ref["d"]["max_u"],
                                          "theta_deg": [round(a, 4) for a in ref["angles"]]},
            "fp32": e32, "fp64": e64, "matched_fp64_K": matched["K"],
            "rule": "FP64 at the fewest sweeps whose max|u| error against the converged FP64 solve is at most "
                    "FP32's, both after the workload's stated step count"}


def kernel_pass(ctx, steps):
    ctx.kernel_timing(True)
    ctx.step(steps)
    stats = {s["name"]: s for s in ctx.kernel_stats()}
    ctx.kernel_timing(False)
    return stats


def adjoint_run(felbm, stream, sweeps):
    """Reverse pass of the graded 1024 x 512 workload (527,360 nodes): FP32
    forward with a checkpoint every 100 steps, FP32 adjoint of the loss
    1/2 sum_i m_i (C_i - C*_i)^2 after 2000 steps, gradient w.r.t. the
    wetting potential of every wall node."""
    import numpy as np
    from workloads import config
    w = config(5)
    n, every = w.steps, w.extra["ckpt_every"]
    ctx, _ = make_ctx(felbm, w, "fp32", sweeps, stream)
    m = ctx.lumped_mass()
    t0 = time.perf_counter()
    ctx.step(n)
    t_plain = time.perf_counter() - t0
    ctx.init(w.C0)
    t0 = time.perf_counter()
    ctx.forward_ckpt(n, every)
    t_fwd = time.perf_counter() - t0
    C = ctx.read("C")
    dLdC = m * (C - w.extra["C_target"])
    t0 = time.perf_counter()
    g = ctx.backward_host(dLdC)
    t_bwd = time.perf_counter() - t0
    state = 18 * 4 * ((w.mesh.n_nodes + 63) // 64 * 64) + 8 * ((w.mesh.n_nodes + 63) // 64 * 64)
    n_states = (n + every - 1) // every + every
    ctx.close()
    return {"workload": w.name, "nodes": w.mesh.n_nodes, "steps": n, "ckpt_every": every,
            "forward_plain_s": round(t_plain, 3), "forward_ckpt_s": round(t_fwd, 3), "backward_s": round(t_bwd, 3),
            "backward_over_forward": round(t_bwd / t_plain, 3),
            "checkpoint_bytes": n_states * state, "states_kept": n_states,
            "loss": float(0.5 * np.sum(m * (C - w.extra["C_target"]) ** 2)),
            "grad_norm": float(np.sqrt(np.sum(g * g))),
            "adjoint_MNUPS": round(w.mesh.n_nodes * n / t_bwd / 1e6, 2)}


def three_d_run(felbm, torch, stream, steps, warmup, sweeps32, sweeps64, compare_steps=200):
    """The 3-D path (D3Q19 on linear tetrahedra) on the paper's 3-D droplet
    setting: hemisphere R = 32 on the bottom wall, theta_eq = 150 deg,
    sigma = 0.0025, 1,490,944 nodes and 8,847,360 tetrahedra with layers
    refined toward the wall.  FP32 at K = 13 and FP64 at K = 30 sweeps (the
    Chebyshev error factor on [1/5, 1] is 0.382 per sweep: 2 * 0.382^13 =
    7e-6 and 2 * 0.382^30 = 6e-13, the two precisions' floors as K = 11 and 26
    on [1/4, 1] in 2-D), and FP64 at the sweep count that matches FP32's
    max|u| error after `compare_steps` steps against a converged FP64 solve
    (the headline rule).  Dominant kernel priced at the model's sweep bytes,
    3 * 38 * s per node for the iterate read (gathered once), the right-hand
    side read and the new iterate written, plus the matrix entries (column
    index and value per off-diagonal entry)."""
    import numpy as np
    from workloads.mesh3d import sessile_drop_3d
    name, mesh, phys, C0, om, _ = sessile_drop_3d()
    N = mesh.n_nodes
    out = {"workload": name, "nodes": N, "tetrahedra": mesh.n_tets}

    def make3(prec, K):
        ctx = felbm.Context3D(sigma=phys.sigma, xi=phys.xi, mobility=phys.mobility, rho_l=phys.rho_l,
                              rho_v=phys.rho_v, nu_l=phys.nu_l, nu_v=phys.nu_v, dt=phys.dt, precision=prec,
                              solver_sweeps=K)
        ctx.bind_stream(stream)
        ctx.upload_mesh(mesh.xyz, mesh.tet, mesh.wall_faces, mesh.period)
        ctx.set_wetting(om)
        ctx.init(C0)
        return ctx

    for prec, K in (("fp32", sweeps32), ("fp64", sweeps64)):
        s = 4 if prec == "fp32" else 8
        log(f"3-D {prec} context K={K}")
        ctx = make3(prec, K)
        d0 = ctx.diagnostics()
        ms = timed_run(torch, ctx, warmup, steps)
        d1 = ctx.diagnostics()
        stats = kernel_pass(ctx, max(steps // 4, 5))
        nnz = ctx.mesh_info()["mass_offdiag_nnz"]
        ctx.close()
        sweep_b = 3 * 38 * s * N + nnz * (4 + s)
        step_b = 2 * 38 * s * N + 200 * N + K * sweep_b
        dom_name = max(stats, key=lambda k: stats[k]["total_ms"])
        dom = stats[dom_name]
        avg_ms = dom["total_ms"] / max(dom["launches"], 1)
        dom_bytes = sweep_b if dom_name.startswith("sweep") else dom["bytes_per_launch"]
        ach = dom_bytes / (avg_ms * 1e-3) / 1e9
        tot = sum(v["total_ms"] for v in stats.values())
        out[prec] = {
            "solver_sweeps": K, "ms_per_step": round(ms / steps, 4), "MNUPS": round(N * steps / (ms * 1e-3) / 1e6, 2),
            "population_updates_per_s": round(38 * N * steps / (ms * 1e-3)),
            "mass_drift": abs(d1["mass"] - d0["mass"]) / d0["mass"], "max_u": d1["max_u"],
            "roofline": {"bound": "hbm", "kernel": dom_name, "achieved": round(ach, 1), "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4), "avg_launch_us": round(avg_ms * 1e3, 2),
                         "algorithmic_bytes_per_launch": dom_bytes,
                         "bytes_rule": "3*38*s per node + (4 + s) per off-diagonal mass entry"},
            "model_roofline": {"bytes_per_step": step_b, "achieved": round(step_b / (ms / steps * 1e-3) / 1e9, 1),
                               "frac": round(step_b / (ms / steps * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                               "bytes_rule": "2*38*s + 200 per node + K x sweep bytes"},
            "kernels": {k: {"launches": v["launches"], "avg_us": round(v["total_ms"] / max(v["launches"], 1) * 1e3, 2),
                            "share": round(v["total_ms"] / max(tot, 1e-9), 4)} for k, v in stats.items() if v["launches"]},
        }
        log(f"3-D {prec}: {ms / steps:.3f} ms/step, {out[prec]['MNUPS']} MNUPS")
    out["fp32_over_fp64_speedup_at_own_floors"] = round(out["fp64"]["ms_per_step"] / out["fp32"]["ms_per_step"], 3)
    out["note"] = ("the 3-D FP32 form carries the composition in FP64 (C = sum h + r), so both precisions "
                   "keep the mass to rounding")
    # equal spurious-current error, the rule of the 2-D headline: FP32 (K = sweeps32) and FP64 at
    # K = 11..16 after `compare_steps` steps against a converged FP64 solve (K = 45); FP64 at the
    # fewest sweeps whose max|u| error is at most FP32's
    def run_err(prec, K):
        log(f"  3-D {prec} K={K}: {compare_steps} steps")
        ctx = make3(prec, K)
        ctx.step(compare_steps)
        d, C = ctx.diagnostics(), ctx.read("C")
        ctx.close()
        return d, C

    ref_d, ref_C = run_err("fp64", 45)

    def err(r):
        d, C = r
        return {"max_u_rel_err": abs(d["max_u"] - ref_d["max_u"]) / ref_d["max_u"],
                "max_C_err": float(np.abs(C - ref_C).max())}

    e32 = err(run_err("fp32", sweeps32))
    e64 = {K: err(run_err("fp64", K)) for K in range(11, 17)}
    ok = [K for K, e in e64.items() if e["max_u_rel_err"] <= e32["max_u_rel_err"]]
    if not ok:
        out["equal_error"] = {"steps": compare_steps, "reference_K": 45, "fp32": dict(e32, K=sweeps32),
                              "fp64": [dict(e, K=K) for K, e in e64.items()], "matched_fp64_K": None,
                              "note": "no FP64 candidate reached FP32's error"}
        return out
    k_eq = min(ok)
    ctx = make3("fp64", k_eq)
    ms_eq = timed_run(torch, ctx, 2, steps)
    ctx.close()
    out["equal_error"] = {
        "steps": compare_steps, "reference_K": 45, "fp32": dict(e32, K=sweeps32),
        "fp64": [dict(e, K=K) for K, e in e64.items()], "matched_fp64_K": k_eq,
        "fp64_ms_per_step": round(ms_eq / steps, 4), "fp64_MNUPS": round(N * steps / (ms_eq * 1e-3) / 1e6, 2),
        "speedup": round(ms_eq / steps / out["fp32"]["ms_per_step"], 3)}
    log(f"3-D equal error: FP64 K={k_eq}, speedup {out['equal_error']['speedup']}")
    return out


def comoving_band_ke(ctx, w, m, R, xi):
    """<rho |u - u_c|^2> over the nodes within xi of the circle of radius R
    about the droplet's current centroid, u_c the droplet's mean velocity
    (weights m C): the parasitic energy in the droplet's own frame, free of a
    slow drift of the droplet as a whole.  Returns (energy, centroid, u_c)."""
    import numpy as np
    C, rho = ctx.read("C"), ctx.read("RHO")
    u = np.stack([ctx.read("UX"), ctx.read("UY")], 1)
    xy, P = w.mesh.xy, w.mesh.period_x
    wgt = m * C
    xc0 = w.droplets[0][0]
    dx0 = xy[:, 0] - xc0
    dx0 -= P * np.round(dx0 / P)
    xc = xc0 + np.sum(wgt * dx0) / wgt.sum()
    yc = np.sum(wgt * xy[:, 1]) / wgt.sum()
    uc = np.sum(wgt[:, None] * u, 0) / wgt.sum()
    dx = xy[:, 0] - xc
    dx -= P * np.round(dx / P)
    r = np.sqrt(dx * dx + (xy[:, 1] - yc) ** 2)
    band = np.abs(r - R) <= xi
    du = u - uc
    return float(np.mean(rho[band] * (du[band] ** 2).sum(1))), (float(xc), float(yc)), (float(uc[0]), float(uc[1]))


SPURIOUS_RUNS = {"nodal_collide": ("nodal_collide", "fp64"), "nodal": ("nodal", "fp64"), "mixed": ("mixed", "fp64"),
                 "mixed32": ("mixed", "fp32")}


def spurious_table(felbm, stream, t_end, sweeps32, sweeps64, samples=16, runs=("nodal_collide", "nodal", "mixed",
                                                                              "mixed32")):
    """Parasitic kinetic energy <rho u.u> in the band R +- xi of a static
    droplet (density ratio 2, equal viscosities) at three mesh resolutions,
    mixed (P0) against nodal (P1) forces: the 2-D analogue of the table of
    Sec. III.A.  Sampled `samples` times up to the physical time t_end and
    averaged over the samples of the second half (after the initial
    relaxation of the tanh profile), both in the fixed band about the initial
    centre and in the droplet's own frame (band about the current centroid,
    velocity relative to the droplet's mean velocity).  FP64 with 26 sweeps
    for the nodal force in the collision step (the scheme the paper compares
    against), the nodal force in the streaming step and the mixed scheme,
    plus the FP32 precision form of the mixed scheme."""
    from workloads import free_droplet
    rows = []
    for level in range(3):
        w = free_droplet(level, t_end)
        chunk = max(1, w.steps // samples)
        xc, yc, R = w.droplets[0]
        for scheme, prec in (SPURIOUS_RUNS[r] for r in runs):
            k = sweeps64 if prec == "fp64" else sweeps32
            log(f"spurious-current table: level {level} ({w.mesh.n_nodes} nodes, {w.steps} steps), {scheme} {prec}")
            ctx, d0 = make_ctx(felbm, w, prec, k, stream, force_scheme=scheme)
            m = ctx.lumped_mass()
            trace = []
            for s in range(samples):
                ctx.step(chunk)
                d = ctx.diagnostics()
                ke_c, cen, uc = comoving_band_ke(ctx, w, m, R, w.phys.xi)
                trace.append((round((s + 1) * chunk * w.phys.dt, 3), d["band_ke"], ke_c, d["max_u"], cen, uc))
                log(f"  t {trace[-1][0]:.0f}  band <rho u.u> {d['band_ke']:.3e}  droplet frame {ke_c:.3e}  "
                    f"centroid ({cen[0]:.3f}, {cen[1]:.3f})  max|u| {d['max_u']:.3e}")
            late = trace[samples // 2:]
            rows.append({"level": level, "nodes": w.mesh.n_nodes, "elements": w.mesh.n_tris, "scheme": scheme,
                         "precision": prec, "dt": w.phys.dt, "steps": chunk * samples, "t_end": trace[-1][0],
                         "band_ke_mean_second_half": float(sum(x[1] for x in late) / len(late)),
                         "comoving_band_ke_mean_second_half": float(sum(x[2] for x in late) / len(late)),
                         "band_ke_final": trace[-1][1], "comoving_band_ke_final": trace[-1][2],
                         "max_u_final": trace[-1][3], "centroid_final": trace[-1][4],
                         "mass_drift": abs(d["mass"] - d0["mass"]) / d0["mass"], "trace": trace})
            ctx.close()
    return rows


def angle_run(felbm, stream, w, sweeps32, samples):
    """One sessile droplet in FP32 up to w.steps, the contact angle measured
    on the C = 0.5 contour `samples` times: from the cap height and base
    (tan(theta/2) = 2h/b) and from a circle fitted to the contour above
    y = 2 xi (cos(theta) = -y_c/r), which needs no wall crossings (a droplet
    on a fully non-wetting wall may touch it at one point only)."""
    import numpy as np
    from paper_1708_04678_amd.analysis import cap_fit_angle, contact_angle

    def measure(C):
        try:
            th, hgt, base = contact_angle(w.mesh.xy, w.mesh.tri, w.mesh.wall_nodes(0), C, w.mesh.period_x)
        except ValueError:
            th, hgt, base = float("nan"), float("nan"), float("nan")
        try:
            th_fit = cap_fit_angle(w.mesh.xy, w.mesh.tri, C, w.mesh.period_x, y_min=2 * w.phys.xi)[0]
        except (ValueError, np.linalg.LinAlgError):
            th_fit = float("nan")
        return th, hgt, base, th_fit
    ctx, d0 = make_ctx(felbm, w, "fp32", sweeps32, stream)
    chunk = max(1, w.steps // samples)
    trace = []
    for s in range(samples):
        try:
            ctx.step(chunk)
        except felbm.FelbmError as e:
            log(f"  diverged: {e}")
            ctx.close()
            return {"nodes": w.mesh.n_nodes, "xi": w.phys.xi, "dt": w.phys.dt, "mobility": w.phys.mobility,
                    "diverged": str(e), "trace": trace}
        d = ctx.diagnostics()
        th, hgt, base, th_fit = measure(ctx.read("C"))
        trace.append((round((s + 1) * chunk * w.phys.dt, 3), round(th, 3), d["max_u"], round(th_fit, 3)))
        log(f"  t {trace[-1][0]:.0f}  theta {th:.2f} deg (h {hgt:.2f}, b {base:.2f}), circle fit {th_fit:.2f}  "
            f"max|u| {d['max_u']:.3e}")
    ctx.close()
    q = trace[(3 * samples) // 4 - 1]
    return {"nodes": w.mesh.n_nodes, "h": round(float(w.mesh.xy[1, 0] - w.mesh.xy[0, 0]), 6), "xi": w.phys.xi,
            "dt": w.phys.dt, "mobility": w.phys.mobility, "sigma": w.phys.sigma, "box": w.name,
            "steps": chunk * samples, "t_end": trace[-1][0],
            "theta_measured": trace[-1][1], "theta_circle_fit": trace[-1][3], "height": round(hgt, 3),
            "base": round(base, 3), "theta_change_last_quarter": round(trace[-1][1] - q[1], 3),
            "theta_fit_change_last_quarter": round(trace[-1][3] - q[3], 3),
            "max_u_final": trace[-1][2], "mass_drift": abs(d["mass"] - d0["mass"]) / d0["mass"], "trace": trace}


def contact_angle_sweep(felbm, stream, t_end, sweeps32, samples=8,
                        thetas=(30.0, 45.0, 60.0, 75.0, 90.0, 105.0, 120.0, 135.0, 150.0),
                        contrasts=((10.0, 1.0), (100.0, 40.0)), sigma=0.01, box=6.4, resolution_study=True):
    """Equilibrium contact angle against the imposed wetting potential
    Omega_c = -cos(theta) (the 2-D analogue of the angle sweep of Sec. III.B):
    a R = 20 droplet on a wall meshed with h = xi / 8, for two density /
    viscosity contrasts, in the FP32 precision form.  Then the resolution
    study: theta = 60 and 120 deg at h / xi = 1/2, 1/4, 1/8, 1/16."""
    import numpy as np
    from workloads import wetting_drop
    sweep = []
    for m_rho, m_nu in contrasts:
        for theta in thetas:
            w = wetting_drop(theta, m_rho, m_nu, refine=2, t_end=t_end, sigma=sigma, box=box)
            log(f"contact-angle sweep: M_rho {m_rho:g} M_nu {m_nu:g} theta {theta:g} ({w.mesh.n_nodes} nodes, "
                f"{w.steps} steps)")
            row = {"theta_imposed": theta, "omega_c": -float(np.cos(np.radians(theta))), "m_rho": m_rho,
                   "m_nu": m_nu}
            row.update(angle_run(felbm, stream, w, sweeps32, samples))
            sweep.append(row)
    resolution = []
    for refine, xi, mobility, dt in () if not resolution_study else ((1, 2.0, 0.2, None), (1, 4.0, 0.2, None), (2, 4.0, 0.2, None),
                                     (4, 4.0, 0.1, 0.0125)):
        for theta in (60.0, 120.0):
            w = wetting_drop(theta, refine=refine, xi=xi, mobility=mobility, dt=dt, t_end=t_end)
            log(f"contact-angle resolution: h {1.0 / refine:g} xi {xi:g} theta {theta:g} ({w.mesh.n_nodes} nodes, "
                f"{w.steps} steps)")
            row = {"theta_imposed": theta, "h_over_xi": 1.0 / (refine * xi), "m_rho": 10.0, "m_nu": 1.0}
            row.update(angle_run(felbm, stream, w, sweeps32, samples))
            resolution.append(row)
    return sweep, resolution


def mobility_study(felbm, stream, t_over_t0, sweeps32, samples=60):
    """Decay of the mean kinetic energy <T> = 0.5 sum(rho u.u) / N of a
    sessile droplet (theta = 120 deg, density ratio 100, viscosity ratio 40,
    R = 20, h = xi / 8) for four mobilities, with time in units of the
    viscous time t0 = rho_l nu_l R / sigma and the mobility as
    S = sqrt(M rho_l nu_l) / R (Sec. III.B, fig:mobility), up to t0 *
    t_over_t0, FP32 precision form.  Trace entries: (t / t0, <T>, max|u|,
    x of the droplet's centroid)."""
    import math
    from paper_1708_04678_amd.analysis import contact_angle
    from workloads import wetting_drop
    rows = []
    for mobility in (0.02, 0.05, 0.1, 0.2):
        w = wetting_drop(120.0, 100.0, 40.0, refine=2, mobility=mobility)
        xc, yc, R = w.droplets[0]
        p = w.phys
        t0 = p.rho_l * p.nu_l * R / p.sigma
        S = math.sqrt(mobility * p.rho_l * p.nu_l) / R
        steps = int(round(t_over_t0 * t0 / p.dt))
        chunk = max(1, steps // samples)
        log(f"mobility study: M {mobility:g} (S {S:.3e}, t0 {t0:.2f}), {w.mesh.n_nodes} nodes, {chunk * samples} steps")
        ctx, d0 = make_ctx(felbm, w, "fp32", sweeps32, stream)
        m = ctx.lumped_mass()
        trace = [(0.0, d0["mean_ke"], d0["max_u"], float(xc))]
        for s in range(samples):
            ctx.step(chunk)
            d = ctx.diagnostics()
            C = ctx.read("C")
            x_c = float((m * C * w.mesh.xy[:, 0]).sum() / (m * C).sum())
            trace.append((round((s + 1) * chunk * p.dt / t0, 4), d["mean_ke"], d["max_u"], x_c))
        th, hgt, base = contact_angle(w.mesh.xy, w.mesh.tri, w.mesh.wall_nodes(0), ctx.read("C"), w.mesh.period_x)
        log(f"  <T> at t/t0 = {trace[-1][0]:g}: {trace[-1][1]:.3e}, max|u| {trace[-1][2]:.3e}, theta {th:.2f} deg")
        rows.append({"mobility": mobility, "S": S, "t0": t0, "nodes": w.mesh.n_nodes, "dt": p.dt,
                     "steps": chunk * samples, "theta_final": round(th, 3),
                     "mass_drift": abs(d["mass"] - d0["mass"]) / d0["mass"], "trace": trace})
        ctx.close()
    return rows


def washburn_length(t, K, eta_l, eta_v, length, l0):
    """Liquid length in a 2-D channel of the given length from
    (eta_l l + eta_v (length - l)) dl/dt = K, l(0) = l0: Poiseuille flow
    between plates with the capillary pressure 2 sigma cos(theta) / H drawn
    across both fluids in the channel, K = H sigma cos(theta) / 6."""
    import numpy as np
    a, b = 0.5 * (eta_l - eta_v), eta_v * length
    c = K * np.asarray(t) + a * l0 * l0 + b * l0
    return (-b + np.sqrt(b * b + 4.0 * a * c)) / (2.0 * a)


def capillary_study(felbm, stream, sweeps32, samples=40, fill=0.75, length_widths=10.0):
    """Capillary intrusion into a 2-D channel (Sec. III.C in its 2-D form):
    for theta = 56, 72, 83 deg the liquid length l(t) = (liquid volume in the
    channel) / H against the Washburn law of `washburn_length`, run until the
    law's l reaches `fill` of the channel.  Over the samples with l beyond
    l0 + H two fits: the pure law, K_pure = d/dt [(eta_l - eta_v) l^2 / 2 +
    eta_v L l]; and the law with a constant extra resistance eta_l l_e (the
    entrance, the reservoir and the moving contact lines), fitted jointly as
    (eta_l - eta_v) l^2 / 2 + eta_v L l + eta_l l_e l = K_fit t + c.  The
    effective cos(theta) is 6 K_fit / (H sigma).  The channel is
    `length_widths` widths long."""
    import numpy as np
    from workloads import capillary_channel
    rows = []
    for theta in (56.0, 72.0, 83.0):
        w = capillary_channel(theta, length=10.0 * length_widths)
        e, p = w.extra, w.phys
        H, L, l0 = e["width"], e["length"], e["l0"]
        eta_l, eta_v = p.rho_l * p.nu_l, p.rho_v * p.nu_v
        K = H * p.sigma * np.cos(np.radians(theta)) / 6.0
        lt = fill * L
        t_end = (0.5 * (eta_l - eta_v) * (lt * lt - l0 * l0) + eta_v * L * (lt - l0)) / K
        steps = int(round(t_end / p.dt))
        chunk = max(1, steps // samples)
        log(f"capillary intrusion: theta {theta:g} ({w.mesh.n_nodes} nodes, {chunk * samples} steps, t {t_end:.0f})")
        ctx, d0 = make_ctx(felbm, w, "fp32", sweeps32, stream)
        m = ctx.lumped_mass()
        inside = (w.mesh.xy[:, 0] > e["x0"]) & (w.mesh.xy[:, 0] < e["x1"])
        trace = []
        for s in range(samples + 1):
            if s:
                ctx.step(chunk)
            t = s * chunk * p.dt
            l_meas = float((m[inside] * ctx.read("C")[inside]).sum() / H)
            if s % 5 == 0:
                log(f"  sample {s}/{samples}: t {t:.0f}, l {l_meas:.2f}")
            trace.append((round(t, 3), round(l_meas, 4), round(float(washburn_length(t, K, eta_l, eta_v, L, l0)), 4)))
        d = ctx.diagnostics()
        ctx.close()
        tt = np.array([x[0] for x in trace])
        ll = np.array([x[1] for x in trace])
        sel = ll > l0 + H
        I = 0.5 * (eta_l - eta_v) * ll * ll + eta_v * L * ll
        K_pure = float(np.polyfit(tt[sel], I[sel], 1)[0])
        A = np.stack([tt[sel], -ll[sel], np.ones(int(sel.sum()))], 1)
        K_fit, R0 = (float(v) for v in np.linalg.lstsq(A, I[sel], rcond=None)[0][:2])
        cos_eff = 6.0 * K_fit / (H * p.sigma)
        log(f"  l(t_end) {ll[-1]:.2f} (law {trace[-1][2]:.2f}); pure law K_fit / K {K_pure / K:.3f}; "
            f"with an entrance length: K_fit / K {K_fit / K:.3f}, entrance length {R0 / eta_l:.2f}")
        rows.append({"theta": theta, "nodes": w.mesh.n_nodes, "width": H, "length": L, "l0": l0, "dt": p.dt,
                     "sigma": p.sigma, "eta_l": eta_l, "eta_v": eta_v, "K": K,
                     "K_fit_pure_law_over_K": K_pure / K, "K_fit": K_fit, "K_fit_over_K": K_fit / K,
                     "entrance_length": R0 / eta_l, "cos_theta_effective": cos_eff,
                     "theta_effective": float(np.degrees(np.arccos(min(1.0, cos_eff)))),
                     "steps": chunk * samples, "max_u_final": d["max_u"],
                     "mass_drift": abs(d["mass"] - d0["mass"]) / d0["mass"], "trace": trace})
    return rows


def _host_cpu():
    """Host CPU description: /proc/cpuinfo model name, lscpu's model, sockets
    and cores, nproc and the CPUs this process may run on."""
    import subprocess
    info = {"nproc": os.cpu_count()}
    try:
        info["cpus_allowed"] = len(os.sched_getaffinity(0))
    except AttributeError:
        info["cpus_allowed"] = os.cpu_count()
    try:
        with open("/proc/cpuinfo") as fh:
            info["model_name"] = next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")), "")
    except OSError:
        info["model_name"] = ""
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for ln in out.splitlines():
            k, _, v = ln.partition(":")
            if k.strip() in ("Model name", "Socket(s)", "Core(s) per socket", "Thread(s) per core", "CPU max MHz"):
                info["lscpu_" + k.strip().lower().replace(" ", "_").replace("(s)", "s")] = v.strip()
    except (OSError, subprocess.SubprocessError):
        pass
    return info


def _oracle_worker(cfg, rows, steps, barrier, out):
    """One oracle process: build the bounded sample, one warm-up step, then
    `steps` timed steps that start together with the other workers."""
    from oracle import Oracle
    from workloads import config
    w = config(cfg, row_limit=rows)
    o = Oracle(w.mesh, w.phys, w.omega_c)
    g, h = o.init_state(w.C0)
    g, h = o.step(g, h)
    if barrier is not None:
        barrier.wait(timeout=900)
    c0, t0 = time.process_time(), time.perf_counter()
    for _ in range(steps):
        g, h = o.step(g, h)
    out.put((time.perf_counter() - t0, time.process_time() - c0, w.mesh.n_nodes))


def _run_oracle_processes(ctx, n, cfg, rows, steps):
    """n concurrent oracle processes (one task each), their timed steps started together."""
    out = ctx.Queue()
    barrier = ctx.Barrier(n) if n > 1 else None
    ps = [ctx.Process(target=_oracle_worker, args=(cfg, rows, steps, barrier, out)) for _ in range(n)]
    for p in ps:
        p.start()
    res = [out.get(timeout=1800) for _ in range(n)]
    for p in ps:
        p.join()
    return res


def cpu_baseline(cfg, rows, steps=2, max_procs=16):
    """The FP64 CPU oracle, as it stands (numpy/scipy, one thread per process),
    on a bounded sample: the bottom `rows` node rows of the same mesh.  First
    one process alone (the one-thread figure), then one process per allowed
    CPU (at most max_procs) running the same sample concurrently, with their
    timed steps started together; the all-core throughput is the summed node
    updates over the slowest process's time."""
    import multiprocessing as mp
    from workloads import config
    full_rows = config(cfg).mesh.nrows
    host = _host_cpu()
    os.environ["OMP_NUM_THREADS"] = "1"       # one thread per oracle process
    os.environ["OPENBLAS_NUM_THREADS"] = "1"
    ctx = mp.get_context("spawn")
    wall1, cpu1, nodes = _run_oracle_processes(ctx, 1, cfg, rows, steps)[0]
    procs = max(1, min(max_procs, host.get("cpus_allowed") or 1))
    res = _run_oracle_processes(ctx, procs, cfg, rows, steps)
    wall_n = max(r[0] for r in res)
    one = nodes * steps / wall1 / 1e6
    allc = procs * nodes * steps / wall_n / 1e6
    return {"value": allc, "unit": "MNUPS", "cores": procs, "kind": "oracle",
            "one_thread_value": one, "one_thread_seconds": round(wall1, 2),
            "seconds": round(wall_n, 2), "cpu_seconds_total": round(sum(r[1] for r in res) + cpu1, 1),
            "host": host,
            "sample": f"{steps} steps (after 1 warm-up step) of the FP64 numpy/scipy oracle on the bottom {rows} of "
                      f"the {full_rows} node rows of the same mesh ({nodes} nodes, same droplets and walls); "
                      f"one process alone, then {procs} concurrent processes (one thread each) on the same sample"}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--config", type=int, default=3)
    # sweeps per step at which each precision's result reaches its own rounding
    # floor against a converged FP64 solve (FP32: max|u| ~1e-5, C ~2e-7;
    # FP64: ~1e-12), measured on the theta = 60 deg and three-droplet workloads
    ap.add_argument("--sweeps32", type=int, default=11, help="solver sweeps per step in FP32")
    ap.add_argument("--sweeps64", type=int, default=26, help="solver sweeps per step in FP64")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--compare-steps", type=int, default=0,
                    help="steps of the FP32-vs-FP64 error comparison (default: the workload's stated count)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-3d", action="store_true", help="skip the 3-D (D3Q19 on tetrahedra) measurement")
    ap.add_argument("--only-3d", action="store_true", help="only run the 3-D measurement and print it")
    ap.add_argument("--sweeps3d", default="13,30", help="FP32,FP64 solver sweeps of the 3-D measurement")
    ap.add_argument("--cpu-rows", type=int, default=65)
    ap.add_argument("--spurious-table", type=float, default=0.0, metavar="T",
                    help="only run the parasitic-current comparison (mixed vs nodal forces, three resolutions) "
                         "up to physical time T and print it")
    ap.add_argument("--spurious-runs", default="nodal_collide,nodal,mixed,mixed32",
                    help="comma-separated runs of --spurious-table: nodal_collide, nodal, mixed, mixed32")
    ap.add_argument("--contact-angle-sweep", type=float, default=0.0, metavar="T",
                    help="only run the equilibrium contact angle against the imposed wetting potential "
                         "(two contrasts, 30-150 deg, and a mesh-resolution study) up to physical time T")
    ap.add_argument("--angles", default="30,45,60,75,90,105,120,135,150", help="angles of --contact-angle-sweep")
    ap.add_argument("--contrasts", default="10:1,100:40", help="M_rho:M_nu pairs of --contact-angle-sweep")
    ap.add_argument("--sigma", type=float, default=0.01, help="surface tension of --contact-angle-sweep")
    ap.add_argument("--box", type=float, default=6.4, help="box length / R of --contact-angle-sweep")
    ap.add_argument("--no-resolution", action="store_true", help="skip the h/xi study of --contact-angle-sweep")
    ap.add_argument("--mobility-study", type=float, default=0.0, metavar="T",
                    help="only run the kinetic-energy decay of a theta = 120 deg droplet for four mobilities up "
                         "to T viscous times")
    ap.add_argument("--capillary", action="store_true",
                    help="only run capillary intrusion into a channel (theta = 56, 72, 83 deg) against Washburn")
    ap.add_argument("--capillary-length", type=float, default=10.0,
                    help="channel length of --capillary in channel widths")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of 1 GiB ten times (HBM counter calibration)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        x = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        y.copy_(x)
        start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        start.record()
        for _ in range(10):
            y.copy_(x)
        stop.record()
        torch.cuda.synchronize()
        ms = start.elapsed_time(stop) / 10
        print(json.dumps({"copy_bytes_read": 1 << 30, "copy_bytes_written": 1 << 30, "copies": 10,
                          "ms_per_copy": round(ms, 4), "copy_GBps": round(2 * (1 << 30) / (ms * 1e-3) / 1e9, 1)}))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); multi-GPU sharding of this path is "
              "a design, not built", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1708_04678_amd as felbm
    from workloads import config

    torch.cuda.set_device(0)
    if args.spurious_table:
        tstream = torch.cuda.Stream()
        torch.cuda.set_stream(tstream)
        rows = spurious_table(felbm, tstream.cuda_stream, args.spurious_table, args.sweeps32, args.sweeps64,
                              runs=tuple(args.spurious_runs.split(",")))
        print(json.dumps({"spurious_current_table": rows}))
        return
    if args.contact_angle_sweep:
        tstream = torch.cuda.Stream()
        torch.cuda.set_stream(tstream)
        sweep, resolution = contact_angle_sweep(
            felbm, tstream.cuda_stream, args.contact_angle_sweep, args.sweeps32,
            thetas=tuple(float(a) for a in args.angles.split(",")),
            contrasts=tuple(tuple(float(v) for v in c.split(":")) for c in args.contrasts.split(",")),
            sigma=args.sigma, box=args.box, resolution_study=not args.no_resolution)
        print(json.dumps({"contact_angle_sweep": sweep, "contact_angle_resolution": resolution}))
        return
    if args.capillary:
        tstream = torch.cuda.Stream()
        torch.cuda.set_stream(tstream)
        print(json.dumps({"capillary_intrusion": capillary_study(felbm, tstream.cuda_stream, args.sweeps32,
                                                                 length_widths=args.capillary_length)}))
        return
    if args.mobility_study:
        tstream = torch.cuda.Stream()
        torch.cuda.set_stream(tstream)
        print(json.dumps({"mobility_study": mobility_study(felbm, tstream.cuda_stream, args.mobility_study,
                                                           args.sweeps32)}))
        return

    # a dedicated (default-priority) torch stream: the library and the timing events share it
    tstream = torch.cuda.Stream()
    torch.cuda.set_stream(tstream)
    stream = tstream.cuda_stream
    k3 = [int(v) for v in args.sweeps3d.split(",")]
    if args.only_3d:
        print(json.dumps({"three_d": three_d_run(felbm, torch, stream, args.steps, args.warmup, k3[0], k3[1])}),
              flush=True)
        return
    log(f"workload {args.config}")
    w = config(args.config)
    N, E = w.mesh.n_nodes, w.mesh.n_tris

    log("fp32 context")
    c32, d0 = make_ctx(felbm, w, "fp32", args.sweeps32, stream)
    ms32 = timed_run(torch, c32, args.warmup, args.steps)
    log(f"fp32 {ms32 / args.steps:.3f} ms/step")
    stats = kernel_pass(c32, args.steps)
    d32 = c32.diagnostics()
    info = c32.mesh_info()

    # dominant kernel: the launch type with the largest total time, priced with
    # the model's per-node sweep bytes (3 * 18 * 4 + 50 B in FP32) x nodes
    dom_name = max(stats, key=lambda k: stats[k]["total_ms"])
    dom = stats[dom_name]
    avg_ms = dom["total_ms"] / max(dom["launches"], 1)
    sweep_kernel = dom_name.startswith("sweep")
    dom_bytes = sweep_model_bytes(4) * N if sweep_kernel else dom["bytes_per_launch"]
    achieved = dom_bytes / (avg_ms * 1e-3) / 1e9
    traffic = None
    tfile = os.path.join(ROOT, "profiles", f"{dom_name}_traffic.json")
    if os.path.exists(tfile):
        with open(tfile) as fh:
            t = json.load(fh)
        if t.get("kernel_source_sha") == kernel_source_sha() and t.get("workload") == w.name:
            traffic = t.get("hbm_bytes_per_launch")
    roofline = {"bound": "hbm", "kernel": dom_name, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "avg_launch_us": round(avg_ms * 1e3, 2), "algorithmic_bytes_per_launch": dom_bytes,
                "bytes_rule": ("model sweep bytes 3*18*4 + 50 = 266 B per node x nodes" if sweep_kernel
                               else "the kernel's own byte count"),
                "detailed_bytes_per_launch": dom["bytes_per_launch"]}
    # whole step against the model's bytes (2*18*s + 100 + K (3*18*s + 50) per node)
    b32 = model_bytes(4, args.sweeps32)
    m_gbs = b32 * N / (ms32 / args.steps * 1e-3) / 1e9
    model_roofline = {"bound": "hbm", "bytes_per_node_step": b32, "achieved": round(m_gbs, 1), "peak": HBM_PEAK_GBS,
                      "unit": "GB/s", "frac": round(m_gbs / HBM_PEAK_GBS, 4)}
    # and against the sum of every kernel's own byte count (includes the FP64 chain and composition transport)
    step_bytes = sum(v["bytes_per_launch"] * v["launches"] for v in stats.values()) / args.steps
    step_gbs = step_bytes / (ms32 / args.steps * 1e-3) / 1e9
    step_roofline = {"bound": "hbm", "algorithmic_bytes_per_step": round(step_bytes),
                     "algorithmic_bytes_per_node_step": round(step_bytes / N, 1), "achieved": round(step_gbs, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(step_gbs / HBM_PEAK_GBS, 4)}
    kernels = {k: {"launches": v["launches"], "avg_us": round(v["total_ms"] / max(v["launches"], 1) * 1e3, 2),
                   "share": round(v["total_ms"] / max(sum(x["total_ms"] for x in stats.values()), 1e-9), 4)}
               for k, v in stats.items() if v["launches"]}

    out = {
        "metric": "MNUPS (mesh-node x 9-pop updates/s) FP32 vs FP64 at equal spurious-current error",
        "value": round(N * args.steps / (ms32 * 1e-3) / 1e6, 2),
        "unit": "MNUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms32 / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "nodes": N, "triangles": E, "mass_offdiag_nnz": info["mass_offdiag_nnz"],
                   "precision": "fp32 populations/arithmetic, fp64 chemical-potential chain and reductions",
                   "solver_sweeps": args.sweeps32, "population_updates_per_s": round(18 * N * args.steps / (ms32 * 1e-3)),
                   "parallelism": "single GPU"},
        "roofline": roofline,
        "model_roofline": model_roofline,
        "step_roofline": step_roofline,
        "kernels": kernels,
    }
    out["mass_drift_fp32"] = abs(d32["mass"] - d0["mass"]) / d0["mass"]
    c32.close()

    if not args.no_fp64:
        # equal spurious-current error: FP32 and FP64 against a converged FP64 solve after the
        # workload's stated step count, FP64 at the fewest sweeps that match FP32's max|u| error
        csteps = args.compare_steps or w.steps
        log(f"precision comparison ({csteps} steps)")
        cmp = precision_comparison(felbm, w, stream, args.sweeps32, list(range(args.sweeps32 - 3, args.sweeps32 + 3)),
                                   steps=csteps)
        k_eq = cmp["matched_fp64_K"]
        timing64 = {}
        for K in sorted({k_eq, args.sweeps64}):
            log(f"fp64 context K={K}")
            c64, _ = make_ctx(felbm, w, "fp64", K, stream)
            ms64 = timed_run(torch, c64, args.warmup, args.steps)
            log(f"fp64 K={K} {ms64 / args.steps:.3f} ms/step")
            c64.close()
            timing64[K] = ms64
        out["equal_error"] = dict(cmp)
        out["equal_error"].update({
            "fp32_MNUPS": out["value"], "fp64_K": k_eq,
            "fp64_MNUPS": round(N * args.steps / (timing64[k_eq] * 1e-3) / 1e6, 2),
            "fp64_ms_per_step": round(timing64[k_eq] / args.steps, 4),
            "speedup": round(timing64[k_eq] / ms32, 3)})
        out["fp64_rounding_floor"] = {
            "K": args.sweeps64, "MNUPS": round(N * args.steps / (timing64[args.sweeps64] * 1e-3) / 1e6, 2),
            "ms_per_step": round(timing64[args.sweeps64] / args.steps, 4),
            "speedup": round(timing64[args.sweeps64] / ms32, 3),
            "model_bytes_per_node_step": model_bytes(8, args.sweeps64),
            "note": "each precision at its own rounding floor (FP32 K = 11, FP64 K = 26): a secondary reading"}

    if not args.no_adjoint:
        log("adjoint (graded 1024x512, 2000 steps)")
        out["adjoint"] = adjoint_run(felbm, stream, args.sweeps32)

    if not args.no_3d:
        log("3-D droplet (D3Q19 on tetrahedra)")
        out["three_d"] = three_d_run(felbm, torch, stream, min(args.steps, 100), min(args.warmup, 10), k3[0], k3[1])

    if not args.no_cpu_baseline:
        log(f"cpu baseline (oracle, bottom {args.cpu_rows} rows, one process, then one per CPU)")
        out["cpu_baseline"] = cpu_baseline(args.config, args.cpu_rows)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
