"""Write adjoint_cfg4_tangent.json: the exact derivative of the 256 x 128
adjoint workload's loss (droplet centroid x plus wetted length squared after
500 steps from the tanh droplet) with respect to the wetting potential of 8
seeded bottom-wall nodes, by the complex-step method through the FP64 CPU
oracle (PCG to 1e-13; every oracle operation is complex-analytic, so
dL/dOmega_k = Im L(Omega + i h e_k) / h exactly to rounding with h = 1e-30).

Calls only the oracle, the seeded workload generators and the loss
definition.  One process per node; about 12 minutes on 8 cores.
Usage: python tests/golden/make_adjoint_cfg4_tangent.py"""
import json
import multiprocessing as mp
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.dirname(HERE))

H = 1e-30


def tangent(k):
    import numpy as np

    from losses import wetted_centroid_loss
    from oracle import Oracle
    from workloads import config
    w = config(4)
    om = w.omega_c.astype(complex)
    if k >= 0:
        om[k] += 1j * H
    o = Oracle(w.mesh, w.phys, om)
    g, h = o.init_state(w.C0.astype(complex))
    g, h = o.run(g, h, w.steps)
    L, _ = wetted_centroid_loss(w.mesh, o.mat.lumped, h.sum(1))
    return k, float(L.real), float(L.imag / H)


if __name__ == "__main__":
    from losses import adjoint_probe_nodes
    from workloads import config
    w = config(4)
    nodes = [int(k) for k in adjoint_probe_nodes(w.mesh)]
    t0 = time.time()
    with mp.get_context("spawn").Pool(min(len(nodes), os.cpu_count() or 1)) as pool:
        res = pool.map(tangent, nodes)
    out = {"workload": w.name, "steps": w.steps, "loss": "x_c + L_w^2 (tests/losses.py)", "complex_step": H,
           "solver": "oracle PCG, relative residual 1e-13", "nodes": [r[0] for r in res],
           "loss_value": res[0][1], "dL_domega": [r[2] for r in res],
           "generated_by": "tests/golden/make_adjoint_cfg4_tangent.py", "seconds": round(time.time() - t0, 1)}
    with open(os.path.join(HERE, "adjoint_cfg4_tangent.json"), "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out, indent=1))
