"""torch.autograd binding of the FE-LBM adjoint: the composition field after
n steps as a differentiable function of the per-node wetting potential
Omega_c.  Torch provides device memory and the stream; the forward run and
the reverse pass run in the library (felbm_forward_ckpt / felbm_backward)."""
from __future__ import annotations

import numpy as np
import torch

from .felbm import Context


class WettingToComposition(torch.autograd.Function):
    """C_final = F(Omega_c): n_steps of the step from the equilibrium of C0,
    with the state checkpointed every `every` steps for the reverse pass."""

    @staticmethod
    def forward(ctx, omega: torch.Tensor, sim: Context, C0: np.ndarray, n_steps: int, every: int):
        stream = torch.cuda.current_stream(omega.device)
        sim.bind_stream(stream.cuda_stream)
        om = omega.detach().to(torch.float64).contiguous()
        sim.set_wetting_device(om.data_ptr())
        sim.init(C0)
        sim.forward_ckpt(n_steps, every)
        C = torch.empty(sim.n_nodes, dtype=torch.float64, device=omega.device)
        sim.read_device("C", C.data_ptr())
        ctx.sim = sim
        ctx.run = sim.adjoint_run()
        return C

    @staticmethod
    def backward(ctx, grad_C: torch.Tensor):
        sim = ctx.sim
        if sim.adjoint_run() != ctx.run:
            raise RuntimeError("the Context was stepped, re-initialised or run forward again since this "
                               "composition was computed; its checkpoints are gone (call composition_after again)")
        g = grad_C.detach().to(torch.float64).contiguous()
        out = torch.empty_like(g)
        sim.bind_stream(torch.cuda.current_stream(g.device).cuda_stream)
        sim.backward(g.data_ptr(), out.data_ptr())
        return out, None, None, None, None


def composition_after(omega: torch.Tensor, sim: Context, C0, n_steps: int, every: int) -> torch.Tensor:
    """Differentiable C after n_steps as a function of omega (float64, on the GPU)."""
    return WettingToComposition.apply(omega, sim, np.asarray(C0, dtype=np.float64), int(n_steps), int(every))
