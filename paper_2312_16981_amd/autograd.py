"""torch.autograd binding of the adjoint of the frozen-tally macroscopic map.

MaterialEnergy.apply(kappa, prob, nsteps) runs `nsteps` steps of the problem
`prob` with opacity `kappa` ([ncell][G] float64 CUDA tensor) on the GPU,
recording them, and returns J = sum_i V_i C_v,i T_i after the last step.
Its backward is ugkwp_adjoint: dJ/dkappa with the particle-phase results of the
recorded run held fixed (net particle flux, survivor density, sampled flags).
Marshalling only: the forward steps and the reverse sweep run in libugkwp.so.
"""
import numpy as np
import torch

from . import ugkwp


class MaterialEnergy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, kappa, prob, nsteps):
        if kappa.dtype != torch.float64 or not kappa.is_cuda:
            raise TypeError("kappa must be a float64 CUDA tensor")
        stream = torch.cuda.current_stream(kappa.device)
        c = ugkwp.from_problem(prob.with_(kappa=kappa.detach().cpu().numpy()), stream=stream.cuda_stream)
        c.record(nsteps)
        c.step(nsteps)
        T = torch.empty(prob.ncell, dtype=torch.float64, device=kappa.device)
        c.get_fields_device(None, T.data_ptr(), inst=0)
        V = (prob.x1 - prob.x0) / prob.nx * ((prob.y1 - prob.y0) / prob.ny if prob.dim == 2 else 1.0)
        w = torch.as_tensor(V * np.asarray(prob.cv, dtype=np.float64), device=kappa.device)
        ctx.c = c
        ctx.w = w
        ctx.shape = kappa.shape
        return (w * T).sum()

    @staticmethod
    def backward(ctx, gJ):
        dJdT = (ctx.w * gJ).contiguous()
        grad = torch.empty(ctx.shape, dtype=torch.float64, device=dJdT.device)
        ctx.c.adjoint_device(dJdT.data_ptr(), grad.data_ptr())
        return grad, None, None
