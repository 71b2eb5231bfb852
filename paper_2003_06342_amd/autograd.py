"""torch.autograd bridge of the HIP forward step and its hand-written adjoint.

``LBMRun.apply(phi0, Tw, prm, T0, nsteps, storage, tape)`` runs the 2-D film
step nsteps times from (phi0, T0) with the wall-temperature row Tw on the
heated floor (face y = 0) and returns (phi^N, T^N); its backward calls the
library's reverse sweep (tape "sqrt": sqrt(T) checkpointing, "binomial":
binomial checkpointing, less memory and more recomputation) with the
incoming dL/dphi^N and dL/dT^N and returns dL/dphi0 and dL/dTw.  Every
operation runs in liblbm.so; torch only holds the tensors.
"""
from __future__ import annotations

import torch

from . import lbm


class LBMRun(torch.autograd.Function):
    @staticmethod
    def forward(ctx, phi0, Tw, prm, T0, nsteps: int, storage: str = "f32", tape: str = "sqrt"):
        policy = {"sqrt": lbm.LBM_TAPE_SQRT, "binomial": lbm.LBM_TAPE_BINOMIAL}[tape]
        sim = lbm.Sim(prm, storage, device=str(phi0.device))
        sim.set_wall_T(1, 0, Tw.detach())
        sim.init(phi0.detach(), T0)
        sim.forward_taped(int(nsteps), policy)
        f = sim.fields(("phi", "T"))
        phiN = f["phi"][0].clone()
        TN = f["T"][0].clone()
        ctx.sim = sim
        return phiN.to(phi0.dtype), TN.to(phi0.dtype)

    @staticmethod
    def backward(ctx, gphi, gT):
        g = ctx.sim.backward(None if gphi is None else gphi.detach().to(torch.float64),
                             tw_face=(1, 0),
                             gT=None if gT is None else gT.detach().to(torch.float64))
        ctx.sim.close()
        dphi0 = g["phi0"].reshape(1, *g["phi0"].shape)
        return dphi0, g["Tw"], None, None, None, None, None
