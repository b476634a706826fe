"""torch.autograd.Function wrappers over the library's energy and reweighting kernels.

EnergyFn:   E_s = E(x_s; theta) for stored configurations x [n_cfg, N, 3] (float32, device) and
            theta = (C_AB, C_BB, kappa_bend, kappa_tors) (float64); backward runs the hand-written
            dE/dx and dE/dtheta kernel.
ReweightFn: (<E>_T, C_V(T)) for temperatures T from energies E_s and fixed sampling weights
            ln W0_s (canonical reweighting of MUCA samples); backward gives dL/dE_s.
Chaining them differentiates reweighted canonical averages with respect to the couplings.
torch only provides device memory and the stream; all arithmetic runs in the HIP library.
"""
from __future__ import annotations

import numpy as np
import torch

from . import Muca, reweight_bwd, reweight_fwd, reweight_workspace_bytes


def _stream():
    return torch.cuda.current_stream().cuda_stream


class EnergyFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x: torch.Tensor, theta: torch.Tensor, muca: Muca, sys: int = 0):
        assert x.is_cuda and x.dtype == torch.float32 and x.is_contiguous()
        th = theta.detach().to("cpu", torch.float64).numpy()
        E = torch.empty(x.shape[0], dtype=torch.float64, device=x.device)
        torch.cuda.current_stream().synchronize()
        muca.energy_fwd_ptr(sys, x.data_ptr(), x.shape[0], th, E.data_ptr())
        muca.synchronize()
        ctx.save_for_backward(x)
        ctx.th = th
        ctx.muca = muca
        ctx.sys = sys
        ctx.theta_device = theta.device
        return E

    @staticmethod
    def backward(ctx, gE: torch.Tensor):
        (x,) = ctx.saved_tensors
        gE = gE.contiguous().to(torch.float64)
        gx = torch.empty_like(x)
        gth = torch.zeros(4, dtype=torch.float64, device=x.device)
        torch.cuda.current_stream().synchronize()
        ctx.muca.energy_bwd_ptr(ctx.sys, x.data_ptr(), x.shape[0], ctx.th, gE.data_ptr(),
                                gx.data_ptr(), gth.data_ptr())
        ctx.muca.synchronize()
        return gx, gth.to(ctx.theta_device), None, None


class ReweightFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, E: torch.Tensor, lnw0: torch.Tensor, temps):
        assert E.is_cuda and E.dtype == torch.float64 and lnw0.dtype == torch.float64
        E = E.contiguous()
        lnw0 = lnw0.contiguous()
        t = np.ascontiguousarray(np.asarray(temps, dtype=np.float64))
        n, nt = E.shape[0], len(t)
        mean = torch.empty(nt, dtype=torch.float64, device=E.device)
        cv = torch.empty_like(mean)
        mom = torch.empty(nt, 3, dtype=torch.float64, device=E.device)
        ws = torch.empty(reweight_workspace_bytes(n, nt), dtype=torch.uint8, device=E.device)
        reweight_fwd(E.data_ptr(), lnw0.data_ptr(), n, t, mean.data_ptr(), cv.data_ptr(),
                     mom.data_ptr(), ws.data_ptr(), ws.numel(), _stream())
        ctx.save_for_backward(E, lnw0, mom)
        ctx.t = t
        return mean, cv

    @staticmethod
    def backward(ctx, g_mean, g_cv):
        E, lnw0, mom = ctx.saved_tensors
        nt = len(ctx.t)
        if g_mean is None:
            g_mean = torch.zeros(nt, dtype=torch.float64, device=E.device)
        if g_cv is None:
            g_cv = torch.zeros(nt, dtype=torch.float64, device=E.device)
        g_mean = g_mean.contiguous().to(torch.float64)
        g_cv = g_cv.contiguous().to(torch.float64)
        gE = torch.empty_like(E)
        reweight_bwd(E.data_ptr(), lnw0.data_ptr(), E.shape[0], ctx.t, mom.data_ptr(),
                     g_mean.data_ptr(), g_cv.data_ptr(), gE.data_ptr(), _stream())
        return gE, None, None


def reweighted_observables(x, theta, lnw0, temps, muca: Muca, sys: int = 0):
    """(<E>_T, C_V(T)) of stored configurations under couplings theta, differentiable in theta."""
    E = EnergyFn.apply(x, theta, muca, sys)
    return ReweightFn.apply(E, lnw0, temps)
