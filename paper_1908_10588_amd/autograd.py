"""torch.autograd.Function wrappers around the library's hand-written adjoints.

Complex tensors are planar float64 torch tensors [2, ...]; the gradient torch
accumulates for such a tensor is [df/dRe, df/dIm], which is exactly the
library's cotangent convention zbar = df/dRe + i df/dIm in planar form.  The
MPO operators are fixed (tdmrg_wop handles); their cotangents are available
from tdmrg_heff2_apply_vjp / tdmrg_local_expm_vjp directly.
"""
import torch

from . import (HeffShape, tdmrg_heff2_apply, tdmrg_heff2_apply_vjp, tdmrg_local_expm,
               tdmrg_local_expm_vjp)


class _Heff2(torch.autograd.Function):
    @staticmethod
    def forward(ctx_, lib_ctx, shape, L, W1, W2, R, theta):
        y = torch.empty_like(theta)
        tdmrg_heff2_apply(lib_ctx, shape, L.contiguous(), W1, W2, R.contiguous(), theta.contiguous(), y)
        ctx_.save_for_backward(L, R, theta)
        ctx_.meta = (lib_ctx, shape, W1, W2)
        return y

    @staticmethod
    def backward(ctx_, ybar):
        L, R, theta = ctx_.saved_tensors
        lib_ctx, shape, W1, W2 = ctx_.meta
        Lb = torch.empty_like(L) if ctx_.needs_input_grad[2] else None
        Rb = torch.empty_like(R) if ctx_.needs_input_grad[5] else None
        tb = torch.empty_like(theta) if ctx_.needs_input_grad[6] else None
        tdmrg_heff2_apply_vjp(lib_ctx, shape, L, W1, W2, R, theta, ybar.contiguous(), Lbar=Lb,
                              Rbar=Rb, thetabar=tb)
        return None, None, Lb, None, None, Rb, tb


class _LocalExpm(torch.autograd.Function):
    @staticmethod
    def forward(ctx_, lib_ctx, shape, L, W1, W2, R, theta, tau, tol, m_max, nquad):
        y = theta.detach().clone().contiguous()
        tdmrg_local_expm(lib_ctx, shape, True, L.contiguous(), W1, W2, R.contiguous(), y, tau,
                         tol=tol, m_max=m_max)
        ctx_.save_for_backward(L, R, theta)
        ctx_.meta = (lib_ctx, shape, W1, W2, tau, tol, m_max, nquad)
        return y

    @staticmethod
    def backward(ctx_, ybar):
        L, R, theta = ctx_.saved_tensors
        lib_ctx, shape, W1, W2, tau, tol, m_max, nquad = ctx_.meta
        Lb = torch.empty_like(L) if ctx_.needs_input_grad[2] else None
        Rb = torch.empty_like(R) if ctx_.needs_input_grad[5] else None
        tb = torch.empty_like(theta) if ctx_.needs_input_grad[6] else None
        tdmrg_local_expm_vjp(lib_ctx, shape, L, W1, W2, R, theta, tau, ybar.contiguous(), Lbar=Lb,
                             Rbar=Rb, thetabar=tb, nquad=nquad, tol=tol, m_max=m_max)
        return None, None, Lb, None, None, Rb, tb, None, None, None, None


def heff2(lib_ctx, shape, L, W1, W2, R, theta):
    """y = H_eff,2 theta, differentiable in L, R and theta."""
    return _Heff2.apply(lib_ctx, tuple(shape), L, W1, W2, R, theta)


def local_expm(lib_ctx, shape, L, W1, W2, R, theta, tau, tol=1e-14, m_max=60, nquad=10):
    """exp(-i tau H_eff,2) theta, differentiable in L, R and theta."""
    return _LocalExpm.apply(lib_ctx, tuple(shape), L, W1, W2, R, theta, float(tau), float(tol),
                            int(m_max), int(nquad))
