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


class _PopulationGrad(torch.autograd.Function):
    """P_state(T) after `steps` 2TDVP steps as a function of the coupling
    constants; one library call runs the forward evolution and its adjoint
    (tdmrg_tdvp2_population_grad), and backward scales the stored gradient."""

    @staticmethod
    def forward(ctx_, lib_ctx, template, run, E, V, omega, g1, g2):
        from . import tdmrg_tdvp2_population_grad
        model = dict(template)
        for name, t in (("E", E), ("V", V), ("omega", omega), ("g1", g1), ("g2_val", g2)):
            model[name] = t.detach().cpu().double().numpy().copy()
        out = tdmrg_tdvp2_population_grad(lib_ctx, model, model["occ"], run["D_cap"], run["steps"], run["dt_fs"],
                                          run["D_max"], run["eps"], run["state"], nquad=run["nquad"])
        grads = [torch.as_tensor(out[k]).to(dtype=t.dtype, device=t.device).reshape(t.shape)
                 for k, t in (("E", E), ("V", V), ("omega", omega), ("g1", g1), ("g2", g2))]
        ctx_.grads = grads
        ctx_.info = {k: out[k] for k in ("ranks", "seconds_forward", "seconds_total", "mean_nodes")}
        return torch.tensor(out["pop"], dtype=E.dtype, device=E.device)

    @staticmethod
    def backward(ctx_, gout):
        return (None, None, None) + tuple(gout * g for g in ctx_.grads)


def population(lib_ctx, model, E, V, omega, g1, g2, steps, dt_fs, D_max, eps, state, D_cap=None, nquad=12):
    """Electronic population P_state after `steps` symmetric 2TDVP steps from
    the model's product state, differentiable in the coupling constants (the
    vibronic Hamiltonian of Section 2.2: E [n_el], V [n_el, n_el], omega
    [n_modes], g1 [n_modes, n_el, n_el], g2 [n_g2]; the remaining fields of
    `model` fix the structure).  The gradients are the library's: V and g1
    carry one constant per unordered state pair, reported symmetric (so a
    symmetric perturbation dV with dV_ij = dV_ji = d changes P by grad_ij d),
    and they are taken at the truncation ranks the forward run chose."""
    run = dict(D_cap=D_cap or D_max, steps=int(steps), dt_fs=float(dt_fs), D_max=int(D_max), eps=float(eps),
               state=int(state), nquad=int(nquad))
    return _PopulationGrad.apply(lib_ctx, model, run, E, V, omega, g1, g2)
