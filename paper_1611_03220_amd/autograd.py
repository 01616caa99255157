"""Differentiable KRR solve on the HIP library (torch.autograd Functions).

KRRSolve:      alpha = (K(X; sigma) + lambda I)^{-1} Y by preconditioned CG (Eq. 1, Alg. 1).
               Backward solves the adjoint system with the same preconditioner,
               abar = (K + lambda I)^{-1} dL/dalpha (the matrix is symmetric), and returns
                 dL/dY      = abar,
                 dL/dlambda = -<abar, alpha>,
                 dL/dsigma  = -<abar, (dK/dsigma) alpha>   (one matrix-free dK/dsigma product).
               The preconditioner (Z, Ut) is treated as a constant: the exact solution does not
               depend on it, only the iteration count does.
               dL/dsigma is the difference of two terms that nearly cancel (here by two orders of
               magnitude), so its dK/dsigma products run in `deriv_prec`, FP64 by default, while
               both solves may run mixed. Mixed dK/dsigma products (errors about 1e-7 of each
               term, the factor D of dK/dsigma carrying the FP32 distance's absolute error) keep
               the gradient within 5e-6 of the oracle's on the 147-class recipe, but miss 1e-4
               (3.7e-4) on a 20-class recipe whose terms cancel by about 3.5 orders.
KernelMatmat:  OUT = K(X1, X2; sigma) V (e.g. validation predictions; the loss below runs this
               forward product in FP64 because the validation residual cancels). Backward:
                 dL/dV     = K(X2, X1) G,
                 dL/dsigma = <G, (dK/dsigma) V>   (krr_kernel_dsigma_inner, FP64 sum).
All arithmetic runs in libkrr; these classes only route tensors.
"""
from __future__ import annotations

import torch

from . import krr


def _scalar(t) -> float:
    return float(t.detach().cpu()) if isinstance(t, torch.Tensor) else float(t)


class KRRSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, sigma, lam, X, Y, Ut, opts):
        s, l = _scalar(sigma), _scalar(lam)
        opts = dict(opts)
        ctx.deriv_prec = opts.pop("deriv_prec", None) or "fp64"
        alpha, rep = krr.pcg_solve(X, s, l, Ut, Y, **opts)
        ctx.save_for_backward(X, alpha, Ut if Ut is not None else torch.empty(0, device=X.device))
        ctx.sig, ctx.lam, ctx.opts, ctx.has_u = s, l, opts, Ut is not None
        ctx.report = rep
        return alpha

    @staticmethod
    def backward(ctx, g):
        X, alpha, Ut = ctx.saved_tensors
        Ut = Ut if ctx.has_u else None
        abar, _ = krr.pcg_solve(X, ctx.sig, ctx.lam, Ut, g.contiguous().to(torch.float64),
                                **ctx.opts)
        ds, dl = krr.grad(X, ctx.sig, alpha, abar, prec=ctx.deriv_prec)
        dev = alpha.device
        gs = torch.tensor(ds, dtype=torch.float64, device=dev)
        gl = torch.tensor(dl, dtype=torch.float64, device=dev)
        return gs, gl, None, abar, None, None


class KernelMatmat(torch.autograd.Function):
    @staticmethod
    def forward(ctx, sigma, X1, X2, V, prec, deriv_prec, fwd_prec):
        s = _scalar(sigma)
        out = krr.kernel_matmat(X1, X2, s, V, prec=fwd_prec or prec)
        ctx.save_for_backward(X1, X2, V)
        ctx.sig, ctx.prec, ctx.deriv_prec = s, prec, deriv_prec
        return out

    @staticmethod
    def backward(ctx, G):
        X1, X2, V = ctx.saved_tensors
        G = G.contiguous()
        gV = krr.kernel_matmat(X2, X1, ctx.sig, G, prec=ctx.prec)
        ds = krr.kernel_dsigma_inner(X1, X2, ctx.sig, V, G, prec=ctx.deriv_prec)
        gs = torch.tensor(ds, dtype=torch.float64, device=V.device)
        return gs, None, None, gV, None, None, None


def krr_solve(X, Y, sigma, lam, Ut=None, **opts):
    """Differentiable alpha = (K(X; sigma) + lam I)^{-1} Y. `sigma`, `lam` may be 0-dim
    FP64 tensors with requires_grad; Y an FP64 tensor (gradient = adjoint solution)."""
    opts.setdefault("raise_on_error", True)
    if Ut is None:
        opts["use_precond"] = False
    return KRRSolve.apply(sigma, lam, X, Y, Ut, opts)


def kernel_matmat(X1, X2, sigma, V, prec="f16x3", deriv_prec="fp64", fwd_prec=None):
    """Differentiable K(X1, X2; sigma) V: forward in `fwd_prec` (default `prec`), the
    transposed product of the backward in `prec`, dK/dsigma products in `deriv_prec`."""
    return KernelMatmat.apply(sigma, X1, X2, V, prec, deriv_prec, fwd_prec)


def validation_loss(Xtr, Ytr, Xv, Yv, sigma, lam, Ut=None, prec="f16x3", deriv_prec="fp64",
                    pred_prec="fp64", **opts):
    """L = 1/2 ||K(Xv, Xtr) alpha - Yv||_F^2 with alpha from the differentiable solve.
    The residual K(Xv, Xtr) alpha - Yv cancels most of the prediction when the model fits,
    so the prediction product runs in `pred_prec` (FP64 by default); the solves and the
    transposed product of the backward run in `prec`, the dK/dsigma products in
    `deriv_prec` (FP64 by default)."""
    alpha = krr_solve(Xtr, Ytr, sigma, lam, Ut, prec=prec, deriv_prec=deriv_prec, **opts)
    pred = kernel_matmat(Xv, Xtr, sigma, alpha, prec=prec, deriv_prec=deriv_prec,
                         fwd_prec=pred_prec)
    return 0.5 * ((pred - Yv) ** 2).sum()
