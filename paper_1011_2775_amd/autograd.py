"""Differentiable Wilson-clover solve x = D(U)^-1 eta with a hand-written adjoint.

Backward pass for an upstream gradient g of x (PyTorch's complex convention,
g = dL/dRe x + i dL/dIm x):

    lambda   = D^-dag g      (one adjoint solve, D^dag = gamma5 D gamma5, so
                              the forward solver and hierarchy serve)
    grad_eta = lambda
    grad_U   = -dRe<lambda, D(U) x>/dU   (hop plus clover force kernels)

Every step runs in the HIP library; this module only routes tensors.
"""
import torch

from . import MG_GCR


class WilsonCloverSolve(torch.autograd.Function):
    """x = D(U)^-1 eta.  `U` must be the gauge field loaded into `wctx`
    (Context.set_gauge / set_clover, plus the multigrid hierarchy for MG_GCR);
    it is an argument so that autograd can route its gradient."""

    @staticmethod
    def forward(fctx, eta, U, wctx, solver, tol, lat, include_clover):
        x, _ = wctx.solve(eta, solver, tol, lat=lat)
        fctx.save_for_backward(x)
        fctx.wctx, fctx.solver, fctx.tol, fctx.lat = wctx, solver, tol, lat
        fctx.include_clover = include_clover
        fctx.u_shape = U.shape
        return x

    @staticmethod
    def backward(fctx, gx):
        (x,) = fctx.saved_tensors
        lam, _ = fctx.wctx.solve_dag(gx.contiguous(), fctx.solver, fctx.tol, lat=fctx.lat)
        g_eta = lam if fctx.needs_input_grad[0] else None
        g_u = None
        if fctx.needs_input_grad[1]:
            g_u = fctx.wctx.force(x, lam, fctx.include_clover, fctx.lat).reshape(fctx.u_shape)
        return g_eta, g_u, None, None, None, None, None


def solve(wctx, eta, U, solver=MG_GCR, tol=1e-10, lat=0, include_clover=True):
    """Differentiable x = D(U)^-1 eta (eta: [nrhs][Lt][Lz][Ly][Lx][4][3] complex128 on the GPU;
    U: the canonical gauge field held by `wctx`)."""
    return WilsonCloverSolve.apply(eta, U, wctx, solver, tol, lat, include_clover)
