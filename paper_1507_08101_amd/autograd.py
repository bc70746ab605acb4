"""torch.autograd functions over the SELL-C-sigma kernels; the matrix values are parameters.

``spmm(theta, X, M)``      Y = A(theta) X. Backward: dX = A^T dY (forward kernel on the SELL
                           copy of A^T), dtheta_p = sum_j dY[row_p, j] X[col_p, j] (pattern-
                           restricted outer product).
``chebyshev(theta, X, M, N, s, c, K)``
                           Y = T_N((A(theta) - c I) / s) X by the three-term recurrence, with the
                           adjoint recurrence in backward and recompute checkpoints every K steps.

``theta`` holds the stored values in the CSR order of the matrix's construction (float64, on
the device); a float32 matrix rounds them to the nearest float32 when they are loaded. Every
step runs in the library's HIP kernels; these classes only sequence the calls.

A matrix handle holds one set of values. Forward uploads its theta and saves it; if the
handle's values changed before backward runs (another forward on the same handle, or any
value update), backward uploads the saved theta again, so that the gradients are those of the
matrix that forward used.
"""
from __future__ import annotations

import torch

from . import (SellMatrix, cheb_ckpt_elems, sell_cheb_backward, sell_cheb_forward, sell_grad_values,
               sell_spmmv, sell_spmmv_T)


def _load_values(ctx, M: SellMatrix, theta):
    th = theta.detach().to(torch.float64).contiguous()
    M.update_values(th)
    ctx.version = M.values_version
    return th


def _restore_values(ctx, M: SellMatrix, th):
    if M.values_version != ctx.version:
        M.update_values(th)
        ctx.version = M.values_version


class _SpMM(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta, X, M: SellMatrix):
        th = _load_values(ctx, M, theta)
        Y = torch.empty((M.nrows, X.shape[1]), dtype=X.dtype, device=X.device)
        sell_spmmv(M, X.contiguous(), Y)
        ctx.save_for_backward(X, th)
        ctx.M = M
        return Y

    @staticmethod
    def backward(ctx, dY):
        X, th = ctx.saved_tensors
        M = ctx.M
        _restore_values(ctx, M, th)
        dY = dY.contiguous()
        dtheta = dX = None
        if ctx.needs_input_grad[1]:
            dX = torch.empty((M.ncols, X.shape[1]), dtype=X.dtype, device=X.device)
            sell_spmmv_T(M, dY, dX, deterministic=True)
        if ctx.needs_input_grad[0]:
            dtheta = torch.empty(M.info["nnz"], dtype=torch.float64, device=X.device)
            sell_grad_values(M, dY, X.contiguous(), dtheta)
        return dtheta, dX, None


class _Chebyshev(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta, X, M: SellMatrix, N: int, s: float, c: float, K: int):
        th = _load_values(ctx, M, theta)
        X = X.contiguous()
        n, b = X.shape
        ckpt = torch.empty(cheb_ckpt_elems(n, b, N, K), dtype=X.dtype, device=X.device)
        Y = torch.empty_like(X)
        sell_cheb_forward(M, X, Y, N, s, c, K, ckpt)
        ctx.save_for_backward(ckpt, th)
        ctx.M, ctx.N, ctx.s, ctx.c, ctx.K, ctx.shape = M, N, s, c, K, (n, b)
        return Y

    @staticmethod
    def backward(ctx, dY):
        ckpt, th = ctx.saved_tensors
        M = ctx.M
        _restore_values(ctx, M, th)
        dY = dY.contiguous()
        dX = torch.empty(ctx.shape, dtype=dY.dtype, device=dY.device)
        dtheta = torch.empty(M.info["nnz"], dtype=torch.float64, device=dY.device)
        sell_cheb_backward(M, dY, ctx.N, ctx.s, ctx.c, ctx.K, ckpt, dX, dtheta)
        return dtheta, dX, None, None, None, None, None


def spmm(theta, X, M: SellMatrix):
    return _SpMM.apply(theta, X, M)


def chebyshev(theta, X, M: SellMatrix, N: int, s: float, c: float = 0.0, K: int = 10):
    return _Chebyshev.apply(theta, X, M, N, s, c, K)
