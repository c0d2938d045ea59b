"""Differentiable product with a dtANS-compressed matrix.

``DtansLinearFn.apply(A, X)`` computes ``Y = A @ X`` for an encoded matrix A
([m, n]) and a dense X ([n, k] or [n]); its backward computes
``dX = A^T @ dY`` by decode-and-scatter over the same compressed streams
(``dtans_spmm_t``).  The matrix itself is a constant: there is no gradient with
respect to A.  Both directions run in the library's HIP kernels; this module
only wires them into ``torch.autograd``.
"""
from __future__ import annotations

import torch

from . import Matrix


class DtansLinearFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, A: Matrix, X: torch.Tensor) -> torch.Tensor:
        ctx.A = A
        ctx.vector = X.dim() == 1
        X2 = X.reshape(-1, 1) if ctx.vector else X
        X2 = X2.contiguous()
        Y = A.spmm(X2)
        return Y.reshape(-1) if ctx.vector else Y

    @staticmethod
    def backward(ctx, dY: torch.Tensor):
        if not ctx.needs_input_grad[1]:
            return None, None
        dY2 = dY.reshape(-1, 1) if ctx.vector else dY
        dX = ctx.A.spmm_t(dY2.contiguous())
        return None, (dX.reshape(-1) if ctx.vector else dX)


class DtansLinear(torch.nn.Module):
    """A fixed sparse linear map y = A x stored in CSR-dtANS (batched inputs
    are [batch, n] and give [batch, m], like ``torch.nn.Linear`` without bias)."""

    def __init__(self, A: Matrix):
        super().__init__()
        self.A = A

    def forward(self, x: torch.Tensor) -> torch.Tensor:
        if x.dim() == 1:
            return DtansLinearFn.apply(self.A, x)
        # [batch, n] -> X = x^T [n, batch] -> Y [m, batch] -> [batch, m]
        Y = DtansLinearFn.apply(self.A, x.t().contiguous())
        return Y.t()
