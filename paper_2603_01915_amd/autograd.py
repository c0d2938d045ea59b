"""Differentiable product with a dtANS-compressed matrix.

``DtansLinearFn.apply(A, X, At=None)`` computes ``Y = A @ X`` for an encoded
matrix A ([m, n]) and a dense X ([n, k] or [n]).  Its backward computes
``dX = A^T @ dY`` in one of two ways:

* without ``At``: decode-and-scatter over A's own compressed streams
  (``dtans_spmm_t``), so the matrix is stored once;
* with ``At``, a second encoded matrix holding A^T ([n, m]): a plain product
  ``At @ dY`` on it, with one writer per output row and no atomic adds,
  at the price of storing the transpose as well (the same trade a CSR user
  makes by keeping an explicit transpose).

The matrix itself is a constant: there is no gradient with respect to A.  Both
directions run in the library's HIP kernels; this module only wires them into
``torch.autograd``.
"""
from __future__ import annotations

from typing import Optional

import numpy as np
import torch

from . import Matrix, _np


def transpose_csr(row_ptr, col, vals, n: int):
    """The CSR arrays of the transpose of an [m, n] CSR matrix (a counting sort
    of the nonzeros by column; within a column, rows stay in increasing
    order).  Host-side preprocessing for the encoder, not part of any product."""
    rp = _np(row_ptr, np.int64)
    ci = _np(col, np.int64)
    v = _np(vals)
    m = len(rp) - 1
    if len(ci) and (ci.min() < 0 or ci.max() >= n):
        raise ValueError("column index out of range [0, %d)" % n)
    rows = np.repeat(np.arange(m, dtype=np.int64), np.diff(rp))
    order = np.argsort(ci, kind="stable")
    rpt = np.zeros(n + 1, np.int64)
    np.cumsum(np.bincount(ci, minlength=n), out=rpt[1:])
    return rpt.astype(np.int32), rows[order].astype(np.int32), v[order]


class DtansLinearFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, A: Matrix, X: torch.Tensor, At: Optional[Matrix] = None) -> torch.Tensor:
        if At is not None and At.shape != (A.shape[1], A.shape[0]):
            raise ValueError("At has shape %s, expected %s" % (At.shape, (A.shape[1], A.shape[0])))
        ctx.A, ctx.At = A, At
        ctx.vector = X.dim() == 1
        X2 = X.reshape(-1, 1) if ctx.vector else X
        X2 = X2.contiguous()
        Y = A.spmm(X2)
        return Y.reshape(-1) if ctx.vector else Y

    @staticmethod
    def backward(ctx, dY: torch.Tensor):
        if not ctx.needs_input_grad[1]:
            return None, None, None
        dY2 = dY.reshape(-1, 1) if ctx.vector else dY
        dY2 = dY2.contiguous()
        dX = ctx.At.spmm(dY2) if ctx.At is not None else ctx.A.spmm_t(dY2)
        return None, (dX.reshape(-1) if ctx.vector else dX), None


class DtansLinear(torch.nn.Module):
    """A fixed sparse linear map y = A x stored in CSR-dtANS (batched inputs
    are [batch, n] and give [batch, m], like ``torch.nn.Linear`` without bias).
    ``At``, an encoded A^T, makes the backward a plain product on it."""

    def __init__(self, A: Matrix, At: Optional[Matrix] = None):
        super().__init__()
        self.A = A
        self.At = At

    @classmethod
    def from_csr(cls, row_ptr, col, vals, n: int, transposed_copy: bool = False,
                 **encode_opts) -> "DtansLinear":
        """Encode A (and, with ``transposed_copy``, A^T with the same options)."""
        A = Matrix.from_csr(row_ptr, col, vals, n, **encode_opts)
        At = None
        if transposed_copy:
            rpt, cit, vt = transpose_csr(row_ptr, col, vals, n)
            At = Matrix.from_csr(rpt, cit, vt, len(_np(row_ptr)) - 1, **encode_opts)
        return cls(A, At)

    def forward(self, x: torch.Tensor) -> torch.Tensor:
        if x.dim() == 1:
            return DtansLinearFn.apply(self.A, x, self.At)
        # [batch, n] -> X = x^T [n, batch] -> Y [m, batch] -> [batch, m]
        Y = DtansLinearFn.apply(self.A, x.t().contiguous(), self.At)
        return Y.t()
