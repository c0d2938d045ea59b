"""Autograd: forward A X and backward A^T dY (decode-and-scatter, or a product
on an encoded transpose) checked with torch.autograd.gradcheck in FP64,
central differences in FP64 on the pruned weight, and the oracle's A^T dy."""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import workloads
from gpu_common import TOL, need_gpu, progress, rel_error

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2603_01915_amd")


def test_gradcheck_small():
    torch = need_gpu()
    from paper_2603_01915_amd.autograd import DtansLinearFn, transpose_csr

    rng = np.random.default_rng(12)
    m, n = 96, 80
    rows = [sorted(rng.choice(n, size=7, replace=False)) for _ in range(m)]
    rp = np.arange(0, 7 * m + 1, 7, dtype=np.int32)
    ci = np.array([c for r in rows for c in r], np.int32)
    v = rng.standard_normal(len(ci))
    for layout, T in (("row", 0), ("nnz", 12)):
        progress("gradcheck %s" % layout)
        A = P.Matrix.from_csr(rp, ci, v, n, layout=layout, lane_nnz=T)
        X = torch.randn(n, 3, dtype=torch.float64, device="cuda", requires_grad=True)
        # the backward scatters with atomic adds: repeated backwards may differ
        # in the last bits, hence nondet_tol
        assert torch.autograd.gradcheck(lambda X: DtansLinearFn.apply(A, X), (X,), eps=1e-6,
                                        atol=1e-9, rtol=1e-7, nondet_tol=1e-12)
        x = torch.randn(n, dtype=torch.float64, device="cuda", requires_grad=True)
        assert torch.autograd.gradcheck(lambda x: DtansLinearFn.apply(A, x), (x,), eps=1e-6,
                                        atol=1e-9, rtol=1e-7, nondet_tol=1e-12)
        # with an encoded transpose the backward has one writer per entry
        rpt, cit, vt = transpose_csr(rp, ci, v, n)
        At = P.Matrix.from_csr(rpt, cit, vt, m, layout=layout, lane_nnz=T)
        assert torch.autograd.gradcheck(lambda X: DtansLinearFn.apply(A, X, At), (X,), eps=1e-6,
                                        atol=1e-9, rtol=1e-7)
        assert torch.autograd.gradcheck(lambda x: DtansLinearFn.apply(A, x, At), (x,), eps=1e-6,
                                        atol=1e-9, rtol=1e-7)


@pytest.mark.parametrize("transposed_copy", [False, True])
def test_pruned_forward_backward_against_oracle(transposed_copy):
    """The pruned 11008 x 4096 BF16-valued weight, batch 16 FP32; the backward
    by decode-and-scatter or on an encoded transpose."""
    torch = need_gpu()
    from paper_2603_01915_amd.autograd import DtansLinearFn, transpose_csr

    rp, ci, v = workloads.pruned_weight()
    m, n = 11008, 4096
    A = P.Matrix.from_csr(rp, ci, v, n)
    At = P.Matrix.from_csr(*transpose_csr(rp, ci, v, n), m) if transposed_copy else None
    X = torch.from_numpy(workloads.vector(n, 5, np.float32, k=16)).cuda().requires_grad_(True)
    dY = workloads.vector(m, 6, np.float32, k=16)
    progress("pruned forward/backward, transposed copy %s" % transposed_copy)
    Y = DtansLinearFn.apply(A, X, At)
    Y.backward(torch.from_numpy(dY).cuda())
    Yh = Y.detach().cpu().numpy()
    dX = X.grad.cpu().numpy()
    Xh = X.detach().cpu().numpy()
    St = sp.csr_matrix((v.astype(np.float64), ci, rp), shape=(m, n)).T.tocsr()
    St.sort_indices()
    for c in range(0, 16, 3):
        y_ref = oracle.spmv(rp, ci, v, Xh[:, c])
        assert rel_error(Yh[:, c], y_ref, oracle.absmv(rp, ci, v, Xh[:, c])) <= TOL[np.float32]
        g_ref = oracle.spmtv(rp, ci, v, n, dY[:, c])
        scale = oracle.absmv(St.indptr, St.indices, St.data, dY[:, c])
        assert rel_error(dX[:, c], g_ref, scale) <= TOL[np.float32]


def test_pruned_central_differences_fp64():
    """Central differences of L(X) = <dY, A X> in FP64 (the FP64 copy of the
    BF16-valued weight is exact) on sampled coordinates: dL/dX[j, b] is
    (A^T dY)[j, b]; L is linear, so the difference quotient is exact up to
    rounding."""
    torch = need_gpu()
    from paper_2603_01915_amd.autograd import DtansLinearFn

    rp, ci, v = workloads.pruned_weight()
    m, n = 11008, 4096
    v64 = v.astype(np.float64)
    A = P.Matrix.from_csr(rp, ci, v64, n)
    X = torch.from_numpy(workloads.vector(n, 5, np.float64, k=16)).cuda().requires_grad_(True)
    dY = torch.from_numpy(workloads.vector(m, 6, np.float64, k=16)).cuda()
    Y = DtansLinearFn.apply(A, X)
    Y.backward(dY)
    grad = X.grad.detach()
    rng = np.random.default_rng(7)
    h = 1e-3
    progress("central differences on 64 coordinates")
    with torch.no_grad():
        for _ in range(64):
            j, b = int(rng.integers(n)), int(rng.integers(16))
            Xp = X.detach().clone()
            Xm = X.detach().clone()
            Xp[j, b] += h
            Xm[j, b] -= h
            Lp = float((dY * A.spmm(Xp)).sum())
            Lm = float((dY * A.spmm(Xm)).sum())
            fd = (Lp - Lm) / (2 * h)
            g = float(grad[j, b])
            # the sums have ~m*16 terms of size ~|dY||A X|; allow their rounding
            assert abs(fd - g) <= 1e-6 * (1 + abs(g)), (j, b, fd, g)


@pytest.mark.parametrize("transposed_copy", [False, True])
def test_linear_module(transposed_copy):
    torch = need_gpu()
    from paper_2603_01915_amd.autograd import DtansLinear

    rp, ci, v = workloads.pruned_weight(rows=200, cols=128)
    # the transposed-copy case also encodes both matrices with the GPU passes
    lin = DtansLinear.from_csr(rp, ci, v, 128, transposed_copy=transposed_copy, gpu_encode=transposed_copy)
    assert (lin.At is not None) == transposed_copy
    x = torch.randn(5, 128, device="cuda", requires_grad=True)
    y = lin(x)
    assert tuple(y.shape) == (5, 200)
    D = torch.from_numpy(sp.csr_matrix((v, ci, rp), shape=(200, 128)).toarray()).cuda()
    assert torch.allclose(y, x @ D.t(), rtol=1e-5, atol=1e-5)
    y.sum().backward()
    assert torch.allclose(x.grad, torch.ones(5, 200, device="cuda") @ D, rtol=1e-5, atol=1e-5)
