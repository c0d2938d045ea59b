"""GPU parity at the full workload sizes, in the launch configuration the
benchmark uses: bit-exact decode compared on the device, y against the
oracle's FP64 product over every row (the C oracle takes well under a second
per product at these sizes)."""
import numpy as np
import pytest

import oracle
import workloads
from gpu_common import TOL, check_spmv, need_gpu, progress, rel_error

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2603_01915_amd")


def decode_equal(torch, A, rp, ci, v):
    r2, c2, v2 = A.decode_csr()
    dt = torch.int64 if v.dtype == np.float64 else torch.int32
    ok = (torch.equal(r2, torch.from_numpy(rp).cuda())
          and torch.equal(c2, torch.from_numpy(ci).cuda())
          and torch.equal(v2.view(dt), torch.from_numpy(v).cuda().view(dt)))
    return ok


@pytest.fixture(scope="module")
def stencil():
    progress("generating the 128^3 stencil")
    return workloads.stencil27(128)


def test_band_full():
    torch = need_gpu()
    rp, ci, v = workloads.band()
    A = P.Matrix.from_csr(rp, ci, v, 4096)
    assert decode_equal(torch, A, rp, ci, v)
    x = workloads.vector(4096, 1)
    check_spmv(A.spmv(torch.from_numpy(x).cuda()).cpu().numpy(), rp, ci, v, x, None, 1, 0, np.float64)


def test_stencil_full_row_layout(stencil):
    torch = need_gpu()
    rp, ci, v = stencil
    n = 128 ** 3
    progress("encode stencil (row layout)")
    A = P.Matrix.from_csr(rp, ci, v, n, layout="row")
    progress("decode stencil on the GPU")
    assert decode_equal(torch, A, rp, ci, v)
    x = workloads.vector(n, 2)
    progress("spmv stencil")
    xd = torch.from_numpy(x).cuda()
    yd = A.spmv(xd)
    y = yd.cpu().numpy()
    err = check_spmv(y, rp, ci, v, x, None, 1.0, 0.0, np.float64)
    progress("stencil rel error %.3g" % err)
    # the LDS-ring SpMV gives the same y bit for bit
    A.set_launch(stream_stage=P.STAGE_RING)
    assert torch.equal(A.spmv(xd), yd)
    B = P.CsrBaseline(rp, ci, v, n)
    check_spmv(B.spmv(torch.from_numpy(x).cuda()).cpu().numpy(), rp, ci, v, x, None, 1, 0,
               np.float64)


def test_stencil_full_nnz_layout(stencil):
    torch = need_gpu()
    rp, ci, v = stencil
    n = 128 ** 3
    A = P.Matrix.from_csr(rp, ci, v, n, layout="nnz", lane_nnz=128)
    assert decode_equal(torch, A, rp, ci, v)
    x = workloads.vector(n, 2)
    check_spmv(A.spmv(torch.from_numpy(x).cuda()).cpu().numpy(), rp, ci, v, x, None, 1, 0,
               np.float64)


@pytest.fixture(scope="module")
def pruned():
    progress("generating the pruned 11008 x 4096 weight")
    return workloads.pruned_weight()


def test_pruned_full(pruned):
    torch = need_gpu()
    rp, ci, v = pruned
    m, n = 11008, 4096
    A = P.Matrix.from_csr(rp, ci, v, n)
    assert decode_equal(torch, A, rp, ci, v)
    x = workloads.vector(n, 4, np.float32)
    check_spmv(A.spmv(torch.from_numpy(x).cuda()).cpu().numpy(), rp, ci, v, x, None, 1, 0,
               np.float32)
    for k in (8, 32):
        progress("pruned spmm k=%d" % k)
        X = workloads.vector(n, 4, np.float32, k=k)
        Y = A.spmm(torch.from_numpy(X).cuda()).cpu().numpy()
        Yref = oracle.spmm(rp, ci, v, X)
        for c in range(0, k, 7):
            scale = oracle.absmv(rp, ci, v, X[:, c])
            assert rel_error(Y[:, c], Yref[:, c], scale) <= TOL[np.float32]
    progress("pruned spmm_t k=16")
    dY = workloads.vector(m, 5, np.float32, k=16)
    dX = A.spmm_t(torch.from_numpy(dY).cuda()).cpu().numpy()
    import scipy.sparse as sp
    At = sp.csr_matrix((v.astype(np.float64), ci, rp), shape=(m, n)).T.tocsr()
    At.sort_indices()
    for c in range(0, 16, 5):
        ref = oracle.spmtv(rp, ci, v, n, dY[:, c])
        scale = oracle.absmv(At.indptr, At.indices, At.data, dY[:, c])
        assert rel_error(dX[:, c], ref, scale) <= TOL[np.float32]
