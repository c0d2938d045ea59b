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
        check_all_columns(Y, rp, ci, v, X)
    progress("pruned spmm_t k=16")
    dY = workloads.vector(m, 5, np.float32, k=16)
    dX = A.spmm_t(torch.from_numpy(dY).cuda()).cpu().numpy()
    import scipy.sparse as sp
    At = sp.csr_matrix((v.astype(np.float64), ci, rp), shape=(m, n)).T.tocsr()
    At.sort_indices()
    check_all_columns(dX, At.indptr.astype(np.int32), At.indices.astype(np.int32), At.data, dY)


def check_all_columns(Y, rp, ci, v, X, Y0=None, alpha=1.0, beta=0.0, dtype=np.float32):
    """Every column of Y against the oracle's FP64 product, relative to
    (|A||X|) column by column (plus |beta Y0| when beta is not zero)."""
    Yref = oracle.spmm(rp, ci, v, X, Y0, alpha=alpha, beta=beta)
    scale = abs(alpha) * oracle.spmm(rp, ci, np.abs(np.asarray(v, np.float64)), np.abs(np.asarray(X, np.float64)))
    if beta != 0:
        scale = scale + abs(beta) * np.abs(np.asarray(Y0, np.float64))
    for c in range(X.shape[1]):
        err = rel_error(Y[:, c], Yref[:, c], scale[:, c])
        assert err <= TOL[dtype], "column %d: relative error %g" % (c, err)


def test_rmat_full():
    """R-MAT scale 22 (67,108,864 nonzeros, FP32) in the encoding and launch
    the benchmark uses: decode bit-exact on the device, every row of y within
    2e-6 of the oracle, then y = -0.5 A x + 2 y."""
    torch = need_gpu()
    progress("generating R-MAT scale 22")
    rp, ci, v = workloads.rmat(22)
    n = 1 << 22
    progress("encode R-MAT (automatic layout)")
    A = P.Matrix.from_csr(rp, ci, v, n)
    info = A.info()
    progress("R-MAT layout %d T %d, %d escaped deltas" % (info["layout"], info["lane_nnz"], info["esc_delta"]))
    assert info["esc_delta"] > 0
    assert decode_equal(torch, A, rp, ci, v)
    x = workloads.vector(n, 3, np.float32)
    xd = torch.from_numpy(x).cuda()
    progress("spmv R-MAT")
    err = check_spmv(A.spmv(xd).cpu().numpy(), rp, ci, v, x, None, 1.0, 0.0, np.float32)
    progress("R-MAT rel error %.3g" % err)
    y0 = workloads.vector(n, 6, np.float32)
    yd = torch.from_numpy(y0.copy()).cuda()
    A.spmv(xd, yd, alpha=-0.5, beta=2.0)
    check_spmv(yd.cpu().numpy(), rp, ci, v, x, y0, -0.5, 2.0, np.float32)


def test_batch_full():
    """The 64 uneven banded FP32 matrices (1k-64k rows) of the batched
    benchmark in one persistent launch: every matrix's y against the oracle,
    for alpha = 1, beta = 0 and for alpha = 0.75, beta = -1.5."""
    torch = need_gpu()
    progress("generating the 64-matrix batch")
    mats = workloads.batch()
    assert len(mats) == 64
    enc = [P.Matrix.from_csr(c[0], c[1], c[2], m, layout="row") for m, c in mats]
    B = P.Batch(enc)
    xs = [workloads.vector(m, 100 + i, np.float32) for i, (m, _) in enumerate(mats)]
    y0 = [workloads.vector(m, 200 + i, np.float32) for i, (m, _) in enumerate(mats)]
    xd = [torch.from_numpy(x).cuda() for x in xs]
    progress("batch spmv, alpha 1 beta 0")
    ys = B.spmv(xd)
    for (m, c), x, y in zip(mats, xs, ys):
        check_spmv(y.cpu().numpy(), c[0], c[1], c[2], x, None, 1.0, 0.0, np.float32)
    progress("batch spmv, alpha 0.75 beta -1.5")
    yd = [torch.from_numpy(y.copy()).cuda() for y in y0]
    B.spmv(xd, yd, alpha=0.75, beta=-1.5)
    for (m, c), x, y, yy in zip(mats, xs, yd, y0):
        check_spmv(y.cpu().numpy(), c[0], c[1], c[2], x, yy, 0.75, -1.5, np.float32)


def test_batch_spmm_full():
    """The 64-matrix batch with k = 8 right-hand sides per matrix: every
    column of every Y_i against the oracle."""
    torch = need_gpu()
    progress("generating the 64-matrix batch (k = 8)")
    mats = workloads.batch()
    enc = [P.Matrix.from_csr(c[0], c[1], c[2], m, layout="row") for m, c in mats]
    B = P.Batch(enc)
    Xs = [workloads.vector(m, 300 + i, np.float32, k=8) for i, (m, _) in enumerate(mats)]
    progress("batch spmm k = 8")
    Ys = B.spmm([torch.from_numpy(X).cuda() for X in Xs])
    for (m, c), X, Y in zip(mats, Xs, Ys):
        Yref = oracle.spmm(c[0], c[1], c[2], X)
        Yn = Y.cpu().numpy()
        for j in range(8):
            assert rel_error(Yn[:, j], Yref[:, j], oracle.absmv(c[0], c[1], c[2], X[:, j])) <= TOL[np.float32]


@pytest.mark.parametrize("layout,sigma", [("row", 0), ("row", 1024), ("nnz", 0)])
def test_skewed_full(layout, sigma):
    """The skewed-rows workload (2^21 rows, heavy-tailed lengths up to 512) in
    the encodings its bench lines time: rows in CSR order, rows sorted within
    windows of 1024, and the nonzero layout."""
    torch = need_gpu()
    progress("skewed rows full size %s sigma=%d" % (layout, sigma))
    rp, ci, v = workloads.skewed_rows()
    n = len(rp) - 1
    A = P.Matrix.from_csr(rp, ci, v, n, layout=layout, sort_window=sigma)
    assert A.info()["sort_window"] == sigma
    assert decode_equal(torch, A, rp, ci, v)
    x = workloads.vector(n, 6)
    check_spmv(A.spmv(torch.from_numpy(x).cuda()).cpu().numpy(), rp, ci, v, x, None, 1, 0, np.float64)
