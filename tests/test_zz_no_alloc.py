"""dtans_spmm_noalloc (the product for callers that cannot allocate device
memory, its partial sums in the library's per-device scratch array) against
dtans_spmm on the same kernels and against the oracle, through the C ABI.

Two calls in a row, the second on a smaller matrix with fewer columns, so
that a stale partial sum left in the shared array by the first call would
show; both layouts; and the size check that rejects a product needing more
scratch than the array holds, before any launch."""
import numpy as np
import pytest

import oracle
import workloads
from gpu_common import TOL, need_gpu, progress, rel_error

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2603_01915_amd")


def _long_rows(seed, m, n, lo, hi):
    """rows of lo..hi nonzeros (uniform), columns spread over [0, n)"""
    rng = np.random.default_rng(seed)
    lens = rng.integers(lo, hi + 1, size=m)
    rows = [np.sort(rng.choice(n, size=int(L), replace=False)) for L in lens]
    rp = np.zeros(m + 1, np.int64)
    rp[1:] = np.cumsum(lens)
    ci = np.concatenate(rows).astype(np.int32)
    v = rng.choice([0.5, -1.25, 2.0, 3.0, -0.75], size=len(ci))
    return rp.astype(np.int32), ci, v


def _check(torch, A, rp, ci, v, n, k, dtype, seed, alpha, beta):
    m = len(rp) - 1
    X = workloads.vector(n, seed, dtype, k=k)
    Y0 = workloads.vector(m, seed + 1, dtype, k=k)
    Xd = torch.from_numpy(X).cuda()
    Ya = torch.from_numpy(Y0.copy()).cuda()
    Yb = torch.from_numpy(Y0.copy()).cuda()
    A.spmm_noalloc(Xd, Ya, alpha=alpha, beta=beta)
    A.spmm(Xd, Yb, alpha=alpha, beta=beta)
    torch.cuda.synchronize()
    ya, yb = Ya.cpu().numpy(), Yb.cpu().numpy()
    # same kernels, same summation order: the two entry points agree bit for bit
    assert np.array_equal(ya.view(np.uint8), yb.view(np.uint8))
    Yref = oracle.spmm(rp, ci, v, X, Y0, alpha=alpha, beta=beta)
    for c in range(k):
        scale = abs(alpha) * oracle.absmv(rp, ci, v, X[:, c]) + abs(beta) * np.abs(Y0[:, c].astype(np.float64))
        assert rel_error(ya[:, c], Yref[:, c], scale) <= TOL[dtype]


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_noalloc_matches_spmm(dtype):
    torch = need_gpu()
    # first call: long rows split over many lanes (nonzero layout), k = 8
    rp1, ci1, v1 = _long_rows(11, 700, 3000, 40, 700)
    v1 = v1.astype(dtype)
    A1 = P.Matrix.from_csr(rp1, ci1, v1, 3000, layout="nnz", lane_nnz=32).to_device()
    progress("noalloc first call: %d rows, %d nonzeros, k=8 %s" % (700, len(ci1), dtype.__name__))
    _check(torch, A1, rp1, ci1, v1, 3000, 8, dtype, 21, 1.0, 0.0)
    # second call, smaller: fewer lanes and columns, beta != 0
    rp2, ci2, v2 = _long_rows(12, 90, 500, 20, 200)
    v2 = v2.astype(dtype)
    A2 = P.Matrix.from_csr(rp2, ci2, v2, 500, layout="nnz", lane_nnz=16).to_device()
    progress("noalloc second call: %d rows, %d nonzeros, k=3 %s" % (90, len(ci2), dtype.__name__))
    _check(torch, A2, rp2, ci2, v2, 500, 3, dtype, 31, -0.5, 2.0)
    # the row layout (no scratch used) and a single vector
    rp3, ci3, v3 = workloads.band(m=600, per_row=16, half=64)
    v3 = v3.astype(dtype)
    A3 = P.Matrix.from_csr(rp3, ci3, v3, 600, layout="row").to_device()
    progress("noalloc row layout k=1 %s" % dtype.__name__)
    _check(torch, A3, rp3, ci3, v3, 600, 1, dtype, 41, 1.0, 0.0)


def test_noalloc_rejects_oversized_product():
    torch = need_gpu()
    # 600,000 nonzeros in lanes of 4: 150,000 lanes x 2 x 32 doubles = 76.8 MB
    # of partial sums for k = 32, above the 64 MiB array
    m, n, per = 15000, 4000, 40
    rng = np.random.default_rng(5)
    ci = np.concatenate([np.sort(rng.choice(n, size=per, replace=False)) for _ in range(m)]).astype(np.int32)
    rp = (np.arange(m + 1) * per).astype(np.int32)
    v = np.ones(len(ci))
    A = P.Matrix.from_csr(rp, ci, v, n, layout="nnz", lane_nnz=4).to_device()
    X = torch.zeros((n, 32), dtype=torch.float64, device="cuda")
    Y = torch.full((m, 32), 7.0, dtype=torch.float64, device="cuda")
    with pytest.raises(P.DtansError) as ei:
        A.spmm_noalloc(X, Y)
    assert ei.value.status == 3  # DTANS_ERANGE
    assert "scratch" in str(ei.value)
    torch.cuda.synchronize()
    assert bool((Y == 7.0).all())  # nothing was launched
    # the same product fits with 8 columns (19.2 MB) and is exact here
    A.spmm_noalloc(X[:, :8].contiguous(), Y[:, :8].contiguous())
