"""GPU parity of row-sorted (SELL-C-sigma base) containers: every product and
the decode work in the original row order, within the oracle's tolerance
(SpMV, SpMM through both the per-lane and the lane-group sinks, the
transposed product on both of its paths, both stream stages, the
multi-matrix launch), bit-exact for decoding; the symmetric product refuses
such matrices."""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import workloads
from gpu_common import TOL, check_spmv, need_gpu, progress, rel_error

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2603_01915_amd")


def irregular(seed=9, m=3000, n=2500):
    """Row lengths from 0 to a few hundred, shuffled: sorting matters."""
    rng = np.random.default_rng(seed)
    lens = np.minimum(n, (rng.pareto(1.2, size=m) * 3).astype(np.int64))
    rows = [np.sort(rng.choice(n, size=k, replace=False)) for k in lens]
    rp = np.zeros(m + 1, np.int64)
    rp[1:] = np.cumsum(lens)
    ci = np.concatenate(rows).astype(np.int32) if rows else np.zeros(0, np.int32)
    v = rng.choice(rng.standard_normal(500), size=len(ci))
    return rp.astype(np.int32), ci, v, n


def cases():
    rp, ci, v = workloads.rmat(scale=11, edge_factor=16)
    yield "rmat11", rp, ci, v, 2 ** 11
    rp, ci, v, n = irregular()
    yield "irregular", rp, ci, v, n
    rp, ci, v, n = irregular(seed=10, n=50000)  # dX too large for LDS: global atomics
    yield "irregular_wide", rp, ci, v, n


CASES = list(cases())


@pytest.mark.parametrize("case", range(len(CASES)), ids=[c[0] for c in CASES])
@pytest.mark.parametrize("sigma", [64, 512])
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_sorted_products(case, sigma, dtype):
    torch = need_gpu()
    name, rp, ci, v, n = CASES[case]
    v = v.astype(dtype)
    m = len(rp) - 1
    progress("sorted rows %s sigma=%d %s" % (name, sigma, dtype.__name__))
    A = P.Matrix.from_csr(rp, ci, v, n, sort_window=sigma)
    assert A.info()["sort_window"] == sigma
    r2, c2, v2 = A.decode_csr()
    torch.cuda.synchronize()
    assert np.array_equal(r2.cpu().numpy(), rp) and np.array_equal(c2.cpu().numpy(), ci)
    assert np.array_equal(v2.cpu().numpy().view(np.uint8), v.view(np.uint8))
    x = workloads.vector(n, 7, dtype)
    xd = torch.from_numpy(x).cuda()
    check_spmv(A.spmv(xd).cpu().numpy(), rp, ci, v, x, None, 1.0, 0.0, dtype)
    y0 = workloads.vector(m, 8, dtype)
    yd = torch.from_numpy(y0.copy()).cuda()
    A.spmv(xd, yd, alpha=-0.75, beta=1.5)
    check_spmv(yd.cpu().numpy(), rp, ci, v, x, y0, -0.75, 1.5, dtype)
    for k in (3, 8, 32):
        X = workloads.vector(n, 4, dtype, k=k)
        Y = A.spmm(torch.from_numpy(X).cuda()).cpu().numpy()
        Yref = oracle.spmm(rp, ci, v, X)
        for c in range(k):
            assert rel_error(Y[:, c], Yref[:, c], oracle.absmv(rp, ci, v, X[:, c])) <= TOL[dtype], (k, c)
    At = sp.csr_matrix((v.astype(np.float64), ci, rp), shape=(m, n)).T.tocsr()
    At.sort_indices()
    for k in (1, 4):
        dY = workloads.vector(m, 6, dtype, k=k)
        dX = A.spmm_t(torch.from_numpy(dY).cuda()).cpu().numpy()
        for c in range(k):
            ref = oracle.spmtv(rp, ci, v, n, dY[:, c])
            scale = oracle.absmv(At.indptr, At.indices, At.data, dY[:, c])
            assert rel_error(dX[:, c], ref, scale) <= TOL[dtype], (k, c)


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_sorted_ring_stage_and_oracle_container(tmp_path, dtype):
    torch = need_gpu()
    name, rp, ci, v, n = CASES[1]
    v = v.astype(dtype)
    progress("sorted rows ring stage %s" % dtype.__name__)
    A = P.Matrix.from_csr(rp, ci, v, n, sort_window=128, stream_stage=P.STAGE_RING)
    assert A.info()["stream_stage"] == P.STAGE_RING
    x = workloads.vector(n, 7, dtype)
    check_spmv(A.spmv(torch.from_numpy(x).cuda()).cpu().numpy(), rp, ci, v, x, None, 1.0, 0.0, dtype)
    path = str(tmp_path / "o.dtans")
    oracle.encode(path, len(rp) - 1, n, rp, ci, v, seed=3, sigma=256)
    B = P.Matrix.load(path)
    _, c2, v2 = B.decode_csr()
    torch.cuda.synchronize()
    assert np.array_equal(c2.cpu().numpy(), ci)
    assert np.array_equal(v2.cpu().numpy().view(np.uint8), v.view(np.uint8))
    check_spmv(B.spmv(torch.from_numpy(x).cuda()).cpu().numpy(), rp, ci, v, x, None, 1.0, 0.0, dtype)


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_sorted_in_batch(dtype):
    """Row-sorted matrices in the multi-matrix launch (k = 1 and k = 8)."""
    torch = need_gpu()
    mats = workloads.batch(count=10, lo_exp=6, hi_exp=12, half=64)
    progress("sorted rows in a batch %s" % dtype.__name__)
    enc, refs = [], []
    for i, (m, (rp, ci, v)) in enumerate(mats):
        v = v.astype(dtype)
        enc.append(P.Matrix.from_csr(rp, ci, v, m, layout="row", sort_window=64 * (1 + i % 3)))
        refs.append((rp, ci, v))
    b = P.Batch(enc)
    xs = [workloads.vector(m, 100 + i, dtype) for i, (m, _) in enumerate(mats)]
    ys = b.spmv([torch.from_numpy(x).cuda() for x in xs])
    for (rp, ci, v), x, y in zip(refs, xs, ys):
        check_spmv(y.cpu().numpy(), rp, ci, v, x, None, 1.0, 0.0, dtype)
    Xs = [workloads.vector(m, 200 + i, dtype, k=8) for i, (m, _) in enumerate(mats)]
    Ys = b.spmm([torch.from_numpy(X).cuda() for X in Xs])
    for (rp, ci, v), X, Y in zip(refs, Xs, Ys):
        Yref = oracle.spmm(rp, ci, v, X)
        Yn = Y.cpu().numpy()
        for c in range(8):
            assert rel_error(Yn[:, c], Yref[:, c], oracle.absmv(rp, ci, v, X[:, c])) <= TOL[dtype]


def test_sorted_refused_by_symmetric():
    torch = need_gpu()
    rp, ci, v = workloads.stencil27(6)
    progress("sorted rows refused by the symmetric product")
    rpu, ciu, vu, diag = P.symmetric_split(rp, ci, v)
    H = P.Matrix.from_csr(rpu, ciu, vu, 6 ** 3, sort_window=64)
    x = torch.from_numpy(workloads.vector(6 ** 3, 1, np.float64)).cuda()
    with pytest.raises(P.DtansError):
        H.spmv_sym(x, torch.from_numpy(diag).cuda())
    torch.cuda.synchronize()


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_sorted_with_in_stream_escapes_and_edges(dtype):
    """Sorted rows and in-stream escapes together, on a matrix whose row
    count is not a multiple of the window, with empty rows and fewer rows
    than a wave at the end; single products, SpMM and the product for callers
    that cannot allocate."""
    torch = need_gpu()
    rng = np.random.default_rng(12)
    m, n = 64 * 5 + 37, 900
    lens = rng.choice([0, 0, 1, 3, 7, 20, 60], size=m)
    rows = [np.sort(rng.choice(n, size=k, replace=False)) for k in lens]
    rp = np.zeros(m + 1, np.int64)
    rp[1:] = np.cumsum(lens)
    ci = np.concatenate(rows).astype(np.int32)
    v = rng.standard_normal(len(ci)).astype(dtype)  # distinct values: escapes
    rp = rp.astype(np.int32)
    progress("sorted rows + in-stream escapes %s" % dtype.__name__)
    A = P.Matrix.from_csr(rp, ci, v, n, sort_window=128, escape_in_stream=True)
    inf = A.info()
    assert inf["sort_window"] == 128 and inf["escape_in_stream"] == 1
    _, c2, v2 = A.decode_csr()
    torch.cuda.synchronize()
    assert np.array_equal(c2.cpu().numpy(), ci)
    assert np.array_equal(v2.cpu().numpy().view(np.uint8), v.view(np.uint8))
    x = workloads.vector(n, 3, dtype)
    check_spmv(A.spmv(torch.from_numpy(x).cuda()).cpu().numpy(), rp, ci, v, x, None, 1.0, 0.0, dtype)
    X = workloads.vector(n, 4, dtype, k=16)
    Xd = torch.from_numpy(X).cuda()
    Y = A.spmm(Xd)
    Yref = oracle.spmm(rp, ci, v, X)
    Yn = Y.cpu().numpy()
    for c in range(16):
        assert rel_error(Yn[:, c], Yref[:, c], oracle.absmv(rp, ci, v, X[:, c])) <= TOL[dtype]
    Y2 = torch.empty_like(Y)
    A.spmm_noalloc(Xd, Y2)
    torch.cuda.synchronize()
    assert torch.equal(Y, Y2)


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_sorted_gpu_encoder_same_container(tmp_path, dtype):
    """The GPU encoder (host arrays in) writes the same sorted-row container,
    byte for byte, as the host encoder; device-resident arrays are refused."""
    torch = need_gpu()
    name, rp, ci, v, n = CASES[1]
    v = v.astype(dtype)
    progress("sorted rows, GPU encoder %s" % dtype.__name__)
    A = P.Matrix.from_csr(rp, ci, v, n, sort_window=256)
    B = P.Matrix.from_csr(rp, ci, v, n, sort_window=256, gpu_encode=True)
    pa, pb = str(tmp_path / "a.dtans"), str(tmp_path / "b.dtans")
    A.save(pa)
    B.save(pb)
    assert open(pa, "rb").read() == open(pb, "rb").read()
    d = [torch.from_numpy(t).cuda() for t in (rp, ci, v)]
    with pytest.raises(P.DtansError):
        P.Matrix.from_csr_device(d[0], d[1], d[2], n, sort_window=256)
    torch.cuda.synchronize()
