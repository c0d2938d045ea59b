"""GPU parity: the HIP kernels against the oracle, through the C ABI.

* decoding is bit-exact against the original CSR, for containers written by
  the library and by the oracle's independent encoder;
* y = alpha*A*x + beta*y is within 1e-12 (FP64) / 2e-6 (FP32) of the oracle's
  FP64 product, relative to (|A||x|)_i;
* SpMM, the transposed product, the multi-matrix launch and the plain-CSR
  baseline are checked the same way.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import workloads
from gpu_common import TOL, check_spmv, need_gpu, progress, rel_error

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2603_01915_amd")

LAYOUTS = [("row", 0), ("nnz", 32), ("nnz", 128)]


def adversarial(seed=3, n=5000):
    rng = np.random.default_rng(seed)
    rows = [[], [7], [1, 2], [0, 0, 3], [], list(range(0, n, 2)), [n - 1], [], [5, 5, 5, 5, 5],
            list(range(100, 113))]
    rows += [sorted(rng.choice(n, size=rng.integers(0, 12), replace=False)) for _ in range(700)]
    rows += [[]] * 70  # a run of empty rows longer than a wave
    rows += [sorted(rng.choice(n, size=rng.integers(1, 4), replace=False)) for _ in range(200)]
    rp = np.zeros(len(rows) + 1, np.int64)
    rp[1:] = np.cumsum([len(r) for r in rows])
    ci = np.array([c for r in rows for c in r], np.int64).astype(np.int32)
    v = rng.standard_normal(len(ci))  # mostly distinct values: value escapes
    v[::5] = 0.5
    return rp.astype(np.int32), ci, v, n


def small_cases():
    rp, ci, v = workloads.band(m=1000, per_row=16, half=256)
    yield "band1000", rp, ci, v, 1000
    rp, ci, v = workloads.stencil27(12)
    yield "stencil12", rp, ci, v, 12 ** 3
    rp, ci, v = workloads.rmat(scale=11, edge_factor=16)
    yield "rmat11", rp, ci, v, 2 ** 11
    rp, ci, v = workloads.pruned_weight(rows=300, cols=256)
    yield "pruned300", rp, ci, v, 256
    rp, ci, v, n = adversarial()
    yield "adversarial", rp, ci, v, n


CASES = list(small_cases())


@pytest.mark.parametrize("case", range(len(CASES)), ids=[c[0] for c in CASES])
@pytest.mark.parametrize("layout,T", LAYOUTS)
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_decode_bit_exact(case, layout, T, dtype):
    torch = need_gpu()
    name, rp, ci, v, n = CASES[case]
    v = v.astype(dtype)
    progress("decode %s %s T=%d %s" % (name, layout, T, dtype.__name__))
    A = P.Matrix.from_csr(rp, ci, v, n, layout=layout, lane_nnz=T)
    r2, c2, v2 = A.decode_csr()
    torch.cuda.synchronize()
    assert np.array_equal(r2.cpu().numpy(), rp)
    assert np.array_equal(c2.cpu().numpy(), ci)
    assert np.array_equal(v2.cpu().numpy().view(np.uint8), v.view(np.uint8))


@pytest.mark.parametrize("layout,T", [(1, 0), (2, 32), (2, 12)])
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_decode_oracle_containers(tmp_path, layout, T, dtype):
    """The GPU decodes containers written by the oracle's own encoder."""
    torch = need_gpu()
    for name, rp, ci, v, n in CASES:
        v = v.astype(dtype)
        progress("oracle container %s layout=%d T=%d %s" % (name, layout, T, dtype.__name__))
        path = str(tmp_path / (name + ".dtans"))
        oracle.encode(path, len(rp) - 1, n, rp, ci, v, layout=layout, lane_nnz=T, seed=11)
        A = P.Matrix.load(path)
        r2, c2, v2 = A.decode_csr()
        torch.cuda.synchronize()
        assert np.array_equal(c2.cpu().numpy(), ci)
        assert np.array_equal(v2.cpu().numpy().view(np.uint8), v.view(np.uint8))
        x = workloads.vector(n, 9, dtype)
        y = A.spmv(torch.from_numpy(x).cuda())
        check_spmv(y.cpu().numpy(), rp, ci, v, x, None, 1.0, 0.0, dtype)


@pytest.mark.parametrize("case", range(len(CASES)), ids=[c[0] for c in CASES])
@pytest.mark.parametrize("layout,T", LAYOUTS)
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_spmv_parity(case, layout, T, dtype):
    torch = need_gpu()
    name, rp, ci, v, n = CASES[case]
    v = v.astype(dtype)
    m = len(rp) - 1
    progress("spmv %s %s T=%d %s" % (name, layout, T, dtype.__name__))
    A = P.Matrix.from_csr(rp, ci, v, n, layout=layout, lane_nnz=T)
    x = workloads.vector(n, 7, dtype)
    xd = torch.from_numpy(x).cuda()
    y = A.spmv(xd)
    check_spmv(y.cpu().numpy(), rp, ci, v, x, None, 1.0, 0.0, dtype)
    # alpha, beta with an existing y; and beta = 0 over a NaN-filled y
    y0 = workloads.vector(m, 8, dtype)
    yd = torch.from_numpy(y0.copy()).cuda()
    A.spmv(xd, yd, alpha=-0.75, beta=1.5)
    check_spmv(yd.cpu().numpy(), rp, ci, v, x, y0, -0.75, 1.5, dtype)
    yn = torch.full((m,), float("nan"), dtype=yd.dtype, device="cuda")
    A.spmv(xd, yn, alpha=2.0, beta=0.0)
    check_spmv(yn.cpu().numpy(), rp, ci, v, x, None, 2.0, 0.0, dtype)
    # repeated calls give the same result bit for bit (no atomics in SpMV)
    y2 = A.spmv(xd)
    assert torch.equal(y, y2)


@pytest.mark.parametrize("case", range(len(CASES)), ids=[c[0] for c in CASES])
@pytest.mark.parametrize("layout,T", LAYOUTS)
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_spmv_stream_stages_agree(case, layout, T, dtype):
    """The SpMV that stages its streams through an LDS ring and the one that
    reads them directly give the same y bit for bit (same products in the
    same order), and both match the oracle."""
    torch = need_gpu()
    name, rp, ci, v, n = CASES[case]
    v = v.astype(dtype)
    m = len(rp) - 1
    x = torch.from_numpy(workloads.vector(n, 7, dtype)).cuda()
    ys = []
    for stage in (P.STAGE_DIRECT, P.STAGE_RING):
        progress("spmv stages %s %s T=%d %s stage=%d" % (name, layout, T, dtype.__name__, stage))
        A = P.Matrix.from_csr(rp, ci, v, n, layout=layout, lane_nnz=T, stream_stage=stage)
        assert A.info()["stream_stage"] == stage
        ys.append(A.spmv(x))
        yn = torch.full((m,), float("nan"), dtype=x.dtype, device="cuda")
        A.spmv(x, yn, alpha=2.0, beta=0.0)
        check_spmv(yn.cpu().numpy(), rp, ci, v, x.cpu().numpy(), None, 2.0, 0.0, dtype)
    assert torch.equal(ys[0], ys[1])
    check_spmv(ys[1].cpu().numpy(), rp, ci, v, x.cpu().numpy(), None, 1.0, 0.0, dtype)
    # SpMM: the ring kernels take fewer columns per pass; a row's nonzeros
    # are summed in the same order by both, so the results agree bit for bit
    # where no row is split over lanes in another way: the row layout, and
    # fewer columns than the direct kernel hands to lane groups (4 FP64 / 8
    # FP32), whose wavefront sums of split rows run in another order
    for k in (3, 8, 37):
        X = torch.from_numpy(workloads.vector(n, 11, dtype, k=k)).cuda()
        Ys = []
        for stage in (P.STAGE_DIRECT, P.STAGE_RING):
            A = P.Matrix.from_csr(rp, ci, v, n, layout=layout, lane_nnz=T, stream_stage=stage)
            Ys.append(A.spmm(X))
        if layout == "row" or k < (4 if dtype == np.float64 else 8):
            assert torch.equal(Ys[0], Ys[1]), (k, float((Ys[0] - Ys[1]).abs().max()))
        Xh = X.cpu().numpy()
        for Y in Ys:
            for c in (0, k - 1):
                check_spmv(Y.cpu().numpy()[:, c], rp, ci, v, np.ascontiguousarray(Xh[:, c]), None,
                           1.0, 0.0, dtype)


@pytest.mark.parametrize("case", range(len(CASES)), ids=[c[0] for c in CASES])
@pytest.mark.parametrize("layout,T", [("row", 0), ("nnz", 32)])
def test_table_formats_agree(case, layout, T):
    """Tables capped at 255 slots per symbol (bases used as stored) and at the
    paper's 256 (bases stored minus one) decode to the same CSR and give the
    same products bit for bit through SpMV and SpMM; the transpose (atomic
    adds, order not fixed) agrees within the tolerance."""
    torch = need_gpu()
    name, rp, ci, v, n = CASES[case]
    m = len(rp) - 1
    dt = v.dtype
    x = torch.from_numpy(workloads.vector(n, 7, dt)).cuda()
    X = torch.from_numpy(workloads.vector(n, 9, dt, k=3)).cuda()
    dY = torch.from_numpy(workloads.vector(m, 10, dt, k=2)).cuda()
    out = []
    for cap in (0, 256):
        progress("table format %s %s T=%d cap=%d" % (name, layout, T, cap))
        A = P.Matrix.from_csr(rp, ci, v, n, layout=layout, lane_nnz=T, max_mult=cap)
        if cap == 0:
            assert A.info()["direct_table"] == 1
        r2, c2, v2 = A.decode_csr()
        assert np.array_equal(c2.cpu().numpy(), ci)
        assert np.array_equal(v2.cpu().numpy(), v)
        out.append((A.spmv(x), A.spmm(X), A.spmm_t(dY)))
    for a, b in zip(out[0][:2], out[1][:2]):
        assert torch.equal(a, b)
    check_spmv(out[0][0].cpu().numpy(), rp, ci, v, x.cpu().numpy(), None, 1.0, 0.0, dt.type)
    At = sp.csr_matrix((v.astype(np.float64), ci, rp), shape=(m, n)).T.tocsr()
    At.sort_indices()
    dYh = dY.cpu().numpy()
    for c in range(2):
        ref = oracle.spmtv(rp, ci, v, n, dYh[:, c])
        scale = oracle.absmv(At.indptr, At.indices, At.data, dYh[:, c])
        for o in out:
            assert rel_error(o[2].cpu().numpy()[:, c], ref, scale) <= TOL[dt.type]


@pytest.mark.parametrize("layout,T", LAYOUTS)
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("k", [1, 3, 8, 32, 37])
def test_spmm_parity(layout, T, dtype, k):
    torch = need_gpu()
    rp, ci, v = workloads.pruned_weight(rows=400, cols=300)
    v = v.astype(dtype)
    m, n = 400, 300
    progress("spmm %s T=%d %s k=%d" % (layout, T, dtype.__name__, k))
    A = P.Matrix.from_csr(rp, ci, v, n, layout=layout, lane_nnz=T)
    X = workloads.vector(n, 4, dtype, k=k)
    Y = A.spmm(torch.from_numpy(X).cuda()).cpu().numpy()
    Yref = oracle.spmm(rp, ci, v, X)
    for c in range(k):
        scale = oracle.absmv(rp, ci, v, X[:, c])
        assert rel_error(Y[:, c], Yref[:, c], scale) <= TOL[dtype]
    # strided X / Y (leading dimension > k) and beta
    Xs = torch.zeros((n, k + 5), dtype=A.torch_dtype, device="cuda")
    Xs[:, :k] = torch.from_numpy(X).cuda()
    Y0 = workloads.vector(m, 5, dtype, k=k)
    Ys = torch.zeros((m, k + 3), dtype=A.torch_dtype, device="cuda")
    Ys[:, :k] = torch.from_numpy(Y0).cuda()
    A.spmm(Xs[:, :k], Ys[:, :k], alpha=0.5, beta=-1.0)
    Yb = Ys[:, :k].cpu().numpy()
    Yref = oracle.spmm(rp, ci, v, X, Y0, alpha=0.5, beta=-1.0)
    for c in range(k):
        scale = 0.5 * oracle.absmv(rp, ci, v, X[:, c]) + np.abs(Y0[:, c].astype(np.float64))
        assert rel_error(Yb[:, c], Yref[:, c], scale) <= TOL[dtype]
    assert torch.count_nonzero(Ys[:, k:]) == 0


@pytest.mark.parametrize("layout,T", LAYOUTS)
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("k", [1, 16])
def test_spmm_t_parity(layout, T, dtype, k):
    torch = need_gpu()
    for name, rp, ci, v, n in CASES:
        v = v.astype(dtype)
        m = len(rp) - 1
        progress("spmm_t %s %s T=%d %s k=%d" % (name, layout, T, dtype.__name__, k))
        A = P.Matrix.from_csr(rp, ci, v, n, layout=layout, lane_nnz=T)
        dY = workloads.vector(m, 6, dtype, k=k)
        dX0 = workloads.vector(n, 3, dtype, k=k)
        dX = torch.from_numpy(dX0.copy()).cuda()
        A.spmm_t(torch.from_numpy(dY).cuda(), dX, alpha=1.25, beta=0.5)
        out = dX.cpu().numpy()
        At = sp.csr_matrix((v.astype(np.float64), ci, rp), shape=(m, n)).T.tocsr()
        At.sort_indices()
        for c in range(k):
            ref = oracle.spmtv(rp, ci, v, n, dY[:, c], dX0[:, c], alpha=1.25, beta=0.5)
            scale = 1.25 * oracle.absmv(At.indptr, At.indices, At.data, dY[:, c]) + \
                0.5 * np.abs(dX0[:, c].astype(np.float64))
            assert rel_error(out[:, c], ref, scale) <= TOL[dtype], (name, c)


@pytest.mark.parametrize("variant", [1, 2, 3])
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_csr_baseline_parity(variant, dtype):
    torch = need_gpu()
    for name, rp, ci, v, n in CASES:
        v = v.astype(dtype)
        progress("csr baseline v%d %s %s" % (variant, name, dtype.__name__))
        B = P.CsrBaseline(rp, ci, v, n, variant=variant)
        x = workloads.vector(n, 7, dtype)
        y = B.spmv(torch.from_numpy(x).cuda())
        check_spmv(y.cpu().numpy(), rp, ci, v, x, None, 1.0, 0.0, dtype)
        X = workloads.vector(n, 4, dtype, k=8)
        Y = B.spmm(torch.from_numpy(X).cuda()).cpu().numpy()
        for c in range(8):
            check_spmv(Y[:, c], rp, ci, v, X[:, c], None, 1.0, 0.0, dtype)


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_rocsparse_baseline_parity(dtype):
    """The rocSPARSE context baseline computes the same products (SpMV and
    SpMM with beta != 0); its tolerance is the same as ours, since the
    library accumulates in the value type (FP32 sums are checked with the
    FP32 bound only up to the row lengths of these cases)."""
    torch = need_gpu()
    for name, rp, ci, v, n in CASES:
        v = v.astype(dtype)
        m = len(rp) - 1
        progress("rocsparse baseline %s %s" % (name, dtype.__name__))
        R = P.RocsparseBaseline(rp, ci, v, n)
        x = workloads.vector(n, 7, dtype)
        y0 = workloads.vector(m, 8, dtype)
        y = torch.from_numpy(y0.copy()).cuda()
        R.spmv(torch.from_numpy(x).cuda(), y, alpha=0.5, beta=2.0)
        y_ref = oracle.spmv(rp, ci, v, x, y0, alpha=0.5, beta=2.0)
        scale = 0.5 * oracle.absmv(rp, ci, v, x) + 2.0 * np.abs(y0.astype(np.float64))
        tol = 1e-12 if dtype == np.float64 else 2e-6 * max(1, int(np.diff(rp).max()) // 16)
        assert rel_error(y.cpu().numpy(), y_ref, scale) <= tol
        X = workloads.vector(n, 4, dtype, k=8)
        Y = R.spmm(torch.from_numpy(X).cuda()).cpu().numpy()
        Yref = oracle.spmm(rp, ci, v, X)
        for c in range(8):
            assert rel_error(Y[:, c], Yref[:, c], oracle.absmv(rp, ci, v, X[:, c])) <= tol
        R.close()


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_batch_matches_single(dtype):
    torch = need_gpu()
    mats = workloads.batch(count=12, lo_exp=6, hi_exp=12, half=64)
    progress("batch of %d %s" % (len(mats), dtype.__name__))
    enc, xs, refs = [], [], []
    for i, (m, (rp, ci, v)) in enumerate(mats):
        v = v.astype(dtype)
        enc.append(P.Matrix.from_csr(rp, ci, v, m, layout="row"))
        x = workloads.vector(m, 100 + i, dtype)
        xs.append(torch.from_numpy(x).cuda())
        refs.append((rp, ci, v, x))
    b = P.Batch(enc)
    ys = b.spmv(xs)
    for (rp, ci, v, x), y, A, xd in zip(refs, ys, enc, xs):
        check_spmv(y.cpu().numpy(), rp, ci, v, x, None, 1.0, 0.0, dtype)
        assert torch.equal(y, A.spmv(xd))  # same kernel body, same order
    ys2 = [torch.ones_like(y) for y in ys]
    b.spmv(xs, ys2, alpha=2.0, beta=-1.0)
    for (rp, ci, v, x), y in zip(refs, ys2):
        check_spmv(y.cpu().numpy(), rp, ci, v, x, np.ones(len(rp) - 1, dtype), 2.0, -1.0, dtype)


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("k", [1, 3, 8, 13, 32])
def test_batch_spmm(dtype, k):
    """Several right-hand sides per matrix in one batched launch per column
    chunk: every column of every Y_i against the oracle, on 16-byte aligned
    X_i / Y_i (lane-group chunks) and on views one element off (single
    columns), with alpha and beta."""
    torch = need_gpu()
    mats = workloads.batch(count=12, lo_exp=6, hi_exp=12, half=64)
    progress("batch spmm of %d %s k=%d" % (len(mats), dtype.__name__, k))
    enc, Xs, refs = [], [], []
    for i, (m, (rp, ci, v)) in enumerate(mats):
        v = v.astype(dtype)
        enc.append(P.Matrix.from_csr(rp, ci, v, m, layout="row"))
        X = workloads.vector(m, 100 + i, dtype, k=k)
        Xs.append(X)
        refs.append((rp, ci, v))
    b = P.Batch(enc)
    Ys = b.spmm([torch.from_numpy(X).cuda() for X in Xs])
    for (rp, ci, v), X, Y in zip(refs, Xs, Ys):
        Yref = oracle.spmm(rp, ci, v, X)
        Yn = Y.cpu().numpy()
        for c in range(k):
            assert rel_error(Yn[:, c], Yref[:, c], oracle.absmv(rp, ci, v, X[:, c])) <= TOL[dtype], c
    # unaligned storage (one element into a buffer), alpha and beta
    Xo, Yo, Y0 = [], [], []
    for (m, _), X in zip(mats, Xs):
        bx = torch.zeros(m * k + 1, dtype=enc[0].torch_dtype, device="cuda")
        bx[1:] = torch.from_numpy(X).cuda().reshape(-1)
        Xo.append(bx[1:].view(m, k))
        y0 = workloads.vector(m, 7, dtype, k=k)
        by = torch.zeros(m * k + 1, dtype=enc[0].torch_dtype, device="cuda")
        by[1:] = torch.from_numpy(y0).cuda().reshape(-1)
        Yo.append(by[1:].view(m, k))
        Y0.append(y0)
    b.spmm(Xo, Yo, alpha=0.5, beta=-1.0)
    for (rp, ci, v), X, Y, y0 in zip(refs, Xs, Yo, Y0):
        Yref = oracle.spmm(rp, ci, v, X, y0, alpha=0.5, beta=-1.0)
        Yn = Y.cpu().numpy()
        for c in range(k):
            scale = 0.5 * oracle.absmv(rp, ci, v, X[:, c]) + np.abs(y0[:, c].astype(np.float64))
            assert rel_error(Yn[:, c], Yref[:, c], scale) <= TOL[dtype], c


def test_empty_and_degenerate():
    torch = need_gpu()
    for layout, T in LAYOUTS:
        progress("degenerate %s %d" % (layout, T))
        # all rows empty
        A = P.Matrix.from_csr(np.zeros(65, np.int32), np.zeros(0, np.int32), np.zeros(0), 10,
                              layout=layout, lane_nnz=T)
        y = torch.full((64,), 3.0, dtype=torch.float64, device="cuda")
        A.spmv(torch.ones(10, dtype=torch.float64, device="cuda"), y, beta=0.5)
        assert torch.all(y == 1.5)
        # a single nonzero
        A = P.Matrix.from_csr(np.array([0, 0, 1, 1], np.int32), np.array([4], np.int32),
                              np.array([2.5]), 6, layout=layout, lane_nnz=T)
        y = A.spmv(torch.arange(6, dtype=torch.float64, device="cuda"))
        assert y.tolist() == [0.0, 10.0, 0.0]
        # one long row among empty rows
        rp = np.array([0, 0, 5000, 5000, 5000], np.int32)
        ci = np.arange(5000, dtype=np.int32)
        v = np.full(5000, 0.25)
        A = P.Matrix.from_csr(rp, ci, v, 5000, layout=layout, lane_nnz=T)
        y = A.spmv(torch.ones(5000, dtype=torch.float64, device="cuda"))
        assert y.tolist() == [0.0, 1250.0, 0.0, 0.0]


def test_launch_shapes_agree():
    """Every launch shape gives the bit-identical y (the lane work and the
    summation order do not depend on the grid)."""
    torch = need_gpu()
    rp, ci, v = workloads.stencil27(20)
    n = 20 ** 3
    x = torch.from_numpy(workloads.vector(n, 2)).cuda()
    ref = None
    shapes = [(wpw, wgcu, P.STAGE_DIRECT) for wpw, wgcu in ((1, 1), (4, 2), (14, 2), (16, 1), (7, 3))]
    shapes += [(16, 0, P.STAGE_RING), (8, 0, P.STAGE_RING), (4, 1, P.STAGE_RING), (1, 2, P.STAGE_RING),
               (16, 1, P.STAGE_RING)]
    for wpw, wgcu, stage in shapes:
        progress("launch shape %d x %d stage %d" % (wpw, wgcu, stage))
        A = P.Matrix.from_csr(rp, ci, v, n, layout="row", waves_per_wg=wpw, wg_per_cu=wgcu,
                              stream_stage=stage)
        y = A.spmv(x)
        if ref is None:
            ref = y
            check_spmv(y.cpu().numpy(), rp, ci, v, x.cpu().numpy(), None, 1.0, 0.0, np.float64)
        assert torch.equal(y, ref)


def long_rows(T, seed=11):
    """Rows spanning many lanes of T nonzeros: ends exactly at lane ends, one
    lane past a wavefront boundary, several wavefronts, and more than 256
    lanes (the wavefront-per-row fix-up), between short and empty rows."""
    rng = np.random.default_rng(seed)
    lens = [3, 64 * T - 3, T, 0, 2 * T, 65 * T + 1, 5, 300 * T + 7, 0, 0, 130 * T, 1, 64 * T, 17]
    n = 20000
    rows = [np.sort(rng.choice(n, size=min(L, n), replace=False)) if L <= n else
            np.sort(rng.integers(0, n, size=L)) for L in lens]
    rp = np.zeros(len(rows) + 1, np.int64)
    rp[1:] = np.cumsum([len(r) for r in rows])
    ci = np.concatenate(rows).astype(np.int32)
    v = rng.choice([0.5, -1.25, 2.0, 3.0], size=len(ci))
    return rp.astype(np.int32), ci, v, n


@pytest.mark.parametrize("T", [32, 44, 128])
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_long_split_rows(T, dtype):
    """Rows split over many lanes: the middle lanes' pieces are summed per
    wavefront before the fix-up; SpMV, SpMM and beta != 0 against the oracle."""
    torch = need_gpu()
    rp, ci, v, n = long_rows(T)
    v = v.astype(dtype)
    progress("long split rows T=%d %s" % (T, dtype.__name__))
    A = P.Matrix.from_csr(rp, ci, v, n, layout="nnz", lane_nnz=T)
    m = len(rp) - 1
    x = workloads.vector(n, 7, dtype)
    y0 = workloads.vector(m, 8, dtype)
    y = torch.from_numpy(y0.copy()).cuda()
    A.spmv(torch.from_numpy(x).cuda(), y, alpha=1.5, beta=-0.5)
    check_spmv(y.cpu().numpy(), rp, ci, v, x, y0, 1.5, -0.5, dtype)
    for k in (3, 8):
        X = workloads.vector(n, 9, dtype, k=k)
        Y = A.spmm(torch.from_numpy(X).cuda()).cpu().numpy()
        Yref = oracle.spmm(rp, ci, v, X)
        for c in range(k):
            scale = oracle.absmv(rp, ci, v, X[:, c])
            assert rel_error(Y[:, c], Yref[:, c], scale) <= TOL[dtype]


@pytest.mark.parametrize("layout,T", [("row", 0), ("nnz", 32)])
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_spmm_t_both_paths(layout, T, dtype):
    """The transposed product with dX privatised in LDS (n small enough for one
    column of dX beside the tables) and with global atomics (n just too large)
    agree with the oracle; k = 5 spans several LDS passes."""
    torch = need_gpu()
    vb = np.dtype(dtype).itemsize
    room = 160 * 1024 - 1024 - 4096 * (8 + vb)
    n_fit = (room // vb - 1) * 32 // 33  # largest n whose one-column block fits
    for n in (n_fit, n_fit + 64):
        rng = np.random.default_rng(n)
        m = 1500
        lens = rng.integers(0, 40, size=m)
        rp = np.zeros(m + 1, np.int64)
        rp[1:] = np.cumsum(lens)
        ci = np.concatenate([np.sort(rng.choice(n, size=L, replace=False)) for L in lens]).astype(np.int32)
        v = rng.choice([0.5, -1.5, 2.0, 0.25], size=len(ci)).astype(dtype)
        rp = rp.astype(np.int32)
        progress("spmm_t paths n=%d %s %s" % (n, layout, dtype.__name__))
        A = P.Matrix.from_csr(rp, ci, v, n, layout=layout, lane_nnz=T)
        k = 5
        dY = workloads.vector(m, 6, dtype, k=k)
        dX0 = workloads.vector(n, 3, dtype, k=k)
        dX = torch.from_numpy(dX0.copy()).cuda()
        A.spmm_t(torch.from_numpy(dY).cuda(), dX, alpha=-0.75, beta=0.5)
        out = dX.cpu().numpy()
        At = sp.csr_matrix((v.astype(np.float64), ci, rp), shape=(m, n)).T.tocsr()
        At.sort_indices()
        for c in range(k):
            ref = oracle.spmtv(rp, ci, v, n, dY[:, c], dX0[:, c], alpha=-0.75, beta=0.5)
            scale = 0.75 * oracle.absmv(At.indptr, At.indices, At.data, dY[:, c]) + \
                0.5 * np.abs(dX0[:, c].astype(np.float64))
            assert rel_error(out[:, c], ref, scale) <= TOL[dtype], (n, c)


@pytest.mark.parametrize("layout,T", [("row", 0), ("nnz", 16)])
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_symmetric_half_storage(layout, T, dtype):
    """y = alpha (S + S^T + diag(d)) x + beta y from the strict upper triangle
    S only, against the oracle's product with the whole symmetric matrix;
    also without a diagonal.  Sizes span several waves with a ragged tail and
    rows of S without entries; the 27-point stencil (symmetrised) covers a
    regular case."""
    torch = need_gpu()
    rng = np.random.default_rng(77)
    cases = []
    n = 3000
    B = sp.random(n, n, density=0.003, format="csr", random_state=rng)
    A = (B + B.T + sp.diags(rng.standard_normal(n))).tocsr()
    A.eliminate_zeros()
    A.sort_indices()
    cases.append(("random", A))
    rp, ci, v = workloads.stencil27(20)
    S0 = sp.csr_matrix((v, ci, rp), shape=(20 ** 3, 20 ** 3))
    A2 = ((S0 + S0.T) * 0.5).tocsr()
    A2.sort_indices()
    cases.append(("stencil20", A2))
    for name, A in cases:
        rpa, cia, va = A.indptr.astype(np.int32), A.indices.astype(np.int32), A.data.astype(dtype)
        rpu, ciu, vu, d = P.symmetric_split(rpa, cia, va)
        progress("symmetric %s %s %s" % (name, layout, dtype.__name__))
        M = P.Matrix.from_csr(rpu, ciu, vu, A.shape[0], layout=layout, lane_nnz=T)
        x = workloads.vector(A.shape[0], 3, dtype)
        y0 = workloads.vector(A.shape[0], 4, dtype)
        xt, dt = torch.from_numpy(x).cuda(), torch.from_numpy(d).cuda()
        for alpha, beta in ((1.0, 0.0), (-0.5, 0.75)):
            yt = torch.from_numpy(y0.copy()).cuda()
            M.spmv_sym(xt, dt, yt, alpha=alpha, beta=beta)
            check_spmv(yt.cpu().numpy(), rpa, cia, va, x, y0, alpha, beta, dtype)
        # without the diagonal
        yt = M.spmv_sym(xt)
        Aod = sp.csr_matrix((vu, ciu, rpu), shape=A.shape)
        Aod = (Aod + Aod.T).tocsr()
        Aod.sort_indices()
        check_spmv(yt.cpu().numpy(), Aod.indptr, Aod.indices, Aod.data, x, np.zeros_like(x), 1.0, 0.0, dtype)
