"""GPU parity of containers whose escaped symbols sit in the word stream
(Sec. IV-F): decoding bit-exact against the CSR arrays (library- and
oracle-written containers), SpMV / SpMM / the transposed product within the
oracle's tolerance and bit-identical to the same matrix with escapes in
separate regions (the same products in the same order), and the LDS-ring
request served by the direct kernels."""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import workloads
from gpu_common import TOL, check_spmv, need_gpu, progress, rel_error

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2603_01915_amd")


def forced_escapes(seed=5):
    """Columns spread far apart: deltas at or above 2^30 are always escaped,
    and most values are distinct (value escapes)."""
    rng = np.random.default_rng(seed)
    A = sp.random(900, 100, density=0.06, format="csr", random_state=rng)
    A.sort_indices()
    ci = (A.indices.astype(np.int64) * 20_000_000).astype(np.int32)
    v = rng.standard_normal(A.nnz)
    v[::5] = 0.5
    return A.indptr.astype(np.int32), ci, v, 2 ** 31 - 1


def cases():
    rp, ci, v = workloads.rmat(scale=11, edge_factor=16)
    v = np.random.default_rng(6).standard_normal(len(v))  # value escapes too
    yield "rmat11", rp, ci, v, 2 ** 11
    rp, ci, v, n = forced_escapes()
    yield "forced", rp, ci, v, n
    rng = np.random.default_rng(7)
    rp, ci, v = workloads.band(m=1500, per_row=12, half=200)
    v = rng.standard_normal(len(v))  # every value distinct
    yield "band_distinct", rp, ci, v, 1500


CASES = list(cases())
LAYOUTS = [("row", 0), ("nnz", 32), ("nnz", 12)]


@pytest.mark.parametrize("case", range(len(CASES)), ids=[c[0] for c in CASES])
@pytest.mark.parametrize("layout,T", LAYOUTS)
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_in_stream_products(case, layout, T, dtype):
    torch = need_gpu()
    name, rp, ci, v, n = CASES[case]
    v = v.astype(dtype)
    m = len(rp) - 1
    progress("in-stream escapes %s %s T=%d %s" % (name, layout, T, dtype.__name__))
    A = P.Matrix.from_csr(rp, ci, v, n, layout=layout, lane_nnz=T, escape_in_stream=True)
    B = P.Matrix.from_csr(rp, ci, v, n, layout=layout, lane_nnz=T)
    ia = A.info()
    assert ia["escape_in_stream"] == 1
    assert B.info()["esc_value"] > 0
    r2, c2, v2 = A.decode_csr()
    torch.cuda.synchronize()
    assert np.array_equal(r2.cpu().numpy(), rp) and np.array_equal(c2.cpu().numpy(), ci)
    assert np.array_equal(v2.cpu().numpy().view(np.uint8), v.view(np.uint8))
    if n > 10 ** 8:  # columns far apart: decoding only (no x of that size)
        return
    x = workloads.vector(n, 7, dtype)
    xd = torch.from_numpy(x).cuda()
    y = A.spmv(xd)
    check_spmv(y.cpu().numpy(), rp, ci, v, x, None, 1.0, 0.0, dtype)
    assert torch.equal(y, B.spmv(xd))
    for k in (3, 8):
        X = workloads.vector(n, 4, dtype, k=k)
        Xd = torch.from_numpy(X).cuda()
        Y = A.spmm(Xd)
        Yref = oracle.spmm(rp, ci, v, X)
        Yn = Y.cpu().numpy()
        for c in range(k):
            assert rel_error(Yn[:, c], Yref[:, c], oracle.absmv(rp, ci, v, X[:, c])) <= TOL[dtype]
        assert torch.equal(Y, B.spmm(Xd))
    dY = workloads.vector(m, 6, dtype)
    dX = A.spmm_t(torch.from_numpy(dY).cuda().reshape(m, 1)).cpu().numpy()[:, 0]
    At = sp.csr_matrix((v.astype(np.float64), ci, rp), shape=(m, n)).T.tocsr()
    At.sort_indices()
    ref = oracle.spmtv(rp, ci, v, n, dY)
    assert rel_error(dX, ref, oracle.absmv(At.indptr, At.indices, At.data, dY)) <= TOL[dtype]


@pytest.mark.parametrize("layout,T", [(1, 0), (2, 8)])
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_in_stream_oracle_containers(tmp_path, layout, T, dtype):
    """The GPU decodes in-stream containers written by the oracle's encoder."""
    torch = need_gpu()
    for name, rp, ci, v, n in CASES:
        v = v.astype(dtype)
        progress("oracle in-stream container %s layout=%d T=%d %s" % (name, layout, T, dtype.__name__))
        path = str(tmp_path / (name + ".dtans"))
        oracle.encode(path, len(rp) - 1, n, rp, ci, v, layout=layout, lane_nnz=T, seed=11, esc_mode=1)
        A = P.Matrix.load(path)
        assert A.info()["escape_in_stream"] == 1
        _, c2, v2 = A.decode_csr()
        torch.cuda.synchronize()
        assert np.array_equal(c2.cpu().numpy(), ci)
        assert np.array_equal(v2.cpu().numpy().view(np.uint8), v.view(np.uint8))


def test_in_stream_ring_request_reads_directly():
    torch = need_gpu()
    name, rp, ci, v, n = CASES[0]
    progress("in-stream ring request")
    A = P.Matrix.from_csr(rp, ci, v, n, layout="row", escape_in_stream=True, stream_stage=P.STAGE_RING)
    assert A.info()["stream_stage"] == P.STAGE_DIRECT
    x = workloads.vector(n, 7, np.float64)
    y = A.spmv(torch.from_numpy(x).cuda())
    check_spmv(y.cpu().numpy(), rp, ci, v, x, None, 1.0, 0.0, np.float64)


def test_in_stream_device_encoder_unsupported():
    torch = need_gpu()
    name, rp, ci, v, n = CASES[0]
    with pytest.raises(P.DtansError):
        P.Matrix.from_csr(rp, ci, v, n, gpu_encode=True, escape_in_stream=True)
    torch.cuda.synchronize()
