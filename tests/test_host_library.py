"""Host side of libdtans, no GPU needed: the library's encoder is checked by the
oracle's decoder (cross-decode), the library's verifying loader accepts the
oracle's containers, error codes, options, statistics and the C ABI exports."""
import ctypes
import os
import re

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import workloads
from oracle import container

P = pytest.importorskip("paper_2603_01915_amd")
from paper_2603_01915_amd import _lib  # noqa: E402

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def rand_csr(m, n, dens, seed, dtype=np.float64, pool=None):
    rng = np.random.default_rng(seed)
    A = sp.random(m, n, density=dens, format="csr", random_state=rng)
    A.sort_indices()
    v = rng.standard_normal(A.nnz) if pool is None else rng.choice(rng.standard_normal(pool), A.nnz)
    return A.indptr.astype(np.int32), A.indices.astype(np.int32), v.astype(dtype)


def test_header_symbols_exported():
    """Every function declared in include/dtans.h is exported by libdtans.so."""
    text = open(os.path.join(ROOT, "include", "dtans.h")).read()
    names = set(re.findall(
        r"^\s*(?:dtans_status|void|const char \*|int64_t|int32_t)\s*\*?\s*(dtans_\w+)\s*\(",
        text, re.M))
    assert len(names) == 34
    lib = ctypes.CDLL(_lib.LIB_PATH)
    for n in sorted(names):
        assert hasattr(lib, n), n
    assert names == set(_lib.SIGNATURES)
    assert P.version().startswith("dtans")


LAYOUTS = [("row", 0), ("nnz", 4), ("nnz", 32), ("nnz", 100)]


@pytest.mark.parametrize("layout,T", LAYOUTS)
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_library_encoder_cross_decoded_by_oracle(tmp_path, layout, T, dtype):
    rp, ci, v = rand_csr(700, 500, 0.02, 1, dtype, pool=300)
    A = P.Matrix.from_csr(rp, ci, v, 500, layout=layout, lane_nnz=T)
    path = str(tmp_path / "lib.dtans")
    A.save(path)
    r2, c2, v2 = oracle.decode(path)
    assert np.array_equal(r2, rp) and np.array_equal(c2, ci)
    assert np.array_equal(v2.view(np.uint8), v.view(np.uint8))
    # and the Python big-integer container codec agrees too
    _, c3, v3 = container.decode(container.read(path))
    assert np.array_equal(c3, ci) and np.array_equal(v3.view(np.uint8), v.view(np.uint8))


@pytest.mark.parametrize("layout,T", [(1, 0), (2, 8), (2, 64)])
def test_library_loads_oracle_containers(tmp_path, layout, T):
    rp, ci, v = rand_csr(300, 200, 0.05, 2, pool=50)
    path = str(tmp_path / "or.dtans")
    oracle.encode(path, 300, 200, rp, ci, v, layout=layout, lane_nnz=T)
    A = P.Matrix.load(path)
    inf = A.info()
    assert inf["layout"] == layout and inf["nnz"] == len(ci)
    # saving it again reproduces the same bytes
    p2 = str(tmp_path / "again.dtans")
    A.save(p2)
    assert open(path, "rb").read() == open(p2, "rb").read()


def test_adversarial_cross_decode(tmp_path):
    rng = np.random.default_rng(3)
    n = 2 ** 31 - 1
    rows = [[], [7], [1, 2], [0, 0, 3], [], [2 ** 30, 2 ** 31 - 2], [4999], [], [5, 5, 5, 5, 5],
            list(range(100, 113)), list(range(0, 20000, 3))]
    rows += [sorted(rng.choice(10 ** 6, size=rng.integers(0, 9), replace=False)) for _ in range(300)]
    rp = np.zeros(len(rows) + 1, np.int64)
    rp[1:] = np.cumsum([len(r) for r in rows])
    ci = np.array([c for r in rows for c in r], np.int64).astype(np.int32)
    v = rng.standard_normal(len(ci))
    v[:6] = [0.0, -0.0, np.inf, -np.inf, np.nan, 5e-324]
    for layout, T in LAYOUTS:
        A = P.Matrix.from_csr(rp.astype(np.int32), ci, v, n, layout=layout, lane_nnz=T)
        path = str(tmp_path / ("adv_%s_%d.dtans" % (layout, T)))
        A.save(path)
        r2, c2, v2 = oracle.decode(path)
        assert np.array_equal(c2, ci) and np.array_equal(v2.view(np.uint8), v.view(np.uint8))
        assert P.Matrix.load(path).nnz == len(ci)


def test_empty_and_tiny(tmp_path):
    for m, n in ((0, 5), (5, 5), (1, 1)):
        rp = np.zeros(m + 1, np.int32)
        A = P.Matrix.from_csr(rp, np.zeros(0, np.int32), np.zeros(0), n)
        assert A.info()["words"] == 0
        path = str(tmp_path / "e.dtans")
        A.save(path)
        r2, c2, _ = oracle.decode(path)
        assert np.array_equal(r2, rp) and len(c2) == 0


def test_error_codes():
    rp = np.array([0, 2, 3], np.int32)
    with pytest.raises(P.DtansError) as e:
        P.Matrix.from_csr(rp, np.array([3, 1, 0], np.int32), np.ones(3), 5)
    assert e.value.status == _lib.EUNSORTED
    with pytest.raises(P.DtansError) as e:
        P.Matrix.from_csr(rp, np.array([1, 9, 0], np.int32), np.ones(3), 5)
    assert e.value.status == _lib.ERANGE
    with pytest.raises(P.DtansError) as e:
        P.Matrix.from_csr(np.array([0, 2, 4], np.int32), np.array([1, 2, 0], np.int32), np.ones(3), 5)
    assert e.value.status == _lib.EINVAL
    with pytest.raises(P.DtansError) as e:
        P.Matrix.from_csr(rp, np.array([1, 2, 0], np.int32), np.ones(3), 5, layout="nnz", lane_nnz=6)
    assert e.value.status == _lib.EINVAL
    with pytest.raises(P.DtansError) as e:
        P.Matrix.load("/nonexistent/file.dtans")
    assert e.value.status == _lib.EIO


def test_sort_rows_option(tmp_path):
    rp = np.array([0, 3, 5], np.int32)
    ci = np.array([4, 0, 2, 3, 1], np.int32)
    v = np.array([1.0, 2.0, 3.0, 4.0, 5.0])
    A = P.Matrix.from_csr(rp, ci, v, 6, sort_rows=True)
    path = str(tmp_path / "s.dtans")
    A.save(path)
    _, c2, v2 = oracle.decode(path)
    assert list(c2) == [0, 2, 4, 1, 3] and list(v2) == [2.0, 3.0, 1.0, 5.0, 4.0]


def test_corrupted_container_rejected(tmp_path):
    rp, ci, v = rand_csr(200, 100, 0.05, 4, pool=20)
    path = str(tmp_path / "c.dtans")
    P.Matrix.from_csr(rp, ci, v, 100).save(path)
    data = bytearray(open(path, "rb").read())
    for off in (400, len(data) // 2, len(data) - 2):
        bad = bytearray(data)
        bad[off] ^= 0x01
        open(path, "wb").write(bad)
        with pytest.raises(P.DtansError) as e:
            P.Matrix.load(path)
        assert e.value.status == _lib.ECORRUPT
    # consistent checksum but one word too few in a wave: the verifying
    # decode notices the mismatch
    open(path, "wb").write(data)
    c = container.read(path)
    end0 = int(c.word_off[1])
    c.words = np.delete(c.words, end0 - 1)
    c.word_off = (c.word_off.astype(np.int64) - np.r_[0, np.ones(len(c.word_off) - 1, np.int64)]).astype(np.uint64)
    container.write(path, c)
    with pytest.raises(P.DtansError) as e:
        P.Matrix.load(path)
    assert e.value.status == _lib.ECORRUPT


def test_wide_fp32_value_symbol_rejected(tmp_path):
    """An FP32 container whose value table holds a symbol wider than 32 bits
    (consistent checksum, written by the oracle's container writer) is
    refused on load."""
    rp = np.array([0, 2, 3], np.int32)
    ci = np.array([0, 1, 1], np.int32)
    v = np.array([1.5, 2.5, -1.0], np.float32)
    path = str(tmp_path / "w.dtans")
    P.Matrix.from_csr(rp, ci, v, 2).save(path)
    c = container.read(path)
    i = next(j for j, s in enumerate(c.vtab.symbol) if s is not None and s != container.ESC)
    old = c.vtab.symbol[i]
    c.vtab.symbol = [(s | (1 << 40)) if s == old else s for s in c.vtab.symbol]
    container.write(path, c)
    with pytest.raises(P.DtansError) as e:
        P.Matrix.load(path)
    assert e.value.status == _lib.ECORRUPT


def test_info_statistics():
    rp, ci, v = workloads.stencil27(16)
    A = P.Matrix.from_csr(rp, ci, v, 16 ** 3, layout="row")
    inf = A.info()
    assert inf["csr_bytes"] == 4 * (16 ** 3 + 1) + 12 * len(ci)
    assert inf["coo_bytes"] == 16 * len(ci)
    assert inf["table_bytes"] == 4096 * 16
    assert inf["stream_bytes"] == 4 * inf["words"] + 4 * inf["esc_delta"] + 8 * inf["esc_value"]
    assert inf["total_bytes"] < inf["csr_bytes"]
    # every symbol costs at least log2(K/M) = 4 bits: at least 1 byte per nonzero
    assert inf["stream_bytes"] >= len(ci)
    # the value alphabet has at most 216 distinct stencil values, all in the table
    assert inf["value_symbols"] <= 216 and inf["esc_value"] == 0
    assert 0 < inf["value_entropy"] <= np.log2(216) + 1e-9
    assert inf["value_cross_entropy"] >= inf["value_entropy"] - 1e-9
    # default first deltas relative to the row: a stencil's are a few offsets,
    # all in the table; with the paper's raw columns most rows escape theirs
    assert inf["first_delta_column"] == 0 and inf["esc_delta"] == 0
    B = P.Matrix.from_csr(rp, ci, v, 16 ** 3, layout="row", first_delta_column=True)
    infb = B.info()
    assert infb["first_delta_column"] == 1 and infb["esc_delta"] > 0
    assert inf["stream_bytes"] < infb["stream_bytes"]


@pytest.mark.parametrize("layout,T", [("row", 0), ("nnz", 32), ("nnz", 12)])
@pytest.mark.parametrize("first_column", [False, True])
def test_first_delta_modes_cross_decode(tmp_path, layout, T, first_column):
    """Both first-delta forms round-trip through the oracle's decoder and the
    Python codec, with leading and inner empty rows, rows crossing lanes and
    columns far from the diagonal (escaped first deltas in either mode)."""
    rng = np.random.default_rng(5)
    m, n = 400, 3000
    rows = [[]] * 3 + [sorted(rng.choice(n, size=rng.integers(0, 20), replace=False))
                       for _ in range(m - 6)] + [[], [n - 1], [0, 1, 2]]
    rp = np.zeros(m + 1, np.int32)
    rp[1:] = np.cumsum([len(r) for r in rows])
    ci = np.array([c for r in rows for c in r], np.int32)
    v = rng.choice(rng.standard_normal(40), len(ci))
    A = P.Matrix.from_csr(rp, ci, v, n, layout=layout, lane_nnz=T, first_delta_column=first_column)
    path = str(tmp_path / "m.dtans")
    A.save(path)
    assert oracle.read_header(path)["first_mode"] == (0 if first_column else 1)
    r2, c2, v2 = oracle.decode(path)
    assert np.array_equal(r2, rp) and np.array_equal(c2, ci) and np.array_equal(v2, v)
    _, c3, v3 = container.decode(container.read(path))
    assert np.array_equal(c3, ci) and np.array_equal(v3, v)
    # and the oracle's encoder in the same mode is read back by the library
    p2 = str(tmp_path / "o.dtans")
    oracle.encode(p2, m, n, rp, ci, v, layout=1 if layout == "row" else 2, lane_nnz=T,
                  first_mode=0 if first_column else 1)
    B = P.Matrix.load(p2)
    assert B.info()["first_delta_column"] == (1 if first_column else 0)


def test_all_bases_256_word_count():
    # one delta symbol and one value symbol: both get multiplicity 256, every
    # check extracts, and a lane of S segments stores S + 2 words (Sec. IV-D)
    S = 9
    m = 64
    rows = [list(range(1, 4 * S + 1))] * m
    rp = np.arange(0, m * 4 * S + 1, 4 * S, dtype=np.int32)
    ci = np.array([c for r in rows for c in r], np.int32)
    A = P.Matrix.from_csr(rp, ci, np.ones(len(ci)), 4 * S + 1, layout="row", max_mult=256,
                          first_delta_column=True)
    assert A.info()["words"] == m * (S + 2)
    assert A.info()["direct_table"] == 0


def test_multiplicity_cap():
    """max_mult caps every symbol's slot count: with the default cap of 255 the
    device table holds the bases directly; a single dominant symbol gets 255
    slots (not 256), which costs a little more than the 4-bit floor; the
    encoding still round-trips through the oracle's decoder."""
    S, m = 9, 64
    rows = [list(range(1, 4 * S + 1))] * m
    rp = np.arange(0, m * 4 * S + 1, 4 * S, dtype=np.int32)
    ci = np.array([c for r in rows for c in r], np.int32)
    v = np.ones(len(ci))
    kw = dict(layout="row", first_delta_column=True)  # one delta symbol
    A = P.Matrix.from_csr(rp, ci, v, 4 * S + 1, **kw)
    B = P.Matrix.from_csr(rp, ci, v, 4 * S + 1, max_mult=256, **kw)
    assert A.info()["direct_table"] == 1 and B.info()["direct_table"] == 0
    assert B.info()["words"] <= A.info()["words"] <= m * (S + 3)
    C = P.Matrix.from_csr(rp, ci, v, 4 * S + 1, max_mult=16, **kw)
    assert C.info()["words"] > A.info()["words"]
    for M in (A, B, C):
        import tempfile, os
        with tempfile.TemporaryDirectory() as td:
            path = os.path.join(td, "m.dtans")
            M.save(path)
            r2, c2, v2 = oracle.decode(path)
            assert np.array_equal(c2, ci) and np.array_equal(v2, v)
    with pytest.raises(P.DtansError):
        P.Matrix.from_csr(rp, ci, v, 4 * S + 1, max_mult=257)


def test_compression_closed_form_bound():
    # at least 4 bits per symbol: compression vs FP64 CSR is at most 12x
    # (Sec. V-A prints 11.77x as its best), vs FP32 CSR at most 8x (7.86x)
    rp, ci, v = workloads.stencil27(24)
    for dt, bound in ((np.float64, 12.0), (np.float32, 8.0)):
        A = P.Matrix.from_csr(rp, ci, v.astype(dt), 24 ** 3)
        inf = A.info()
        assert inf["csr_bytes"] / inf["stream_bytes"] <= bound


def _auto_resolution(rp, ci, v, n, **kw):
    """What dtans_encode_csr resolves for the given (partly automatic) options."""
    A = P.Matrix.from_csr(rp, ci, v, n, **kw)
    info = A.info()
    return info["layout"], info["lane_nnz"]


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_autotune_candidates_regular(dtype):
    """A regular many-row matrix: the automatic encoding (row layout, direct
    reads, the library's own launch shape) comes first, the other shapes and
    the LDS-ring kernels follow, then the nonzero layout with lane lengths
    around its automatic choice; every direct-read shape respects the CU's
    wave slots and the LDS-limited workgroups per CU."""
    rp, ci, v = workloads.band(200_000, 8, 32, seed=3)
    v = v.astype(dtype)
    c = P.autotune_candidates(rp, len(ci), dtype)
    assert c[0]["layout"] == P.LAYOUT_ROW and c[0]["lane_nnz"] == 0
    assert c[0]["stream_stage"] == P.STAGE_DIRECT
    lay, T = _auto_resolution(rp, ci, v, 200_000)
    assert (lay, T) == (c[0]["layout"], c[0]["lane_nnz"])
    info = P.Matrix.from_csr(rp, ci, v, 200_000).info()
    assert info["waves_per_wg"] == c[0]["waves_per_wg"]
    assert info["stream_stage"] == P.STAGE_DIRECT
    maxwg = 2 if dtype == np.float64 else 3
    # the library's shape: two 16-wave workgroups (8 waves per SIMD)
    assert (c[0]["waves_per_wg"], c[0]["wg_per_cu"]) == (16, 2)
    keys = [tuple(o.values()) for o in c]
    assert len(set(keys)) == len(keys)
    Ts = sorted({o["lane_nnz"] for o in c if o["layout"] == P.LAYOUT_NNZ})
    assert len(Ts) >= 2 and all(t % 4 == 0 and 32 <= t <= 512 for t in Ts)
    for lay in (P.LAYOUT_ROW, P.LAYOUT_NNZ):
        assert {o["stream_stage"] for o in c if o["layout"] == lay} == {P.STAGE_RING, P.STAGE_DIRECT}
    for o in c:
        if o["stream_stage"] == P.STAGE_RING:
            assert o["waves_per_wg"] in (4, 8, 16) and o["wg_per_cu"] == 0
            continue
        slots = 32 if o["layout"] == P.LAYOUT_ROW else 28
        assert 1 <= o["wg_per_cu"] <= maxwg
        assert 2 <= o["waves_per_wg"] <= min(16, slots // o["wg_per_cu"])
    # encodings are grouped: each (layout, lane_nnz) appears in one run
    runs = [k[:2] for i, k in enumerate(keys) if i == 0 or keys[i - 1][:2] != k[:2]]
    assert len(runs) == len(set(runs))
    # a fixed stage is kept
    c = P.autotune_candidates(rp, len(ci), dtype, layout="row", stream_stage=P.STAGE_DIRECT)
    assert c and all(o["stream_stage"] == P.STAGE_DIRECT for o in c)


def test_autotune_candidates_small_and_fixed():
    rp, ci, v = rand_csr(300, 200, 0.05, 2)
    c = P.autotune_candidates(rp, len(ci))
    lay, T = _auto_resolution(rp, ci, v, 200)
    assert lay == P.LAYOUT_NNZ and (c[0]["layout"], c[0]["lane_nnz"]) == (lay, T)
    # fixed fields are kept in every candidate
    c = P.autotune_candidates(rp, len(ci), layout="nnz", wg_per_cu=1)
    assert c and all(o["layout"] == P.LAYOUT_NNZ and o["wg_per_cu"] == 1 for o in c)
    c = P.autotune_candidates(rp, len(ci), layout="row", waves_per_wg=4)
    assert c and all(o["layout"] == P.LAYOUT_ROW and o["waves_per_wg"] == 4 for o in c)
    c = P.autotune_candidates(rp, len(ci), layout="nnz", lane_nnz=64, waves_per_wg=8, wg_per_cu=2,
                              stream_stage=P.STAGE_DIRECT)
    assert c == [{"layout": P.LAYOUT_NNZ, "lane_nnz": 64, "waves_per_wg": 8, "wg_per_cu": 2,
                  "stream_stage": P.STAGE_DIRECT}]
    # several right-hand sides: direct and ring candidates as for SpMV
    c = P.autotune_candidates(rp, len(ci), k=8)
    assert {o["stream_stage"] for o in c} == {P.STAGE_DIRECT, P.STAGE_RING}
    # empty matrix: one encoding, still valid shapes
    c = P.autotune_candidates(np.zeros(1, np.int32), 0)
    assert c and c[0]["layout"] == P.LAYOUT_NNZ


def test_autotune_candidates_errors():
    rp, ci, v = rand_csr(50, 40, 0.1, 3)
    with pytest.raises(P.DtansError):
        P.autotune_candidates(rp, len(ci) + 1)            # row_ptr does not end at nnz
    with pytest.raises(P.DtansError):
        P.autotune_candidates(rp, len(ci), lane_nnz=6)     # not a multiple of 4
    with pytest.raises(P.DtansError):
        P.autotune_candidates(rp, len(ci), k=0)
    with pytest.raises(P.DtansError):
        P.autotune_candidates(rp, len(ci), waves_per_wg=17)
    with pytest.raises(P.DtansError):
        P.autotune_candidates(rp, len(ci), stream_stage=3)
    bad = rp.copy()
    bad[10] = bad[11] + 1
    with pytest.raises(P.DtansError):
        P.autotune_candidates(bad, len(ci))


def test_autotune_without_gpu_fails_loudly():
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("a GPU is present; the GPU tests cover the autotuner")
    rp, ci, v = rand_csr(64, 64, 0.1, 4)
    with pytest.raises(P.DtansError) as e:
        P.autotune(rp, ci, v, 64, budget_s=1.0)
    assert e.value.status == _lib.EHIP


def test_transpose_csr_matches_scipy():
    """The host transpose used for an encoded A^T (autograd backward) equals
    scipy's, including empty rows and columns and a ragged tail."""
    from paper_2603_01915_amd.autograd import transpose_csr

    for m, n, dens, seed in ((37, 53, 0.08, 1), (1, 9, 0.5, 2), (64, 3, 0.4, 3), (5, 5, 0.0, 4)):
        rp, ci, v = rand_csr(m, n, dens, seed)
        rpt, cit, vt = transpose_csr(rp, ci, v, n)
        T = sp.csr_matrix((v, ci, rp), shape=(m, n)).T.tocsr()
        T.sort_indices()
        assert rpt.dtype == np.int32 and cit.dtype == np.int32 and vt.dtype == v.dtype
        assert np.array_equal(rpt, T.indptr) and np.array_equal(cit, T.indices)
        assert np.array_equal(vt, T.data)
    with pytest.raises(ValueError):
        transpose_csr(np.array([0, 1], np.int32), np.array([4], np.int32), np.ones(1), 4)


def test_symmetric_split():
    """Strict upper triangle and diagonal (duplicates summed) of a symmetric
    matrix, against scipy; S + S^T + diag gives the matrix back."""
    rng = np.random.default_rng(8)
    B = sp.random(90, 90, density=0.05, format="csr", random_state=rng)
    A = (B + B.T + sp.diags(rng.standard_normal(90))).tocsr()
    A.sort_indices()
    rpu, ciu, vu, d = P.symmetric_split(A.indptr, A.indices, A.data)
    U = sp.triu(A, k=1).tocsr()
    U.sort_indices()
    assert np.array_equal(rpu, U.indptr) and np.array_equal(ciu, U.indices) and np.array_equal(vu, U.data)
    assert np.array_equal(d, A.diagonal())
    S = sp.csr_matrix((vu, ciu, rpu), shape=(90, 90))
    assert abs(S + S.T + sp.diags(d) - A).max() == 0
    # duplicated diagonal entries are summed
    rpu, ciu, vu, d = P.symmetric_split(np.array([0, 2, 3], np.int32), np.array([0, 0, 1], np.int32),
                                        np.array([1.5, 2.0, 4.0]))
    assert list(d) == [3.5, 4.0] and len(ciu) == 0 and list(rpu) == [0, 0, 0]
