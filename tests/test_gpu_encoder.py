"""The encoder's per-nonzero passes on the GPU (dtans_encode_csr_gpu: keys,
histograms, symbols, words, escape regions): every container is
byte-identical to the host encoder's and decoded exactly by the oracle, over
both layouts, value types and first-delta modes, rows that are empty,
duplicated, very long (many 16-step flag words) or escape-heavy, ragged last
lanes and waves, degenerate sizes, the all-256-bases case where every check
extracts, and the full-size stencil and pruned weight."""
import time

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import workloads
from gpu_common import need_gpu, progress

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2603_01915_amd")

LAYOUTS = [("row", 0), ("nnz", 4), ("nnz", 32), ("nnz", 100)]


def rand_csr(m, n, dens, seed, dtype=np.float64, pool=None):
    rng = np.random.default_rng(seed)
    A = sp.random(m, n, density=dens, format="csr", random_state=rng)
    A.sort_indices()
    v = rng.standard_normal(A.nnz) if pool is None else rng.choice(rng.standard_normal(pool), A.nnz)
    return A.indptr.astype(np.int32), A.indices.astype(np.int32), v.astype(dtype)


def both(tmp_path, tag, rp, ci, v, n, **kw):
    """Encode on the host and with the GPU passes; the two files must be
    equal byte for byte, and the oracle must decode the GPU's exactly."""
    need_gpu()
    progress("encoder %s" % tag)
    A = P.Matrix.from_csr(rp, ci, v, n, **kw)
    B = P.Matrix.from_csr(rp, ci, v, n, gpu_encode=True, **kw)
    pa, pb = str(tmp_path / (tag + "_host.dtans")), str(tmp_path / (tag + "_gpu.dtans"))
    A.save(pa)
    B.save(pb)
    assert open(pa, "rb").read() == open(pb, "rb").read(), tag
    r2, c2, v2 = oracle.decode(pb)
    assert np.array_equal(r2, rp) and np.array_equal(c2, ci)
    assert np.array_equal(np.asarray(v2).view(np.uint8), np.asarray(v).view(np.uint8))
    return B


@pytest.mark.parametrize("layout,T", LAYOUTS)
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_random_matrices(tmp_path, layout, T, dtype):
    rp, ci, v = rand_csr(700, 500, 0.02, 1, dtype, pool=300)
    both(tmp_path, "rand_%s_%d" % (layout, T), rp, ci, v, 500, layout=layout, lane_nnz=T)


def test_adversarial_rows(tmp_path):
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
        both(tmp_path, "adv_%s_%d" % (layout, T), rp.astype(np.int32), ci, v, n, layout=layout, lane_nnz=T)


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_escape_heavy(tmp_path, dtype):
    """More distinct deltas and values than 4096 slots hold: thousands of
    escapes of both kinds, in every layout and both first-delta modes."""
    rng = np.random.default_rng(21)
    m = 400
    rows = [sorted(rng.choice(10 ** 7, size=rng.integers(0, 40), replace=False)) for _ in range(m)]
    rp = np.zeros(m + 1, np.int64)
    rp[1:] = np.cumsum([len(r) for r in rows])
    ci = np.array([c for r in rows for c in r], np.int64).astype(np.int32)
    v = rng.standard_normal(len(ci)).astype(dtype)
    for layout, T in (("row", 0), ("nnz", 8), ("nnz", 100)):
        for fdc in (False, True):
            B = both(tmp_path, "esc_%s_%d_%d" % (layout, T, fdc), rp.astype(np.int32), ci, v, 10 ** 7,
                     layout=layout, lane_nnz=T, first_delta_column=fdc)
            inf = B.info()
            assert inf["esc_delta"] > 1000 and inf["esc_value"] > 1000


def test_sort_rows_option(tmp_path):
    """Rows given with unsorted columns and sort_rows: both encoders sort them
    the same way (values follow their columns)."""
    rng = np.random.default_rng(41)
    rp, ci, v = rand_csr(500, 400, 0.03, 5)
    perm_ci, perm_v = ci.copy(), v.copy()
    for i in range(500):
        b, e = rp[i], rp[i + 1]
        p = rng.permutation(e - b)
        perm_ci[b:e] = ci[b:e][p]
        perm_v[b:e] = v[b:e][p]
    need_gpu()
    A = P.Matrix.from_csr(rp, perm_ci, perm_v, 400, sort_rows=True)
    B = P.Matrix.from_csr(rp, perm_ci, perm_v, 400, sort_rows=True, gpu_encode=True)
    pa, pb = str(tmp_path / "h.dtans"), str(tmp_path / "g.dtans")
    A.save(pa)
    B.save(pb)
    assert open(pa, "rb").read() == open(pb, "rb").read()
    r2, c2, v2 = oracle.decode(pb)
    assert np.array_equal(c2, ci) and np.array_equal(np.asarray(v2), v)


def test_long_rows_many_flag_words(tmp_path):
    """Rows of 1..1500 nonzeros side by side in one wave: lanes start their
    backward pass at very different steps and use up to 24 flag words."""
    rng = np.random.default_rng(9)
    m, n = 200, 50000
    lens = rng.integers(1, 1500, size=m)
    lens[::17] = 0
    rp = np.zeros(m + 1, np.int64)
    rp[1:] = np.cumsum(lens)
    ci = np.concatenate([np.sort(rng.choice(n, size=k, replace=False)) for k in lens]).astype(np.int32)
    v = rng.choice(rng.standard_normal(40), size=len(ci)).astype(np.float32)
    both(tmp_path, "long_rows", rp.astype(np.int32), ci, v, n, layout="row")
    both(tmp_path, "long_rows_nnz", rp.astype(np.int32), ci, v, n, layout="nnz", lane_nnz=512)


def test_degenerate_sizes(tmp_path):
    for m, n in ((0, 5), (5, 5), (1, 1)):
        rp = np.zeros(m + 1, np.int32)
        B = both(tmp_path, "empty_%d" % m, rp, np.zeros(0, np.int32), np.zeros(0), n)
        assert B.info()["words"] == 0
    # one nonzero; one full wave plus one lane
    both(tmp_path, "one", np.array([0, 1], np.int32), np.array([0], np.int32), np.ones(1), 1)
    rp, ci, v = rand_csr(65, 65, 0.3, 4)
    both(tmp_path, "wave_plus_one", rp, ci, v, 65, layout="row")
    # the same from device arrays
    torch = need_gpu()
    cases = [(np.zeros(1, np.int32), np.zeros(0, np.int32), np.zeros(0), 5),
             (np.zeros(6, np.int32), np.zeros(0, np.int32), np.zeros(0), 5),
             (np.array([0, 1], np.int32), np.array([0], np.int32), np.ones(1), 1), (rp, ci, v, 65)]
    for q, (r, c, x, n) in enumerate(cases):
        A = P.Matrix.from_csr(r, c, x, n)
        B = P.Matrix.from_csr_device(*device_arrays(torch, r, c, x), n)
        pa, pb = str(tmp_path / ("dh%d" % q)), str(tmp_path / ("dd%d" % q))
        A.save(pa)
        B.save(pb)
        assert open(pa, "rb").read() == open(pb, "rb").read(), q


def test_all_bases_256(tmp_path):
    """One delta and one value symbol of multiplicity 256: every check
    extracts, no group loads a word (S + 2 words per lane, Sec. IV-D)."""
    S, m = 9, 64
    rp = np.arange(0, m * 4 * S + 1, 4 * S, dtype=np.int32)
    ci = np.tile(np.arange(1, 4 * S + 1, dtype=np.int32), m)
    B = both(tmp_path, "bases256", rp, ci, np.ones(len(ci)), 4 * S + 1, layout="row", max_mult=256,
             first_delta_column=True)
    assert B.info()["words"] == m * (S + 2)


def test_full_size_stencil_and_pruned(tmp_path):
    torch = need_gpu()
    rp, ci, v = workloads.stencil27(128)
    n = 128 ** 3
    t0 = time.perf_counter()
    P.Matrix.from_csr(rp, ci, v, n, layout="row")
    th = time.perf_counter() - t0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    both(tmp_path, "stencil128", rp, ci, v, n, layout="row")
    progress("stencil 128^3: host encode %.2f s; host + GPU encodes and checks %.2f s"
             % (th, time.perf_counter() - t0))
    rp, ci, v = workloads.pruned_weight()
    both(tmp_path, "pruned", rp, ci, v, 4096)


def test_full_size_rmat(tmp_path):
    """R-MAT scale 22 (2^22 rows, 67 M nonzeros, tens of millions of escaped
    deltas), from host and from device arrays."""
    torch = need_gpu()
    rp, ci, v = workloads.rmat(22)
    n = 1 << 22
    B = both(tmp_path, "rmat22", rp, ci, v, n)
    assert B.info()["esc_delta"] > 10 ** 7
    D = P.Matrix.from_csr_device(*device_arrays(torch, rp, ci, v), n)
    pd = str(tmp_path / "rmat22_dev.dtans")
    D.save(pd)
    assert open(pd, "rb").read() == open(str(tmp_path / "rmat22_gpu.dtans"), "rb").read()


def device_arrays(torch, rp, ci, v):
    return (torch.from_numpy(np.ascontiguousarray(rp, np.int32)).cuda(),
            torch.from_numpy(np.ascontiguousarray(ci, np.int32)).cuda(),
            torch.from_numpy(np.ascontiguousarray(v)).cuda())


@pytest.mark.parametrize("layout,T", LAYOUTS)
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_device_inputs_identical(tmp_path, layout, T, dtype):
    """dtans_encode_csr_device (CSR arrays already in device memory) writes
    the host encoder's container, including escape-heavy and empty rows."""
    torch = need_gpu()
    rng = np.random.default_rng(33)
    m = 300
    rows = [sorted(rng.choice(10 ** 6, size=rng.integers(0, 30), replace=False)) for _ in range(m)]
    rows[5] = []
    rows[6] = list(range(0, 3000, 2))
    rp = np.zeros(m + 1, np.int64)
    rp[1:] = np.cumsum([len(r) for r in rows])
    rp = rp.astype(np.int32)
    ci = np.array([c for r in rows for c in r], np.int64).astype(np.int32)
    v = rng.choice(rng.standard_normal(6000), size=len(ci)).astype(dtype)
    progress("device inputs %s %d %s" % (layout, T, dtype.__name__))
    A = P.Matrix.from_csr(rp, ci, v, 10 ** 6, layout=layout, lane_nnz=T)
    B = P.Matrix.from_csr_device(*device_arrays(torch, rp, ci, v), 10 ** 6, layout=layout, lane_nnz=T)
    pa, pb = str(tmp_path / "h.dtans"), str(tmp_path / "d.dtans")
    A.save(pa)
    B.save(pb)
    assert open(pa, "rb").read() == open(pb, "rb").read()
    r2, c2, v2 = oracle.decode(pb)
    assert np.array_equal(r2, rp) and np.array_equal(c2, ci)
    assert np.array_equal(np.asarray(v2).view(np.uint8), v.view(np.uint8))


def test_device_inputs_errors():
    """Bad columns in device arrays give the host encoder's error class and
    the first failing row (a serial scan's first error), and no handle."""
    torch = need_gpu()
    from paper_2603_01915_amd import _lib

    rp = np.array([0, 2, 4, 6, 8], np.int32)
    good = np.array([1, 3, 0, 2, 5, 6, 1, 7], np.int32)
    v = np.ones(8)
    cases = [
        (np.array([1, 3, 0, 2, 6, 5, 1, 9], np.int32), "EUNSORTED", 2),  # row 2 unsorted before row 3 range
        (np.array([1, 3, 0, 8, 6, 5, 1, 7], np.int32), "ERANGE", 1),     # 8 >= n in row 1
        (np.array([1, 3, -1, 2, 5, 6, 1, 7], np.int32), "ERANGE", 1),
        (np.array([3, 1, 0, 2, 5, 6, 1, 7], np.int32), "EUNSORTED", 0),
    ]
    progress("device inputs: error rows")
    for ci, cls, row in cases:
        for path in ("host", "gpu", "device"):
            with pytest.raises(_lib.DtansError) as ei:
                if path == "device":
                    P.Matrix.from_csr_device(*device_arrays(torch, rp, ci, v), 8)
                else:
                    P.Matrix.from_csr(rp, ci, v, 8, gpu_encode=path == "gpu")
            assert str(ei.value).find(cls) >= 0 and str(ei.value).endswith("row %d" % row), (str(ei.value), path)
    B = P.Matrix.from_csr_device(*device_arrays(torch, rp, good, v), 8)
    assert B.nnz == 8
    with pytest.raises(_lib.DtansError):
        P.Matrix.from_csr_device(*device_arrays(torch, rp, good, v), 8, layout="row", lane_nnz=0,
                                 max_mult=300)
