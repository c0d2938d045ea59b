"""Row-sorted (SELL-C-sigma) base for CSR-dtANS: the paper names base formats
other than CSR as the next step (Sec. VII).  With a window sigma (a multiple
of C = 64, the lanes of a wave), rows are encoded sorted by descending length
within each window of sigma rows, ties in their original order (the sigma
sorting of SELL-C-sigma, Kreutzer et al. 2014), and the order is stored.
Pins:

* the order itself on hand-made row lengths (stable, descending, per window);
* the C oracle and the Python container codec write identical bytes from the
  same tables and decode each other's containers back to the original rows;
* a sorted container's words are those of the row-permuted CSR matrix encoded
  in CSR order (the sort changes nothing but the order of the rows);
* the library's encoder writes containers both oracles decode, and loads and
  re-saves oracle-written ones unchanged; malformed orders are rejected.
"""
import struct

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import paper_2603_01915_amd as P
from oracle import container


def _rand(m, n, seed, dtype=np.float64, pool=30):
    rng = np.random.default_rng(seed)
    lens = rng.choice([0, 1, 2, 3, 5, 9, 17, 40], size=m)
    rows = [sorted(rng.choice(n, size=min(n, k), replace=False)) for k in lens]
    rp = np.zeros(m + 1, np.int64)
    rp[1:] = np.cumsum([len(r) for r in rows])
    ci = np.array([c for r in rows for c in r], np.int64)
    v = rng.choice(rng.standard_normal(pool), size=len(ci)).astype(dtype)
    return rp.astype(np.int32), ci.astype(np.int32), v


def test_order_by_hand():
    lens = [1, 3, 3, 0, 2] + [5] * 59 + [0, 7, 7, 1]
    order = container.sigma_order(lens, 64)
    # window 0: the 59 rows of length 5 (rows 5..63, in order), then rows 1, 2
    # (length 3, in order), 4, 0, 3; window 1: rows 65, 66, 67, 64
    assert order[:59] == list(range(5, 64))
    assert order[59:64] == [1, 2, 4, 0, 3]
    assert order[64:] == [65, 66, 67, 64]


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("sigma", [64, 128, 1024])
def test_oracles_agree_sorted(tmp_path, dtype, sigma):
    rp, ci, v = _rand(300, 200, 3, dtype)
    m, n = 300, 200
    dt = 2 if dtype == np.float64 else 1
    p1 = str(tmp_path / "c.dtans")
    oracle.encode(p1, m, n, rp, ci, v, seed=21, sigma=sigma)
    assert oracle.read_header(p1)["sigma"] == sigma
    r2, c2, v2 = oracle.decode(p1)
    assert np.array_equal(r2, rp) and np.array_equal(c2, ci) and np.array_equal(v2, v)
    c = container.read(p1)
    assert c.sigma == sigma and list(c.perm) == container.sigma_order(np.diff(rp), sigma)
    r3, c3, v3 = container.decode(c)
    assert np.array_equal(r3, rp) and np.array_equal(c3, ci) and np.array_equal(v3, v)
    c6 = container.encode(m, n, rp, ci, v, dt, 1, 0, tables=(c.dtab, c.vtab), seed=c.seed, sigma=sigma)
    p2 = str(tmp_path / "p.dtans")
    container.write(p2, c6)
    assert open(p1, "rb").read() == open(p2, "rb").read()


def test_sorted_is_permuted_csr(tmp_path):
    """The words of a sorted container are those of the row-permuted matrix
    encoded in CSR order with the same tables."""
    rp, ci, v = _rand(500, 300, 4)
    m, n = 500, 300
    perm = container.sigma_order(np.diff(rp), 128)
    A = sp.csr_matrix((v, ci, rp), shape=(m, n))[perm]
    A.sort_indices()
    p1, p2 = str(tmp_path / "s.dtans"), str(tmp_path / "q.dtans")
    oracle.encode(p1, m, n, rp, ci, v, seed=5, sigma=128)
    c1 = container.read(p1)
    c2 = container.encode(m, n, A.indptr, A.indices, A.data, 2, 1, 0, tables=(c1.dtab, c1.vtab), seed=5)
    assert np.array_equal(c1.words, c2.words) and np.array_equal(c1.row_ptr, c2.row_ptr)
    assert np.array_equal(c1.escd, c2.escd) and np.array_equal(c1.escv, c2.escv)


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("sigma", [64, 512])
@pytest.mark.parametrize("esc", [False, True])
def test_library_sorted_containers(tmp_path, dtype, sigma, esc):
    rp, ci, v = _rand(900, 700, 6, dtype, pool=6000)
    A = P.Matrix.from_csr(rp, ci, v, 700, sort_window=sigma, escape_in_stream=esc)
    inf = A.info()
    assert inf["sort_window"] == sigma and inf["layout"] == P.LAYOUT_ROW
    path = str(tmp_path / "lib.dtans")
    A.save(path)
    r2, c2, v2 = oracle.decode(path)
    assert np.array_equal(r2, rp) and np.array_equal(c2, ci)
    assert np.array_equal(v2.view(np.uint8), v.view(np.uint8))
    assert oracle.read_header(path)["sigma"] == sigma
    p2 = str(tmp_path / "again.dtans")
    P.Matrix.load(path).save(p2)
    assert open(path, "rb").read() == open(p2, "rb").read()


def test_library_loads_oracle_sorted(tmp_path):
    rp, ci, v = _rand(400, 300, 7)
    path = str(tmp_path / "or.dtans")
    oracle.encode(path, 400, 300, rp, ci, v, sigma=192)
    A = P.Matrix.load(path)
    assert A.info()["sort_window"] == 192
    p2 = str(tmp_path / "again.dtans")
    A.save(p2)
    assert open(path, "rb").read() == open(p2, "rb").read()


def test_invalid_windows_and_orders(tmp_path):
    rp, ci, v = _rand(200, 100, 8)
    with pytest.raises(P.DtansError):
        P.Matrix.from_csr(rp, ci, v, 100, sort_window=100)
    with pytest.raises(P.DtansError):
        P.Matrix.from_csr(rp, ci, v, 100, layout="nnz", lane_nnz=8, sort_window=64)
    with pytest.raises(oracle.OracleError):
        oracle.encode(str(tmp_path / "x.dtans"), 200, 100, rp, ci, v, layout=2, lane_nnz=8, sigma=64)
    # stored orders that are not the sorted one: two tied rows out of their
    # original order, and a row moved to another window
    path = str(tmp_path / "o.dtans")
    oracle.encode(path, 200, 100, rp, ci, v, sigma=64)
    c0 = container.read(path)
    lens = np.diff(c0.row_ptr)
    tie = next(r for r in range(63) if lens[r] == lens[r + 1])
    bad = str(tmp_path / "bad.dtans")
    for a, b in ((tie, tie + 1), (0, 64)):
        c = container.read(path)
        c.perm = c.perm.copy()
        c.perm[a], c.perm[b] = c.perm[b], c.perm[a]
        container.write(bad, c)
        with pytest.raises(oracle.OracleError):
            oracle.decode(bad)
        with pytest.raises(P.DtansError):
            P.Matrix.load(bad)
        with pytest.raises(ValueError):
            container.decode(container.read(bad))
    # a window that is not a multiple of 64
    data = bytearray(open(path, "rb").read())
    struct.pack_into("<I", data, 112, 96)
    open(bad, "wb").write(bytes(data))
    with pytest.raises(oracle.OracleError):
        oracle.decode(bad)
    with pytest.raises(P.DtansError):
        P.Matrix.load(bad)
