"""Pins of the oracle's reference CSR-dtANS codec.

* round trips are bit-exact on random and adversarial matrices (the method is
  lossless, Sec. I/IV);
* the C oracle and the Python big-integer container codec (whose per-lane
  arithmetic is pinned to the paper's worked examples) decode each other's
  containers and produce byte-identical containers from the same tables;
* closed forms for the number of stream words of a lane (Sec. IV-D/F);
* decoder state invariants (Sec. IV-D) and the base pass agreeing with the
  decoder's branches (Sec. IV-E);
* corrupted containers are rejected.
"""
import os
import random
import struct

import numpy as np
import pytest
import scipy.sparse as sp
from hypothesis import given, settings, strategies as st

import oracle
from oracle import container, toy


def csr_from_rows(n, rows, dtype=np.float64, vals=None, rng=None):
    rp = np.zeros(len(rows) + 1, np.int64)
    rp[1:] = np.cumsum([len(r) for r in rows])
    ci = np.array([c for r in rows for c in r], np.int64)
    if vals is None:
        rng = rng or np.random.default_rng(0)
        vals = rng.choice(np.array([0.5, -1.0, 2.0, 3.0]), size=len(ci))
    return rp.astype(np.int32), ci.astype(np.int32), np.asarray(vals, dtype)


def roundtrip(tmp_path, m, n, rp, ci, v, layout, T, name="a.dtans"):
    p = str(tmp_path / name)
    oracle.encode(p, m, n, rp, ci, v, layout=layout, lane_nnz=T)
    r2, c2, v2 = oracle.decode(p)
    assert np.array_equal(r2, rp)
    assert np.array_equal(c2, ci)
    assert v2.dtype == v.dtype and np.array_equal(v2.view(np.uint8), v.view(np.uint8))
    return p


LAYOUTS = [(1, 0), (2, 4), (2, 8), (2, 64)]


@pytest.mark.parametrize("layout,T", LAYOUTS)
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_roundtrip_random(tmp_path, layout, T, dtype):
    rng = np.random.default_rng(1)
    A = sp.random(400, 300, density=0.03, format="csr", random_state=rng)
    A.sort_indices()
    v = rng.choice(rng.standard_normal(40), size=A.nnz).astype(dtype)
    roundtrip(tmp_path, 400, 300, A.indptr, A.indices, v, layout, T)


@pytest.mark.parametrize("layout,T", LAYOUTS)
def test_roundtrip_adversarial(tmp_path, layout, T):
    rng = np.random.default_rng(2)
    n = 5000
    rows = [[], [7], [1, 2], [0, 0, 3], [], list(range(0, 5000, 2)), [4999], [],
            [5, 5, 5, 5, 5], list(range(100, 113))]
    rows += [sorted(rng.choice(n, size=rng.integers(0, 9), replace=False)) for _ in range(150)]
    rp, ci, _ = csr_from_rows(n, rows)
    # values: special bit patterns and many distinct values (escapes)
    v = rng.standard_normal(len(ci))
    specials = [0.0, -0.0, np.inf, -np.inf, np.nan, 5e-324, -2.2250738585072014e-308, 1.0]
    v[:len(specials)] = specials
    v = v.copy()
    bits = v.view(np.uint64)
    bits[3] = 0x7FF8DEADBEEF0001  # NaN with a payload
    roundtrip(tmp_path, len(rows), n, rp, ci, v, layout, T)
    v32 = v.astype(np.float32)
    v32.view(np.uint32)[4] = 0x7FC0ABCD
    roundtrip(tmp_path, len(rows), n, rp, ci, v32, layout, T, "b.dtans")


@pytest.mark.parametrize("layout,T", LAYOUTS)
def test_roundtrip_huge_columns(tmp_path, layout, T):
    # deltas at and above 2^30 must be escaped; columns near 2^31
    n = 2 ** 31 - 1
    rows = [[0, 2 ** 30, 2 ** 31 - 2], [2 ** 31 - 2], [5, 6, 2 ** 30 + 7], [], [1, 2, 3, 4, 5]]
    rp, ci, v = csr_from_rows(n, rows)
    p = roundtrip(tmp_path, len(rows), n, rp, ci, v, layout, T)
    assert oracle.read_header(p)["n_esc_delta"] >= 3


def test_roundtrip_all_values_escaped(tmp_path):
    rng = np.random.default_rng(3)
    m, per = 300, 10
    rows = [sorted(rng.choice(1000, size=per, replace=False)) for _ in range(m)]
    rp, ci, _ = csr_from_rows(1000, rows)
    v = rng.standard_normal(len(ci))  # 3000 distinct values > table room
    p = roundtrip(tmp_path, m, 1000, rp, ci, v, 1, 0)
    assert oracle.read_header(p)["n_esc_value"] > 0


@pytest.mark.parametrize("layout,T", LAYOUTS)
def test_empty_matrices(tmp_path, layout, T):
    rp = np.zeros(11, np.int32)
    roundtrip(tmp_path, 10, 10, rp, np.zeros(0, np.int32), np.zeros(0), layout, T)
    rp = np.zeros(1, np.int32)
    roundtrip(tmp_path, 0, 10, rp, np.zeros(0, np.int32), np.zeros(0), layout, T, "b.dtans")


@settings(max_examples=40, deadline=None)
@given(seed=st.integers(0, 2 ** 31), m=st.integers(0, 70), n=st.integers(1, 90),
       dens=st.floats(0.0, 0.6), layout=st.sampled_from(LAYOUTS),
       f64=st.booleans(), pool=st.integers(1, 300))
def test_roundtrip_property(tmp_path_factory, seed, m, n, dens, layout, f64, pool):
    rng = np.random.default_rng(seed)
    A = sp.random(m, n, density=dens, format="csr", random_state=rng)
    A.sort_indices()
    dtype = np.float64 if f64 else np.float32
    v = rng.choice(rng.standard_normal(pool), size=A.nnz).astype(dtype)
    tmp = tmp_path_factory.mktemp("prop")
    roundtrip(tmp, m, n, A.indptr, A.indices, v, layout[0], layout[1])


# ------------------------------------------------ cross-implementation checks
def small_matrix(seed, m=130, n=90, dens=0.08, dtype=np.float64, unique_every=0, big_cols=False):
    rng = np.random.default_rng(seed)
    A = sp.random(m, n, density=dens, format="csr", random_state=rng)
    A.sort_indices()
    ci = A.indices.astype(np.int64)
    if big_cols:
        ci = ci * 20_000_000
    v = rng.choice(np.array([0.5, 1.0, 2.0, -3.25, 7.0]), size=A.nnz).astype(dtype)
    if unique_every:
        v[::unique_every] = rng.standard_normal(len(v[::unique_every]))
    return A.indptr.astype(np.int32), ci.astype(np.int32), v, (2 ** 31 - 1 if big_cols else n)


@pytest.mark.parametrize("layout,T", [(1, 0), (2, 8), (2, 12)])
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("case", [0, 1, 2])
def test_cross_decode_and_identical_bytes(tmp_path, layout, T, dtype, case):
    rp, ci, v, n = small_matrix(10 + case, dtype=dtype, unique_every=3 if case == 1 else 0,
                                big_cols=case == 2)
    m = len(rp) - 1
    dt = 2 if dtype == np.float64 else 1
    p1 = str(tmp_path / "c.dtans")
    oracle.encode(p1, m, n, rp, ci, v, layout=layout, lane_nnz=T, seed=77)
    # C container -> Python reader + big-integer lockstep decoder
    c = container.read(p1)
    _, c3, v3 = container.decode(c)
    assert np.array_equal(c3, ci) and np.array_equal(v3.view(np.uint8), v.view(np.uint8))
    # same tables -> the Python encoder writes the same bytes
    c6 = container.encode(m, n, rp, ci, v, dt, layout, T, tables=(c.dtab, c.vtab), seed=c.seed)
    p2 = str(tmp_path / "p.dtans")
    container.write(p2, c6)
    assert open(p1, "rb").read() == open(p2, "rb").read()
    # Python container with its own tables -> C decoder
    c4 = container.encode(m, n, rp, ci, v, dt, layout, T, seed=5)
    container.write(p2, c4)
    _, c5, v5 = oracle.decode(p2)
    assert np.array_equal(c5, ci) and np.array_equal(v5.view(np.uint8), v.view(np.uint8))


# ------------------------------------------------------------- closed forms
def pad_tables(t):
    k = container.K - len(t.symbol)
    return toy.Tables(t.symbol + [None] * k, t.digit + [0] * k, t.base + [0] * k)


@pytest.mark.parametrize("b,formula", [(256, lambda S: S + 2), (1, lambda S: 3 * S),
                                       (16, lambda S: 2 * S + 1)])
@pytest.mark.parametrize("S", [1, 2, 3, 7, 20])
def test_word_count_closed_forms(tmp_path, b, formula, S):
    p = toy.CSR_DTANS
    tab = pad_tables(toy.Tables.from_multiplicities([("x", b)]))
    u = ["x"] * (p.l * S)
    assert toy.dtans_word_count(u, tab, p) == formula(S)
    words = toy.dtans_encode(u, tab, p)
    assert len(words) == formula(S)
    out, used = toy.dtans_decode(words, tab, len(u), p)
    assert out == u and used == len(words)
    # the same through containers and the C decoder: 3 rows of 4S nonzeros
    # with every delta 1 and every value 1.0
    dt = pad_tables(toy.Tables.from_multiplicities([(1, b)]))
    vt = pad_tables(toy.Tables.from_multiplicities([(0x3FF0000000000000, b)]))
    rows = [list(range(1, 4 * S + 1))] * 3
    rp, ci, v = csr_from_rows(4 * S + 1, rows, vals=np.ones(12 * S))
    c = container.encode(3, 4 * S + 1, rp, ci, v, 2, 1, 0, tables=(dt, vt))
    assert len(c.words) == 3 * formula(S)
    path = str(tmp_path / "cf.dtans")
    container.write(path, c)
    _, c2, v2 = oracle.decode(path)
    assert np.array_equal(c2, ci) and np.array_equal(v2, v)
    if b == 256:
        # the C encoder's own fit gives one symbol per alphabet -> base 256
        oracle.encode(path, 3, 4 * S + 1, rp, ci, v)
        assert oracle.read_header(path)["n_words"] == 3 * formula(S)


def test_word_count_bounds_random():
    # S + 2 <= words <= 3S for any lane (Sec. IV-D: at most o words per
    # segment, at least the o - f unconditional ones)
    rng = random.Random(4)
    p = toy.CSR_DTANS
    tab = pad_tables(toy.Tables.from_multiplicities([(s, rng.randint(1, 256)) for s in range(12)]))
    for _ in range(30):
        S = rng.randint(1, 12)
        u = [rng.randrange(12) for _ in range(p.l * S)]
        w = toy.dtans_encode(u, tab, p)
        assert S + 2 <= len(w) <= 3 * S
        out, used = toy.dtans_decode(w, tab, len(u), p)
        assert out == u and used == len(w)


def test_state_invariants_real_parameters():
    rng = random.Random(5)
    p = toy.CSR_DTANS
    tab = pad_tables(toy.Tables.from_multiplicities([(s, rng.randint(1, 256)) for s in range(15)]))
    for _ in range(20):
        S = rng.randint(2, 10)
        u = [rng.randrange(15) for _ in range(p.l * S)]
        w = toy.dtans_encode(u, tab, p)
        trace = []
        out, _ = toy.dtans_decode(w, tab, len(u), p, trace=trace)
        assert out == u
        flags = toy.dtans_base_pass(u, tab, p)
        assert [t["kind"] == "extract" for t in trace] == [x for fj in flags for x in fj]
        for t in trace:
            d0, r0 = t["before"]
            d1, r1 = t["after"]
            assert 0 <= d0 < r0 < 2 ** 64  # a digit group fits in 64 bits
            assert 0 <= d1 < r1 < 2 ** 32  # after a check the state is one word


# ------------------------------------------------------------- corruption
def test_corruption_detected(tmp_path):
    rp, ci, v, n = small_matrix(20)
    m = len(rp) - 1
    p = str(tmp_path / "x.dtans")
    oracle.encode(p, m, n, rp, ci, v)
    data = bytearray(open(p, "rb").read())
    # a flipped bit anywhere after the header fails the checksum
    for off in (300, len(data) // 2, len(data) - 3):
        bad = bytearray(data)
        bad[off] ^= 0x10
        open(p, "wb").write(bad)
        with pytest.raises(oracle.OracleError):
            oracle.decode(p)
    # truncation
    open(p, "wb").write(data[:-8])
    with pytest.raises(oracle.OracleError):
        oracle.decode(p)
    # a wave that stores one word too few or too many (checksum recomputed)
    open(p, "wb").write(data)
    c = container.read(p)
    for delta in (-1, +1):
        c2 = container.read(p)
        end0 = int(c2.word_off[1])
        if delta < 0:
            c2.words = np.delete(c2.words, end0 - 1)
        else:
            c2.words = np.insert(c2.words, end0, np.uint32(12345))
        c2.word_off = c2.word_off.astype(np.int64)
        c2.word_off[1:] += delta
        c2.word_off = c2.word_off.astype(np.uint64)
        container.write(p, c2)
        with pytest.raises(oracle.OracleError):
            oracle.decode(p)
    assert c.num_waves >= 2
