"""Compressed size: the library's alphabet fit against the exact optimum.

Sec. IV-F chooses table symbols and multiplicities so that the expected total
size is smallest.  ``oracle.fit.exact_fit`` computes that minimum by dynamic
programming; it is pinned here by exhaustive enumeration on tiny tables, by
closed forms, and then used to check the tables the library writes (read
back from its container by the oracle's own reader) at K = 4096.
"""
import collections
import math

import numpy as np
import pytest

from oracle import container
from oracle import fit

P = pytest.importorskip("paper_2603_01915_amd")


# ------------------------------------------------------------- pins of the oracle
@pytest.mark.parametrize("seed", range(40))
def test_exact_fit_matches_enumeration(seed):
    """The dynamic programme reaches the minimum found by enumerating every
    kept subset and every multiplicity vector (K = 16, cap 3..6)."""
    rng = np.random.default_rng(seed)
    q = int(rng.integers(1, 5))
    K = 16
    cap = int(rng.integers(3, 7))
    raw = int(rng.choice([4, 5, 8]))  # >= log2(K): escaping never beats a slot by itself
    is_delta = bool(rng.integers(0, 2))
    hist = {int(k): int(rng.integers(1, 60)) for k in rng.choice(1000, q, replace=False)}
    if is_delta and rng.integers(0, 2):
        hist[fit.DELTA_LIMIT + 5] = int(rng.integers(1, 30))  # must escape
    best, _ = fit.exact_fit(hist, raw, is_delta, K=K, cap=cap)
    bf = fit.brute_force(hist, raw, is_delta, K=K, cap=cap)
    assert best == pytest.approx(bf, rel=1e-12, abs=1e-12)


def test_exact_fit_closed_forms():
    # two equally frequent symbols share the 4096 slots equally (cap 2048
    # admitted): each costs log2(4096 / 2048) = 1 bit
    bits, t = fit.exact_fit({1: 100, 2: 100}, 32, K=4096, cap=2048)
    assert t == 2 and bits == pytest.approx(200.0)
    # fewer than K / M symbols: every one sits at the cap, 12 - 8 = 4 bits
    bits, t = fit.exact_fit({1: 7, 2: 3, 3: 11}, 64, K=4096, cap=256)
    assert t == 3 and bits == pytest.approx(4.0 * 21)
    # a single symbol at cap 255
    bits, _ = fit.exact_fit({9: 10}, 32, K=4096, cap=255)
    assert bits == pytest.approx(10 * math.log2(4096 / 255))
    # more distinct symbols than slots, all equally rare: t of them keep one
    # slot each (12 bits) and the escape symbol takes the other slots up to
    # the cap, so the size is min over t of 12 t + (5000 - t)(log2(K / m_E) + 32)
    hist = {k: 1 for k in range(5000)}
    bits, t = fit.exact_fit(hist, 32, K=4096, cap=255)
    f = {u: 12.0 * u + (5000 - u) * (math.log2(4096 / min(255, 4096 - u)) + 32) for u in range(1, 4096)}
    u_best = min(f, key=lambda u: (f[u], u))
    assert t == u_best and bits == pytest.approx(f[u_best])
    # column deltas at or above 2^30 are always escaped
    bits, t = fit.exact_fit({1: 50, (1 << 30) + 1: 2}, 32, is_delta=True, K=4096, cap=255)
    assert t == 1
    assert bits == pytest.approx(50 * math.log2(4096 / 255) + 2 * (math.log2(4096 / 255) + 32))


def test_exact_fit_detects_a_worse_table():
    """A table one slot away from the optimum scores strictly higher."""
    hist = {1: 1000, 2: 10, 3: 10}
    bits, _ = fit.exact_fit(hist, 32, K=16, cap=16)
    worse = fit.size_of([1000, 10, 10], [13, 2, 1], 0, 1, 32, K=16)
    assert worse > bits + 1.0


# ----------------------------------------------------- the library's tables
def _tables(path):
    c = container.read(path)
    out = []
    for t in (c.dtab, c.vtab):
        base_of, esc = {}, None
        for s, b in zip(t.symbol, t.base):
            if s is None:
                continue
            if s == container.ESC:
                esc = b
            else:
                base_of[s] = b
        out.append((base_of, esc))
    return c, out


def _matrix(rng, m, per_row, value_pool_counts, gap_pool):
    """CSR with rows of `per_row` nonzeros whose column gaps are drawn from
    `gap_pool` and whose values follow the multiset `value_pool_counts`
    (value -> count, shuffled over the nonzeros)."""
    vals = np.concatenate([np.full(c, v) for v, c in value_pool_counts.items()])
    nnz = m * per_row
    assert len(vals) >= nnz
    vals = rng.permutation(vals)[:nnz]
    cols = []
    for i in range(m):
        g = rng.choice(gap_pool, per_row)
        g[0] = rng.integers(0, 50)
        cols.append(np.cumsum(g))
    ci = np.concatenate(cols).astype(np.int32)
    n = int(ci.max()) + 1
    rp = np.arange(0, nnz + 1, per_row, dtype=np.int32)
    return rp, ci, vals, n


CASES = {
    # few symbols: fewer than K / M, so every symbol sits at the cap
    "three_values": (lambda rng: {1.5: 9000, -2.0: 5000, 0.25: 1000}),
    # geometric counts over 24 symbols
    "geometric": (lambda rng: {float(v): int(20000 * 0.7 ** i) + 1
                               for i, v in enumerate(rng.standard_normal(24))}),
    # Zipf head and a tail of rare values
    "zipf_tail": (lambda rng: {**{float(v): int(6000 / (i + 1)) + 1
                                  for i, v in enumerate(rng.standard_normal(30))},
                               **{float(v): 1 for v in rng.standard_normal(60) + 100.0}}),
}


@pytest.mark.parametrize("case", sorted(CASES))
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("max_mult", [0, 256])
def test_library_fit_reaches_optimum(tmp_path, case, dtype, max_mult):
    """Both alphabets of the library's container cost exactly the optimum of
    the expected total size (up to rounding of the sums)."""
    rng = np.random.default_rng(10 + sorted(CASES).index(case))
    pool = {dtype(v): c for v, c in CASES[case](rng).items()}
    per_row = 16
    m = min(sum(pool.values()) // per_row, 900)
    rp, ci, v, n = _matrix(rng, m, per_row, pool, np.array([1, 1, 1, 2, 2, 3, 5, 8, 40, 300]))
    A = P.Matrix.from_csr(rp, ci, v.astype(dtype), n, layout="row", max_mult=max_mult)
    path = str(tmp_path / "a.dtans")
    A.save(path)
    c, ((dbase, desc), (vbase, vesc)) = _tables(path)
    cap = 255 if max_mult == 0 else max_mult
    ranges = container.lane_ranges(1, 0, m, len(ci), rp)
    dh = collections.Counter(container.delta_keys(rp, ci, ranges, c.first_mode))
    vh = collections.Counter(container.value_keys(v.astype(dtype), 2 if dtype == np.float64 else 1))
    raw_v = 64 if dtype == np.float64 else 32
    for hist, base_of, esc, raw, is_delta in ((dh, dbase, desc, 32, True), (vh, vbase, vesc, raw_v, False)):
        got = fit.table_size(hist, base_of.keys(), base_of, esc, raw, is_delta)
        best, _ = fit.exact_fit(hist, raw, is_delta, cap=cap)
        assert got <= best * (1 + 1e-12) + 1e-9, (case, is_delta, got, best)


def test_library_fit_more_symbols_than_slots(tmp_path):
    """More distinct values than table slots: the library escapes exactly
    the rarest ones and reaches the optimum."""
    rng = np.random.default_rng(5)
    distinct = rng.permutation(np.arange(1, 6001, dtype=np.float32) * np.float32(0.5))
    counts = {float(x): (30 if i < 40 else 1) for i, x in enumerate(distinct)}
    pool = {np.float32(k): c for k, c in counts.items()}
    per_row = 8
    m = sum(pool.values()) // per_row
    rp, ci, v, n = _matrix(rng, m, per_row, pool, np.array([1, 2, 3]))
    A = P.Matrix.from_csr(rp, ci, v.astype(np.float32), n, layout="row")
    path = str(tmp_path / "a.dtans")
    A.save(path)
    _, (_, (vbase, vesc)) = _tables(path)
    vh = collections.Counter(container.value_keys(v.astype(np.float32), 1))
    assert vesc is not None and len(vbase) <= 4095
    got = fit.table_size(vh, vbase.keys(), vbase, vesc, 32)
    best, _ = fit.exact_fit(vh, 32, cap=255)
    assert got <= best * (1 + 1e-12) + 1e-9, (got, best)
