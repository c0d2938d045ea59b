"""Delta-encoding evidence of Sec. IV-A / Fig. 4: the empirical entropy of
the column indices against that of the row-wise deltas (the oracle's delta
keys in the paper's form: a row's first delta is its column) for three
random graph models at average degrees about 5, 10 and 20, and the
tridiagonal case the paper describes (two deltas of 1 per row).  The figure's
values are not in the text, so these are its stated trends: a reduction for
every model, growing with the degree, about constant as the node count grows
for Erdős–Rényi (whose gaps are geometric: a reduction near
log2(degree / e) bits), largest for the near-lattice Watts–Strogatz graphs."""
import math

import numpy as np
import pytest

import workloads
from oracle import container


def entropy(keys) -> float:
    _, c = np.unique(np.asarray(keys, dtype=np.uint64), return_counts=True)
    p = c / c.sum()
    return float(-(p * np.log2(p)).sum())


def reduction(rp, ci):
    n = len(rp) - 1
    ranges = container.lane_ranges(1, 0, n, len(ci), rp)
    d = container.delta_keys(rp, ci, ranges, first_mode=0)
    return entropy(ci) - entropy(d), entropy(ci), entropy(d)


def test_tridiagonal_deltas():
    """Rows (i-1, i, i+1) clipped to [0, n): every row's first delta is its
    first column (0 for rows 0 and 1, then 1 .. n-2) and the others are 1,
    so the deltas take the value 0 twice, 1 (2n - 1) times and 2 .. n-2 once
    each: H(delta) follows in closed form, about a third of H(col)."""
    n = 4096
    rows = [[c for c in (i - 1, i, i + 1) if 0 <= c < n] for i in range(n)]
    rp = np.zeros(n + 1, np.int64)
    rp[1:] = np.cumsum([len(r) for r in rows])
    ci = np.array([c for r in rows for c in r], np.int32)
    ranges = container.lane_ranges(1, 0, n, len(ci), rp)
    d = np.array(container.delta_keys(rp, ci, ranges, first_mode=0), np.int64)
    total = 3 * n - 2
    counts = [2, 2 * n - 1] + [1] * (n - 3)
    assert len(d) == total == sum(counts)
    h = -sum(c / total * math.log2(c / total) for c in counts)
    assert abs(entropy(d) - h) < 1e-12
    assert entropy(d) < 0.45 * entropy(ci)


@pytest.mark.parametrize("model", ["er", "ws", "ba"])
def test_random_graph_models(model):
    gens = {
        "er": [lambda n, s, d=d: workloads.erdos_renyi(n, d, seed=3001 + s) for d in (5, 10, 20)],
        "ws": [lambda n, s, k=k: workloads.watts_strogatz(n, k, seed=3002 + s) for k in (4, 10, 20)],
        "ba": [lambda n, s, m=m: workloads.barabasi_albert(n, m, seed=3003 + s) for m in (3, 5, 10)],
    }[model]
    red = {}
    for n in (1024, 4096):
        for g, gen in enumerate(gens):
            rp, ci = gen(n, g)
            deg = len(ci) / n
            r, hc, hd = reduction(rp, ci)
            red[n, g] = r
            assert r > 0.5, (model, n, deg, hc, hd)
            if model == "er":
                # geometric gaps: about log2(deg / e) bits, plus the first
                # deltas' share
                assert abs(r - math.log2(deg / math.e)) < 0.45, (n, deg, r)
    for n in (1024, 4096):
        assert red[n, 0] < red[n, 1] < red[n, 2], (model, n, red)
    if model == "er":
        for g in range(3):
            assert abs(red[1024, g] - red[4096, g]) < 0.15, red
    if model == "ws":
        assert min(red.values()) > 4.0, red
