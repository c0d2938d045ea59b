"""GPU parity of the FP64 row-layout SpMV on the segments that are not full
(a row's last one to three nonzeros, lanes whose row has ended): x is read in
16-byte pairs there too, a lane holding only the first nonzero of a pair
reading the pair that ends at its column, so these cases put nonzeros at the
first and last column, in runs of adjacent columns and alone, with rows of
every length from 0 to 40 mixed in one wave.  y against the oracle, and bit
for bit against the general tables (no paired loads there, same products in
the same order)."""
import numpy as np
import pytest

import workloads
from gpu_common import check_spmv, need_gpu, progress

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2603_01915_amd")


def short_rows(seed, m, n, maxlen, edge=0.25, minlen=0):
    """Rows of minlen..maxlen nonzeros built from runs of 1-4 adjacent columns,
    with column 0 and column n-1 each in about `edge` of the rows; values
    from 16 distinct ones (direct tables)."""
    rng = np.random.default_rng(seed)
    pool = rng.standard_normal(16)
    rows = []
    for _ in range(m):
        want = int(rng.integers(minlen, maxlen + 1))
        cols = set()
        if rng.random() < edge:
            cols.add(0)
        if rng.random() < edge:
            cols.add(n - 1)
        while len(cols) < min(want, n):
            s = int(rng.integers(0, n))
            cols.update(range(s, min(n, s + int(rng.integers(1, 5)))))
        c = np.array(sorted(cols), np.int64)
        if len(c) > want:  # keep the edge columns when trimming
            keep = [x for x in c if x in (0, n - 1)]
            rest = [x for x in c if x not in (0, n - 1)]
            c = np.array(sorted(keep[:want] + rest[:max(0, want - len(keep))]), np.int64)
        rows.append(c)
    rp = np.zeros(m + 1, np.int64)
    rp[1:] = np.cumsum([len(c) for c in rows])
    ci = np.concatenate(rows) if rp[-1] else np.zeros(0, np.int64)
    v = pool[rng.integers(0, 16, size=len(ci))]
    return rp.astype(np.int32), ci.astype(np.int32), v


CASES = [  # name, n, m, shortest and longest row, share of rows at the edges
    ("n1", 1, 70, 0, 1, 0.5),
    ("n2", 2, 130, 0, 2, 0.5),
    ("n3", 3, 200, 0, 3, 0.5),
    ("short", 500, 64 * 6 + 17, 0, 7, 0.25),
    ("mixed", 3000, 64 * 20 + 5, 0, 40, 0.25),
    ("long", 4000, 64 * 12, 29, 40, 0.1),  # full steps first, then short ones
]


@pytest.mark.parametrize("case", range(len(CASES)), ids=[c[0] for c in CASES])
def test_short_segments_spmv(case):
    torch = need_gpu()
    name, n, m, minlen, maxlen, edge = CASES[case]
    rp, ci, v = short_rows(100 + case, m, n, maxlen, edge, minlen)
    progress("short segments %s: m=%d n=%d nnz=%d" % (name, m, n, len(ci)))
    A = P.Matrix.from_csr(rp, ci, v, n, layout="row")
    assert A.info()["direct_table"] == 1
    G = P.Matrix.from_csr(rp, ci, v, n, layout="row", max_mult=256)
    x = workloads.vector(n, 5, np.float64)
    xd = torch.from_numpy(x).cuda()
    y = A.spmv(xd)
    assert torch.equal(y, G.spmv(xd))
    check_spmv(y.cpu().numpy(), rp, ci, v, x, None, 1.0, 0.0, np.float64)
    y0 = workloads.vector(m, 6, np.float64)
    yd = torch.from_numpy(y0.copy()).cuda()
    A.spmv(xd, yd, alpha=1.25, beta=-0.5)
    check_spmv(yd.cpu().numpy(), rp, ci, v, x, y0, 1.25, -0.5, np.float64)


def test_short_segments_unread_nonfinite_x():
    """Lanes without a nonzero read columns 0 and 1 (and a lane holding only
    the first nonzero of a pair reads its left neighbour): infinite and NaN
    values there must not reach y when no row uses those columns."""
    torch = need_gpu()
    n, m = 300, 64 * 4 + 9
    rp, ci, v = short_rows(7, m, n, 9, edge=0.0)
    keep = ci >= 3  # no row uses columns 0-2
    rows = np.repeat(np.arange(m), np.diff(rp))[keep]
    ci, v = ci[keep], v[keep]
    rp = np.concatenate([[0], np.cumsum(np.bincount(rows, minlength=m))]).astype(np.int32)
    progress("short segments, non-finite unread x")
    A = P.Matrix.from_csr(rp, ci, v, n, layout="row")
    assert A.info()["direct_table"] == 1
    x = workloads.vector(n, 8, np.float64)
    x[0], x[1], x[2] = np.inf, np.nan, -np.inf
    y = A.spmv(torch.from_numpy(x).cuda()).cpu().numpy()
    assert np.all(np.isfinite(y))
    check_spmv(y, rp, ci, v, x, None, 1.0, 0.0, np.float64)
