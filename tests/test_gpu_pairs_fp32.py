"""GPU parity of the FP32 SpMV's per-lane paired x loads: an 8-byte load
ending at column k+1 serves nonzero k too where the two columns are adjacent.
These matrices mix adjacent and separate columns, repeat columns (allowed in
the input), use the first and last column, and leave the columns no row uses
non-finite in x (a pair load may read one of them; its value must never reach
y).  Both layouts, y against the oracle within the FP32 tolerance."""
import numpy as np
import pytest

from gpu_common import check_spmv, need_gpu, progress

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2603_01915_amd")


def paired_rows(seed, m, n, lo, hi, dup=0.1, edge=0.2):
    """Rows of lo..hi nonzeros: half of the columns of a random window kept
    (so about half the column pairs are adjacent), some repeated, column 0 and
    n-1 in about `edge` of the rows; columns 3, 7, 11, ... are never used."""
    rng = np.random.default_rng(seed)
    allowed = np.array([c for c in range(n) if c % 4 != 3 or c in (0, n - 1)])
    rows = []
    for _ in range(m):
        want = int(rng.integers(lo, hi + 1))
        if len(allowed) <= 2 * want:
            c = np.sort(rng.choice(allowed, size=min(want, len(allowed)), replace=False))
        else:
            s = int(rng.integers(0, len(allowed) - 2 * want))
            window = allowed[s:s + 2 * want]
            c = np.sort(rng.choice(window, size=want, replace=False))
        extra = [0] if rng.random() < edge else []
        extra += [n - 1] if rng.random() < edge else []
        reps = c[rng.random(len(c)) < dup]
        rows.append(np.sort(np.concatenate([c, np.array(extra, np.int64), reps]).astype(np.int64)))
    rp = np.zeros(m + 1, np.int64)
    rp[1:] = np.cumsum([len(c) for c in rows])
    ci = np.concatenate(rows)
    v = rng.standard_normal(len(ci)).astype(np.float32)
    return rp.astype(np.int32), ci.astype(np.int32), v


CASES = [  # name, n, m, shortest and longest row
    ("n1", 1, 300, 0, 3),
    ("n2", 2, 300, 0, 6),
    ("n5", 5, 500, 0, 12),
    ("wide", 4096, 700, 100, 400),
    ("mixed", 2000, 3000, 0, 60),
]


@pytest.mark.parametrize("layout", ["row", "nnz"])
@pytest.mark.parametrize("case", range(len(CASES)), ids=[c[0] for c in CASES])
def test_fp32_pairs_spmv(case, layout):
    torch = need_gpu()
    name, n, m, lo, hi = CASES[case]
    rp, ci, v = paired_rows(300 + case, m, n, lo, hi)
    progress("fp32 pairs %s %s: m=%d n=%d nnz=%d" % (name, layout, m, n, len(ci)))
    A = P.Matrix.from_csr(rp, ci, v, n, layout=layout)
    x = np.random.default_rng(7).standard_normal(n).astype(np.float32)
    if n > 4:
        x[3:n - 1:4] = np.nan  # columns no row uses
    xd = torch.from_numpy(x).cuda()
    y = A.spmv(xd).cpu().numpy()
    assert np.all(np.isfinite(y))
    check_spmv(y, rp, ci, v, x, None, 1.0, 0.0, np.float32)
    y0 = np.random.default_rng(8).standard_normal(m).astype(np.float32)
    yd = torch.from_numpy(y0.copy()).cuda()
    A.spmv(xd, yd, alpha=-0.5, beta=2.0)
    check_spmv(yd.cpu().numpy(), rp, ci, v, x, y0, -0.5, 2.0, np.float32)
