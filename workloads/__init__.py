"""Seeded synthetic inputs shared by the tests, the oracle checks and the bench.

This module holds only input generation (sparsity patterns, values, dense
vectors).  It contains none of the compression method's arithmetic and imports
neither the oracle nor the product package.

The workloads stand in for the SuiteSparse matrices the paper evaluates on
(Sec. V), which are not available here.  Matrix seeds are 1000 + config and
vector seeds 2000 + config; every generator takes a size parameter so that the
tests can run the same recipe at small sizes.

  1. band: 4096 x 4096, 16 columns per row drawn without replacement from
     [i-256, i+256] (clipped), values from a pool of 64 distinct N(0,1)
     doubles, x ~ U(-1,1).
  2. stencil: 27-point stencil on a g^3 grid (g = 128: 2,097,152 rows,
     382^3 = 55,742,968 nonzeros), value = coefficient c_k ~ N(0,1) of the
     neighbour offset times a scale s ~ U(0.5, 2) of the row's octant (at most
     216 distinct doubles), x ~ U(-1,1).
  3. R-MAT: scale 22 (a,b,c,d) = (0.57,0.19,0.19,0.05), 16 * 2^22 unique
     directed edges (self loops kept), float values in {0.5, 1, 2}.
  4a. pruned weight: N(0, 0.02^2) float [11008, 4096] rounded to bfloat16
     (nearest even) and back, the 22,544,384 largest |w| kept (ties by flat
     index), CSR over rows.
  4b. batch: 64 square matrices with round(2^(10+6u)) rows, 8..64 columns per
     row within +-512 of the diagonal, a 64-value float pool per matrix.
  6. skewed rows: 2^21 x 2^21, row lengths 1 + floor(6 * Lomax(1.3)) capped
     at 512 (a heavy tail around a mean near 20), columns uniform within
     +-32768 of the diagonal, duplicates merged, values from a pool of 256
     distinct N(0,1) doubles: the irregular-but-not-power-law rows a sorted
     (SELL-C-sigma) base is meant for.
  5. graph models for the delta-entropy study: Erdős–Rényi G(n, d/(n-1)),
     Watts–Strogatz (k neighbours, rewiring 0.1), Barabási–Albert (m links
     per new node), as symmetric patterns.
"""
from __future__ import annotations

from typing import List, Tuple

import numpy as np

CSR = Tuple[np.ndarray, np.ndarray, np.ndarray]  # (row_ptr int32, col int32, val)


def _to_csr(m: int, rows: np.ndarray, cols: np.ndarray, vals: np.ndarray) -> CSR:
    """COO already sorted by (row, col) -> CSR with int32 indices."""
    counts = np.bincount(rows, minlength=m)
    row_ptr = np.zeros(m + 1, np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    return row_ptr.astype(np.int32), cols.astype(np.int32), vals


def _distinct_normal_pool(rng: np.random.Generator, k: int, dtype) -> np.ndarray:
    pool: List[float] = []
    seen = set()
    while len(pool) < k:
        v = dtype(rng.standard_normal())
        key = np.array([v], dtype=dtype).tobytes()
        if key not in seen:
            seen.add(key)
            pool.append(v)
    return np.array(pool, dtype=dtype)


def _window_rows(rng: np.random.Generator, m: int, n: int, lengths: np.ndarray, half: int,
                 chunk: int = 65536) -> Tuple[np.ndarray, np.ndarray]:
    """For row i, lengths[i] distinct columns drawn uniformly without
    replacement from [max(0, i-half), min(n-1, i+half)], sorted.

    The first L distinct values of an i.i.d. uniform sequence form a uniform
    random L-subset; rows that do not reach L distinct values within the
    drawn sequence are completed by a full shuffle of their window."""
    rows_out, cols_out = [], []
    draws = 2 * int(lengths.max(initial=0)) + 8
    for s in range(0, m, chunk):
        e = min(m, s + chunk)
        r = np.arange(s, e)
        lo = np.maximum(0, r - half)
        width = np.minimum(n - 1, r + half) - lo + 1
        L = lengths[s:e]
        seq = (rng.random((e - s, draws)) * width[:, None]).astype(np.int64)
        order = np.argsort(seq, axis=1, kind="stable")
        srt = np.take_along_axis(seq, order, axis=1)
        firstocc = np.ones_like(srt, dtype=bool)
        firstocc[:, 1:] = srt[:, 1:] != srt[:, :-1]
        isnew = np.empty_like(firstocc)
        np.put_along_axis(isnew, order, firstocc, axis=1)
        rank = np.cumsum(isnew, axis=1)
        keep = isnew & (rank <= L[:, None])
        short = rank[:, -1] < L
        if short.any():  # rare: complete these rows exactly
            for i in np.flatnonzero(short):
                perm = rng.permutation(int(width[i]))[:L[i]]
                seq[i, :] = -1
                seq[i, :L[i]] = perm
                keep[i, :] = False
                keep[i, :L[i]] = True
        picked = np.where(keep, seq + lo[:, None], np.iinfo(np.int64).max)
        picked.sort(axis=1)
        take = np.arange(draws)[None, :] < L[:, None]
        rows_out.append(np.broadcast_to(r[:, None], picked.shape)[take])
        cols_out.append(picked[take])
    return np.concatenate(rows_out), np.concatenate(cols_out)


def vector(n: int, config: int, dtype=np.float64, k: int = 0) -> np.ndarray:
    """x ~ U(-1, 1) of length n (or an [n, k] row-major block), seed 2000+config."""
    rng = np.random.default_rng(2000 + config)
    shape = (n,) if k == 0 else (n, k)
    return rng.uniform(-1.0, 1.0, size=shape).astype(dtype)


# ---------------------------------------------------------------- config 1
def band(m: int = 4096, per_row: int = 16, half: int = 256, seed: int = 1001) -> CSR:
    rng = np.random.default_rng(seed)
    pool = _distinct_normal_pool(rng, 64, np.float64)
    lengths = np.full(m, per_row, np.int64)
    width_ok = np.minimum(m - 1, np.arange(m) + half) - np.maximum(0, np.arange(m) - half) + 1
    lengths = np.minimum(lengths, width_ok)
    rows, cols = _window_rows(rng, m, m, lengths, half)
    vals = pool[rng.integers(0, 64, size=len(cols))]
    return _to_csr(m, rows, cols, vals)


# ---------------------------------------------------------------- config 2
def stencil27(g: int = 128, seed: int = 1002) -> CSR:
    """Row index z*g^2 + y*g + x; neighbour offsets in {-1,0,1}^3 in
    lexicographic (dz, dy, dx) order, which is ascending column order."""
    rng = np.random.default_rng(seed)
    coef = _distinct_normal_pool(rng, 27, np.float64)
    scale = rng.uniform(0.5, 2.0, size=8)
    m = g ** 3
    span = lambda c: 3 - (c == 0).astype(np.int64) - (c == g - 1)  # noqa: E731
    cz, cy, cx = np.meshgrid(np.arange(g), np.arange(g), np.arange(g), indexing="ij")
    counts = (span(cz) * span(cy) * span(cx)).ravel()
    row_ptr = np.zeros(m + 1, np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    nnz = int(row_ptr[-1])
    cols = np.empty(nnz, np.int32)
    vals = np.empty(nnz, np.float64)
    d = np.array([-1, 0, 1])
    off = (d[:, None, None] * g * g + d[None, :, None] * g + d[None, None, :]).ravel()
    yy, xx = np.meshgrid(np.arange(g), np.arange(g), indexing="ij")
    yy, xx = yy.ravel(), xx.ravel()
    vy = ((yy[:, None] + d) >= 0) & ((yy[:, None] + d) < g)
    vx = ((xx[:, None] + d) >= 0) & ((xx[:, None] + d) < g)
    quad = (yy >= g // 2) * 2 + (xx >= g // 2)
    plane_rows = np.arange(g * g)
    for z in range(g):  # one z-plane at a time keeps the work cache sized
        vz = ((z + d) >= 0) & ((z + d) < g)
        V = (vz[None, :, None, None] & vy[:, None, :, None] & vx[:, None, None, :]).reshape(-1, 27)
        base = z * g * g
        lo, hi = row_ptr[base], row_ptr[base + g * g]
        cols[lo:hi] = (base + plane_rows[:, None] + off[None, :])[V]
        sc = scale[(z >= g // 2) * 4 + quad]
        vals[lo:hi] = (coef[None, :] * sc[:, None])[V]
    return row_ptr.astype(np.int32), cols, vals


# ---------------------------------------------------------------- config 3
def rmat(scale: int = 22, edge_factor: int = 16, abcd=(0.57, 0.19, 0.19, 0.05),
         seed: int = 1003, batch: int = 1 << 24) -> CSR:
    rng = np.random.default_rng(seed)
    n = 1 << scale
    target = edge_factor * n
    a, b, c, _ = abcd
    t1, t2, t3 = a, a + b, a + b + c
    keys = np.empty(0, np.int64)
    batch = min(batch, max(1 << 12, 2 * target))
    while len(keys) < target:
        r = np.zeros(batch, np.int64)
        cc = np.zeros(batch, np.int64)
        for _ in range(scale):
            u = rng.random(batch)
            r = (r << 1) | (u >= t2)
            cc = (cc << 1) | (((u >= t1) & (u < t2)) | (u >= t3))
        keys = np.unique(np.concatenate([keys, (r << scale) | cc]))
    pick = np.sort(rng.choice(len(keys), size=target, replace=False))
    keys = keys[pick]
    rows, cols = keys >> scale, keys & (n - 1)
    vals = rng.choice(np.array([0.5, 1.0, 2.0], np.float32), size=target)
    return _to_csr(n, rows, cols, vals)


# ---------------------------------------------------------------- config 4a / 5
def _bf16_round(w: np.ndarray) -> np.ndarray:
    """float32 -> nearest bfloat16 (ties to even) -> float32."""
    u = w.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32)


def pruned_weight(rows: int = 11008, cols: int = 4096, keep: int = None, seed: int = 1004,
                  std: float = 0.02) -> CSR:
    import torch  # only for its seeded normal generator

    if keep is None:
        keep = rows * cols // 2
    gen = torch.Generator().manual_seed(seed)
    w = (torch.randn(rows, cols, generator=gen, dtype=torch.float32) * std).numpy().ravel()
    w = _bf16_round(w)
    mag = np.abs(w)
    # the keep largest |w|, ties broken by the smaller flat index
    thr = np.partition(mag, mag.size - keep)[mag.size - keep]
    above = mag > thr
    need = keep - int(above.sum())
    at = np.flatnonzero(mag == thr)[:need]
    mask = above
    mask[at] = True
    flat = np.flatnonzero(mask)
    r, c = flat // cols, flat % cols
    return _to_csr(rows, r, c, w[flat].astype(np.float32))


# ---------------------------------------------------------------- config 4b
def batch(count: int = 64, seed: int = 1005, lo_exp: int = 10, hi_exp: int = 16,
          min_len: int = 8, max_len: int = 64, half: int = 512) -> List[Tuple[int, CSR]]:
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        m = int(round(2.0 ** (lo_exp + (hi_exp - lo_exp) * rng.random())))
        pool = _distinct_normal_pool(rng, 64, np.float32)
        width_ok = np.minimum(m - 1, np.arange(m) + half) - np.maximum(0, np.arange(m) - half) + 1
        lengths = np.minimum(rng.integers(min_len, max_len + 1, size=m), width_ok)
        rows, cols = _window_rows(rng, m, m, lengths, half)
        vals = pool[rng.integers(0, 64, size=len(cols))]
        out.append((m, _to_csr(m, rows, cols, vals)))
    return out


# ---------------------------------------------------------------- config 6
def skewed_rows(m: int = 1 << 21, half: int = 32768, cap: int = 512, seed: int = 1006) -> CSR:
    rng = np.random.default_rng(seed)
    lengths = np.minimum(cap, 1 + np.floor(6 * rng.pareto(1.3, size=m))).astype(np.int64)
    rows = np.repeat(np.arange(m, dtype=np.int64), lengths)
    cols = np.clip(rows + rng.integers(-half, half + 1, size=len(rows)), 0, m - 1)
    key = np.unique(rows * m + cols)  # sorted by (row, col), duplicates merged
    rows, cols = key // m, key % m
    pool = _distinct_normal_pool(rng, 256, np.float64)
    return _to_csr(m, rows, cols, pool[rng.integers(0, 256, size=len(cols))])


# ---------------------------------------------------------------------------
# Random graph models for the delta-entropy study (Sec. IV-A, Fig. 4):
# undirected simple graphs as symmetric CSR patterns (sorted columns, no
# self loops), seeded.
# ---------------------------------------------------------------------------
def _sym_pattern(n: int, i: np.ndarray, j: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    a = np.concatenate([i, j]).astype(np.int64)
    b = np.concatenate([j, i]).astype(np.int64)
    keep = a != b
    key = np.unique(a[keep] * n + b[keep])
    r, c = key // n, key % n
    rp = np.zeros(n + 1, np.int64)
    np.cumsum(np.bincount(r, minlength=n), out=rp[1:])
    return rp.astype(np.int32), c.astype(np.int32)


def erdos_renyi(n: int, avg_degree: float, seed: int = 3001):
    """G(n, p) with p = avg_degree / (n - 1)."""
    rng = np.random.default_rng(seed)
    p = avg_degree / (n - 1)
    I, J = [], []
    for i in range(n - 1):
        k = rng.binomial(n - 1 - i, p)
        if k:
            J.append(rng.choice(np.arange(i + 1, n), size=k, replace=False))
            I.append(np.full(k, i))
    if not I:
        return _sym_pattern(n, np.zeros(0, np.int64), np.zeros(0, np.int64))
    return _sym_pattern(n, np.concatenate(I), np.concatenate(J))


def watts_strogatz(n: int, k: int, beta: float = 0.1, seed: int = 3002):
    """Ring lattice with k neighbours per node (k/2 on each side), each edge's
    far end rewired to a uniform node with probability beta."""
    rng = np.random.default_rng(seed)
    I, J = [], []
    for s in range(1, k // 2 + 1):
        i = np.arange(n)
        j = (i + s) % n
        j = np.where(rng.random(n) < beta, rng.integers(0, n, n), j)
        I.append(i)
        J.append(j)
    return _sym_pattern(n, np.concatenate(I), np.concatenate(J))


def barabasi_albert(n: int, m: int, seed: int = 3003):
    """Preferential attachment: every new node links to m earlier nodes drawn
    with probability proportional to their degree (m initial nodes)."""
    rng = np.random.default_rng(seed)
    targets = list(range(m))
    repeated: List[int] = []
    I, J = [], []
    for v in range(m, n):
        for t in set(targets):
            I.append(v)
            J.append(t)
        repeated.extend(targets)
        repeated.extend([v] * m)
        targets = [repeated[x] for x in rng.integers(0, len(repeated), m)]
    return _sym_pattern(n, np.array(I, np.int64), np.array(J, np.int64))
