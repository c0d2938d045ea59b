"""Autotuner on the GPU: the options it returns encode a matrix whose product
matches the oracle, fixed options are respected, the budget bounds the search
and the cache file short-cuts a repeated search."""
import time

import numpy as np
import pytest

import oracle
import workloads
from gpu_common import TOL, need_gpu, progress, rel_error

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2603_01915_amd")


def _check(opts, rp, ci, v, n, torch, k=1):
    A = P.Matrix.from_csr(rp, ci, v, n, **opts)
    info = A.info()
    assert info["layout"] == opts["layout"]
    if opts["layout"] == P.LAYOUT_NNZ:
        assert info["lane_nnz"] == opts["lane_nnz"]
    assert info["waves_per_wg"] == opts["waves_per_wg"]
    x = workloads.vector(n, 9, v.dtype, k=0 if k == 1 else k)
    X = torch.from_numpy(x).cuda()
    Y = (A.spmv(X) if k == 1 else A.spmm(X)).cpu().numpy().reshape(len(rp) - 1, k)
    x2 = x.reshape(n, k)
    for c in range(k):
        ref = oracle.spmv(rp, ci, v, x2[:, c])
        assert rel_error(Y[:, c], ref, oracle.absmv(rp, ci, v, x2[:, c])) <= TOL[v.dtype.type]


def test_autotune_band_and_cache(tmp_path):
    torch = need_gpu()
    rp, ci, v = workloads.band(200_000, 8, 32, seed=3)
    cache = str(tmp_path / "tune.txt")
    progress("autotune band 200000 rows, budget 6 s")
    t0 = time.time()
    opts, ms = P.autotune(rp, ci, v, 200_000, budget_s=6.0, cache=cache)
    assert ms > 0 and np.isfinite(ms)
    assert time.time() - t0 < 60
    cands = P.autotune_candidates(rp, len(ci), v.dtype)
    assert opts in cands
    _check(opts, rp, ci, v, 200_000, torch)
    lines = open(cache).read().splitlines()
    assert len(lines) == 1 and lines[0].startswith("dtans-autotune-v2 ")
    # a repeated search is answered from the cache
    t0 = time.time()
    opts2, ms2 = P.autotune(rp, ci, v, 200_000, budget_s=6.0, cache=cache)
    assert (opts2, round(ms2, 6)) == (opts, round(ms, 6))
    assert time.time() - t0 < 5
    assert len(open(cache).read().splitlines()) == 1
    # another k or another matrix is a new entry
    P.autotune(rp, ci, v, 200_000, k=4, budget_s=2.0, cache=cache)
    assert len(open(cache).read().splitlines()) == 2


def test_autotune_fixed_fields_and_budget():
    torch = need_gpu()
    rp, ci, v = workloads.pruned_weight(rows=2048, cols=1024, keep=400_000)
    progress("autotune pruned 2048x1024, fixed layout and workgroups")
    opts, ms = P.autotune(rp, ci, v, 1024, k=8, budget_s=4.0, layout="nnz", wg_per_cu=1)
    assert opts["layout"] == P.LAYOUT_NNZ and opts["wg_per_cu"] == 1 and ms > 0
    _check(opts, rp, ci, v, 1024, torch, k=8)
    # budget 0: only the first (automatic) encoding is timed
    progress("autotune with budget 0")
    opts, ms = P.autotune(rp, ci, v, 1024, budget_s=0.0)
    first = P.autotune_candidates(rp, len(ci), v.dtype)[0]
    assert (opts["layout"], opts["lane_nnz"]) == (first["layout"], first["lane_nnz"])
    _check(opts, rp, ci, v, 1024, torch)
