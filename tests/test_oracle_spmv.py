"""Pins of the oracle's FP64 SpMV family (Sec. III-A) against independent
definitions: the Fig. 2 CSR example, dense products, scipy, exact rational
arithmetic and linearity."""
import json
import os
from fractions import Fraction

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import workloads


def rand_csr(m, n, density, rng, dtype=np.float64):
    A = sp.random(m, n, density=density, format="csr", random_state=rng, dtype=np.float64)
    A.sort_indices()
    return A.indptr.astype(np.int32), A.indices.astype(np.int32), A.data.astype(dtype), A


def test_fig2_csr(golden_dir):
    g = json.load(open(os.path.join(golden_dir, "csr_fig2.json")))
    D = np.array(g["dense"], dtype=np.float64)
    A = sp.csr_matrix(D)
    A.sort_indices()
    assert list(A.data) == g["values"]
    assert list(A.indices) == g["column_indices"]
    assert list(A.indptr) == g["row_start"]
    x = np.array([1.0, -2.0, 3.0, 0.5])
    y = oracle.spmv(g["row_start"], g["column_indices"], g["values"], x)
    assert np.array_equal(y, D @ x)  # small integers: exact
    assert np.array_equal(y, [-14 + 2.5, 3 + 6, -8, 0.5])


def test_spmv_matches_scipy_and_dense():
    rng = np.random.default_rng(5)
    for m, n, dens in ((1, 1, 1.0), (7, 3, 0.5), (300, 200, 0.05), (50, 1000, 0.01)):
        rp, ci, v, A = rand_csr(m, n, dens, rng)
        x = rng.uniform(-1, 1, n)
        y = oracle.spmv(rp, ci, v, x)
        assert np.allclose(y, A @ x, rtol=1e-14, atol=1e-14)
        assert np.allclose(y, A.toarray() @ x, rtol=1e-13, atol=1e-13)


def test_spmv_exact_rational():
    # integer matrix and vector: the FP64 result is exact, compare to Fractions
    rng = np.random.default_rng(6)
    m, n = 40, 30
    D = rng.integers(-5, 6, size=(m, n)) * (rng.random((m, n)) < 0.3)
    A = sp.csr_matrix(D.astype(np.float64))
    A.sort_indices()
    x = rng.integers(-7, 8, size=n)
    y = oracle.spmv(A.indptr, A.indices, A.data, x.astype(np.float64), alpha=2.0)
    for i in range(m):
        exact = 2 * sum(Fraction(int(D[i, j])) * int(x[j]) for j in range(n))
        assert Fraction(y[i]) == exact


def test_spmv_linearity_columns():
    rng = np.random.default_rng(7)
    rp, ci, v, A = rand_csr(60, 25, 0.2, rng)
    D = A.toarray()
    for j in range(25):
        e = np.zeros(25)
        e[j] = 1.0
        assert np.array_equal(oracle.spmv(rp, ci, v, e), D[:, j])


def test_alpha_beta_semantics():
    rng = np.random.default_rng(8)
    rp, ci, v, A = rand_csr(30, 20, 0.3, rng)
    x = rng.uniform(-1, 1, 20)
    y0 = rng.uniform(-1, 1, 30)
    y = oracle.spmv(rp, ci, v, x, y0, alpha=-0.5, beta=3.0)
    assert np.allclose(y, -0.5 * (A @ x) + 3.0 * y0, rtol=1e-14, atol=1e-15)
    # beta = 0 never reads y: NaN in y does not propagate
    y = oracle.spmv(rp, ci, v, x, np.full(30, np.nan), alpha=1.0, beta=0.0)
    assert np.all(np.isfinite(y))
    # empty rows give alpha*0 + beta*y
    rp2 = np.zeros(31, np.int32)
    y = oracle.spmv(rp2, np.zeros(0, np.int32), np.zeros(0), x, y0, alpha=2.0, beta=0.25)
    assert np.array_equal(y, 0.25 * y0)


def test_absmv():
    rng = np.random.default_rng(9)
    rp, ci, v, A = rand_csr(80, 60, 0.1, rng)
    x = rng.uniform(-1, 1, 60)
    assert np.allclose(oracle.absmv(rp, ci, v, x), abs(A) @ np.abs(x), rtol=1e-14, atol=0)


def test_spmtv_and_spmm():
    rng = np.random.default_rng(10)
    rp, ci, v, A = rand_csr(70, 45, 0.1, rng)
    x = rng.uniform(-1, 1, 70)
    y0 = rng.uniform(-1, 1, 45)
    y = oracle.spmtv(rp, ci, v, 45, x, y0, alpha=1.5, beta=-1.0)
    assert np.allclose(y, 1.5 * (A.T @ x) - y0, rtol=1e-13, atol=1e-14)
    X = rng.uniform(-1, 1, (45, 5))
    Y0 = rng.uniform(-1, 1, (70, 5))
    Y = oracle.spmm(rp, ci, v, X, Y0, alpha=0.5, beta=2.0)
    assert np.allclose(Y, 0.5 * (A @ X) + 2.0 * Y0, rtol=1e-13, atol=1e-14)
    # each column of SpMM is one SpMV
    for c in range(5):
        assert np.array_equal(oracle.spmm(rp, ci, v, X)[:, c], oracle.spmv(rp, ci, v, X[:, c]))


def test_workload_band_against_scipy():
    rp, ci, v = workloads.band()
    A = sp.csr_matrix((v, ci, rp), shape=(4096, 4096))
    x = workloads.vector(4096, 1)
    assert np.allclose(oracle.spmv(rp, ci, v, x), A @ x, rtol=1e-13, atol=1e-13)


def test_fp32_inputs_widen_exactly():
    rng = np.random.default_rng(11)
    rp, ci, v, A = rand_csr(40, 40, 0.2, rng, dtype=np.float32)
    x = rng.uniform(-1, 1, 40).astype(np.float32)
    y = oracle.spmv(rp, ci, v, x)
    A32 = sp.csr_matrix((v.astype(np.float64), ci, rp), shape=A.shape)
    ref = A32 @ x.astype(np.float64)
    assert np.allclose(y, ref, rtol=1e-14, atol=1e-15)


@pytest.mark.parametrize("g", [3, 6])
def test_stencil_rows_brute_force(g):
    rp, ci, v = workloads.stencil27(g)
    x = workloads.vector(g ** 3, 2)
    y = oracle.spmv(rp, ci, v, x)
    D = sp.csr_matrix((v, ci, rp), shape=(g ** 3, g ** 3)).toarray()
    assert np.allclose(y, D @ x, rtol=1e-13, atol=1e-13)
