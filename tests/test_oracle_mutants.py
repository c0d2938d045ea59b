"""The oracle's pins catch plausible mistakes: each case plants one mistake in
a copy of the C oracle (a dropped term, a transposed operand, a wrong index
or sign, a changed digit or bit order, a reversed sort), builds it on the CPU
and checks that the pin covering that part fails.  The oracle itself is not
changed; the copies live in a temporary directory.
"""
import ctypes
import os
import subprocess

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from oracle import container

SRC = os.path.join(os.path.dirname(oracle.__file__), "dtans_oracle.c")

MUTANTS = {
    # SpMV without the beta term (a dropped term)
    "spmv_beta": ("y[i] = (beta == 0.0) ? alpha * s : alpha * s + beta * y[i];", "y[i] = alpha * s;"),
    # SpMV multiplying by x at the row instead of the column (transposed operand)
    "spmv_index": ("s += val[p] * x[col[p]];", "s += val[p] * x[i];"),
    # A^T x accumulating x at the column (wrong index)
    "spmtv_index": ("acc[col[p]] += val[p] * x[i];", "acc[col[p]] += val[p] * x[col[p] % m];"),
    # SpMM reading X transposed
    "spmm_stride": ("s += val[p] * X[(int64_t)col[p] * ldx + c];", "s += val[p] * X[(int64_t)c * ldx + col[p] % ldx];"),
    # the encoder's column delta with the wrong sign
    "delta_sign": ("dkey[g] = (uint64_t)(col[g] - col[g - 1]);", "dkey[g] = (uint64_t)(col[g - 1] - col[g]);"),
    # the decoder appending a digit as the most significant one
    "digit_order": ("d[q] = d[q] * T->base[s] + T->digit[s];", "d[q] = d[q] + T->digit[s] * r[q];"),
    # unpack taking slot 1 from the highest 12 bits
    "unpack_order": ("slot[t] = (int)(V & 0xfff);\n        V >>= 12;",
                     "slot[7 - t] = (int)(V & 0xfff);\n        V >>= 12;"),
    # the row-sort window ordering rows by ascending length
    "sigma_ascending": ("row_ptr[perm[j - 1] + 1] - row_ptr[perm[j - 1]] < len",
                        "row_ptr[perm[j - 1] + 1] - row_ptr[perm[j - 1]] > len"),
}


@pytest.fixture(scope="module")
def builder(tmp_path_factory):
    src = open(SRC).read()
    d = tmp_path_factory.mktemp("mutants")

    def build(name):
        old, new = MUTANTS[name]
        assert src.count(old) == 1, name
        path = d / (name + ".c")
        path.write_text(src.replace(old, new))
        so = str(d / (name + ".so"))
        subprocess.check_call(["gcc", "-O1", "-std=gnu11", "-shared", "-fPIC", "-fopenmp", "-o", so, str(path)])
        return so
    return build


@pytest.fixture
def use(monkeypatch, builder):
    """Point the oracle package at a mutant library for one test."""
    def switch(name):
        good = oracle.lib()  # the real one, to copy the signatures from
        L = ctypes.CDLL(builder(name))
        for fn in ("oracle_set_threads", "oracle_csr_spmv_f64", "oracle_csr_absmv_f64", "oracle_csr_spmtv_f64",
                   "oracle_csr_spmm_f64", "oracle_encode", "oracle_decode", "oracle_read_header"):
            f, g = getattr(L, fn), getattr(good, fn)
            f.argtypes = g.argtypes
            f.restype = g.restype
        monkeypatch.setattr(oracle, "_lib", L)
    return switch


def _mat(seed=1, m=60, n=60, dens=0.1, pool=None):
    rng = np.random.default_rng(seed)
    A = sp.random(m, n, density=dens, format="csr", random_state=rng)
    A.sort_indices()
    v = A.data if pool is None else rng.choice(rng.standard_normal(pool), size=A.nnz)
    return A.indptr.astype(np.int32), A.indices.astype(np.int32), np.asarray(v, np.float64)


# ------------------------------------------------------------------ pins
def pin_spmv():
    rp, ci, v = _mat()
    A = sp.csr_matrix((v, ci, rp), shape=(60, 60))
    x = np.linspace(-1, 1, 60)
    y0 = np.cos(np.arange(60.0))
    np.testing.assert_allclose(oracle.spmv(rp, ci, v, x, y0.copy(), alpha=0.5, beta=2.0),
                               0.5 * (A @ x) + 2.0 * y0, rtol=1e-13, atol=1e-13)


def pin_spmtv():
    rp, ci, v = _mat(m=50, n=70)
    A = sp.csr_matrix((v, ci, rp), shape=(50, 70))
    x = np.linspace(-1, 1, 50)
    np.testing.assert_allclose(oracle.spmtv(rp, ci, v, 70, x), A.T @ x, rtol=1e-13, atol=1e-13)


def pin_spmm():
    rp, ci, v = _mat(m=40, n=30)
    A = sp.csr_matrix((v, ci, rp), shape=(40, 30))
    X = np.arange(30 * 5, dtype=np.float64).reshape(30, 5) / 7.0
    np.testing.assert_allclose(oracle.spmm(rp, ci, v, X), A @ X, rtol=1e-13, atol=1e-13)


def pin_roundtrip(tmp_path, layout=1, T=0, sigma=0):
    rp, ci, v = _mat(seed=3, m=200, n=150, dens=0.06, pool=20)
    p = str(tmp_path / "r.dtans")
    oracle.encode(p, 200, 150, rp, ci, v, layout=layout, lane_nnz=T, sigma=sigma)
    r2, c2, v2 = oracle.decode(p)
    assert np.array_equal(r2, rp) and np.array_equal(c2, ci) and np.array_equal(v2, v)
    # the Python big-integer codec (pinned to the paper's worked examples)
    # reads the same container
    r3, c3, v3 = container.decode(container.read(p))
    assert np.array_equal(r3, rp) and np.array_equal(c3, ci) and np.array_equal(v3, v)
    if sigma:
        assert list(container.read(p).perm) == container.sigma_order(np.diff(rp), sigma)


@pytest.mark.parametrize("name,pin", [("spmv_beta", "spmv"), ("spmv_index", "spmv"), ("spmtv_index", "spmtv"),
                                      ("spmm_stride", "spmm")])
def test_product_mutants_fail_their_pins(use, name, pin):
    {"spmv": pin_spmv, "spmtv": pin_spmtv, "spmm": pin_spmm}[pin]()  # passes on the real oracle
    use(name)
    with pytest.raises(AssertionError):
        {"spmv": pin_spmv, "spmtv": pin_spmtv, "spmm": pin_spmm}[pin]()


@pytest.mark.parametrize("name,layout,T,sigma", [("delta_sign", 1, 0, 0), ("digit_order", 2, 8, 0),
                                                 ("unpack_order", 1, 0, 0), ("sigma_ascending", 1, 0, 64)])
def test_codec_mutants_fail_their_pins(tmp_path, use, name, layout, T, sigma):
    pin_roundtrip(tmp_path, layout, T, sigma)  # passes on the real oracle
    use(name)
    with pytest.raises((AssertionError, oracle.OracleError, ValueError)):
        pin_roundtrip(tmp_path, layout, T, sigma)
