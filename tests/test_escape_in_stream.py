"""Escaped symbols stored inside the word stream (Sec. IV-F).

The paper gives two places for the raw bits of an escaped symbol: read from
the stream right after the decoding step that meets the escape symbol, or
from a separate stream.  The default containers use a separate region per
wave; escape mode 1 puts a step's escaped deltas and then its escaped values,
each nonzero position in lane order, into the word stream between the words
read before the step and the words its checks read (FP64 values as two
words, low half first).  Pins:

* hand-laid streams: a one-row matrix with a forced delta escape and a value
  escape, whose stream words are written out here from the layout above;
* the C oracle and the Python big-integer container codec write identical
  bytes from the same tables and decode each other's containers;
* the in-stream container holds exactly the separate container's words plus
  one word per escaped delta and one (FP32) or two (FP64) per escaped value;
* the library's encoder writes containers both oracles decode, and loads
  (decoding every stream on the host) oracle-written in-stream containers.
"""
import struct

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import paper_2603_01915_amd as P
from oracle import container


def _rand(m, n, dens, seed, dtype, pool, unique_every=0, big_cols=False):
    rng = np.random.default_rng(seed)
    A = sp.random(m, n, density=dens, format="csr", random_state=rng)
    A.sort_indices()
    ci = A.indices.astype(np.int64)
    if big_cols:  # deltas at or above 2^30 are always escaped
        ci = ci * 20_000_000
        n = 2 ** 31 - 1
    v = rng.choice(rng.standard_normal(pool), size=A.nnz).astype(dtype)
    if unique_every:
        v[::unique_every] = rng.standard_normal(len(v[::unique_every]))
    return A.indptr.astype(np.int32), ci.astype(np.int32), v, n


def _escaped(tab, keys):
    """Keys a table does not hold (their symbol is the escape)."""
    held = set(x for x in tab.symbol if x is not None and x != container.ESC)
    return [k for k in keys if k not in held]


def test_hand_laid_stream(tmp_path):
    # one row of three nonzeros (one step), FP64: columns 0, 1, 2^30 + 5
    # (deltas 0, 1, 2^30 + 4: the last is escaped whatever the tables), values
    # 1.5, 1.5, 7.25 (7.25 seen once: escaped by the simple tables)
    col = [0, 1, 2 ** 30 + 5]
    rp = np.array([0, 3], np.int32)
    ci = np.array(col, np.int32)
    v = np.array([1.5, 1.5, 7.25])
    n = 2 ** 30 + 10
    sep = container.encode(1, n, rp, ci, v, 2, 1, 0, seed=3, esc_mode=0)
    ins = container.encode(1, n, rp, ci, v, 2, 1, 0, tables=(sep.dtab, sep.vtab), seed=3, esc_mode=1)
    dk = _escaped(sep.dtab, [0, 1, 2 ** 30 + 4])
    bits = struct.unpack("<Q", struct.pack("<d", 7.25))[0]
    assert 2 ** 30 + 4 in dk and _escaped(sep.vtab, [struct.unpack("<Q", struct.pack("<d", x))[0] for x in v]) == [bits]
    # separate mode: 3 initial words (one lane, one step, no checks), escapes aside
    assert len(sep.words) == 3 and list(sep.escd) == dk and list(sep.escv) == [bits]
    # in-stream mode: the same 3 words, then the step's escaped deltas in
    # position order, then its escaped value as low and high word
    assert list(ins.words) == list(sep.words) + dk + [bits & 0xFFFFFFFF, bits >> 32]
    assert len(ins.escd) == 0 and len(ins.escv) == 0
    # both decoders read the hand-laid stream back
    p = str(tmp_path / "h.dtans")
    container.write(p, ins)
    r2, c2, v2 = oracle.decode(p)
    assert list(c2) == col and np.array_equal(v2, v)
    _, c3, v3 = container.decode(container.read(p))
    assert list(c3) == col and np.array_equal(v3, v)
    assert oracle.read_header(p)["esc_mode"] == 1


def test_hand_laid_two_steps_fp32(tmp_path):
    # one row of 6 nonzeros (two steps), FP32, deltas 0, 2^30 + 1, 1, 1, 1,
    # 2^30 - 6: escapes in both steps, the last step's after every word
    col = [0, 2 ** 30 + 1, 2 ** 30 + 2, 2 ** 30 + 3, 2 ** 30 + 4, 2 ** 31 - 2]
    deltas = [0, 2 ** 30 + 1, 1, 1, 1, 2 ** 30 - 6]
    rp = np.array([0, 6], np.int32)
    ci = np.array(col, np.int32)
    v = np.array([2.0] * 6, np.float32)
    sep = container.encode(1, 2 ** 31 - 1, rp, ci, v, 1, 1, 0, seed=4)
    ins = container.encode(1, 2 ** 31 - 1, rp, ci, v, 1, 1, 0, tables=(sep.dtab, sep.vtab), seed=4, esc_mode=1)
    e0, e1 = _escaped(sep.dtab, deltas[:4]), _escaped(sep.dtab, deltas[4:])
    assert 2 ** 30 + 1 in e0 and 2 ** 30 - 6 in e1
    assert list(sep.escd) == e0 + e1 and len(sep.escv) == 0
    w = list(sep.words)
    # 3 initial words, step 0's escapes, step 0's words (the rest of the
    # separate stream: step 1 reads none), step 1's escapes last
    assert list(ins.words) == w[:3] + e0 + w[3:] + e1
    p = str(tmp_path / "h2.dtans")
    container.write(p, ins)
    _, c2, v2 = oracle.decode(p)
    assert list(c2) == col and np.array_equal(v2, v)


@pytest.mark.parametrize("layout,T", [(1, 0), (2, 8), (2, 12)])
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("case", [0, 1, 2])
def test_oracles_agree_in_stream(tmp_path, layout, T, dtype, case):
    rp, ci, v, n = _rand(130, 90, 0.08, 10 + case, dtype, 5, unique_every=3 if case == 1 else 0,
                         big_cols=case == 2)
    m = len(rp) - 1
    dt = 2 if dtype == np.float64 else 1
    p1 = str(tmp_path / "c.dtans")
    oracle.encode(p1, m, n, rp, ci, v, layout=layout, lane_nnz=T, seed=77, esc_mode=1)
    c = container.read(p1)
    assert c.esc_mode == 1 and len(c.escd) == 0 and len(c.escv) == 0
    _, c3, v3 = container.decode(c)
    assert np.array_equal(c3, ci) and np.array_equal(v3.view(np.uint8), v.view(np.uint8))
    c6 = container.encode(m, n, rp, ci, v, dt, layout, T, tables=(c.dtab, c.vtab), seed=c.seed, esc_mode=1)
    p2 = str(tmp_path / "p.dtans")
    container.write(p2, c6)
    assert open(p1, "rb").read() == open(p2, "rb").read()
    c4 = container.encode(m, n, rp, ci, v, dt, layout, T, seed=5, esc_mode=1)
    container.write(p2, c4)
    _, c5, v5 = oracle.decode(p2)
    assert np.array_equal(c5, ci) and np.array_equal(v5.view(np.uint8), v.view(np.uint8))


@pytest.mark.parametrize("layout,T", [(1, 0), (2, 16)])
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_word_count_identity(tmp_path, layout, T, dtype):
    rp, ci, v, n = _rand(400, 300, 0.05, 21, dtype, 100000)
    m = len(rp) - 1
    p0, p1 = str(tmp_path / "s.dtans"), str(tmp_path / "i.dtans")
    oracle.encode(p0, m, n, rp, ci, v, layout=layout, lane_nnz=T, seed=9, esc_mode=0)
    oracle.encode(p1, m, n, rp, ci, v, layout=layout, lane_nnz=T, seed=9, esc_mode=1)
    h0, h1 = oracle.read_header(p0), oracle.read_header(p1)
    assert h0["n_esc_value"] > 0
    per_value = 2 if dtype == np.float64 else 1
    assert h1["n_words"] == h0["n_words"] + h0["n_esc_delta"] + per_value * h0["n_esc_value"]
    assert h1["n_esc_delta"] == 0 and h1["n_esc_value"] == 0


@pytest.mark.parametrize("layout,T", [("row", 0), ("nnz", 8), ("nnz", 60)])
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_library_in_stream_containers(tmp_path, layout, T, dtype):
    rp, ci, v, n = _rand(700, 500, 0.03, 31, dtype, 100000)
    A = P.Matrix.from_csr(rp, ci, v, n, layout=layout, lane_nnz=T, escape_in_stream=True)
    B = P.Matrix.from_csr(rp, ci, v, n, layout=layout, lane_nnz=T)
    ia, ib = A.info(), B.info()
    assert ia["escape_in_stream"] == 1 and ib["escape_in_stream"] == 0
    assert ib["esc_value"] > 0 and ia["esc_delta"] == 0 and ia["esc_value"] == 0
    per_value = 2 if dtype == np.float64 else 1
    assert ia["words"] == ib["words"] + ib["esc_delta"] + per_value * ib["esc_value"]
    path = str(tmp_path / "lib.dtans")
    A.save(path)
    r2, c2, v2 = oracle.decode(path)
    assert np.array_equal(r2, rp) and np.array_equal(c2, ci)
    assert np.array_equal(v2.view(np.uint8), v.view(np.uint8))
    _, c3, v3 = container.decode(container.read(path))
    assert np.array_equal(c3, ci) and np.array_equal(v3.view(np.uint8), v.view(np.uint8))
    # loading decodes every stream on the host; saving again gives the same bytes
    p2 = str(tmp_path / "again.dtans")
    P.Matrix.load(path).save(p2)
    assert open(path, "rb").read() == open(p2, "rb").read()


@pytest.mark.parametrize("layout,T", [(1, 0), (2, 8)])
def test_library_loads_oracle_in_stream(tmp_path, layout, T):
    rp, ci, v, n = _rand(300, 100, 0.05, 2, np.float64, 50, unique_every=2, big_cols=True)
    path = str(tmp_path / "or.dtans")
    oracle.encode(path, 300, n, rp, ci, v, layout=layout, lane_nnz=T, esc_mode=1)
    A = P.Matrix.load(path)
    assert A.info()["escape_in_stream"] == 1
    p2 = str(tmp_path / "again.dtans")
    A.save(p2)
    assert open(path, "rb").read() == open(p2, "rb").read()


def test_corrupted_in_stream_rejected(tmp_path):
    rp, ci, v, n = _rand(200, 100, 0.05, 4, np.float32, 1000, big_cols=True)
    path = str(tmp_path / "x.dtans")
    oracle.encode(path, 200, n, rp, ci, v, esc_mode=1)
    data = bytearray(open(path, "rb").read())
    # claim separate regions for an in-stream stream: the words no longer add up
    struct.pack_into("<I", data, 108, 0)
    bad = str(tmp_path / "bad.dtans")
    open(bad, "wb").write(bytes(data))
    with pytest.raises(oracle.OracleError):
        oracle.decode(bad)
    with pytest.raises(P.DtansError):
        P.Matrix.load(bad)
    struct.pack_into("<I", data, 108, 2)
    open(bad, "wb").write(bytes(data))
    with pytest.raises(oracle.OracleError):
        oracle.decode(bad)
    with pytest.raises(P.DtansError):
        P.Matrix.load(bad)
