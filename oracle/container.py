"""CSR-dtANS container file: a Python reader/writer and a big-integer codec.

TEST INFRASTRUCTURE ONLY (oracle side).  It reads and writes the container
byte format with its own code and decodes/encodes whole matrices through the
generic toy codec of ``oracle.toy`` at the CSR-dtANS parameters (W = 2^32,
K = 4096, M = 256, l = 8, o = 3, f = 2; Sec. IV-D).  It is slow and meant for
matrices of at most a few thousand nonzeros, where it pins the C oracle's wave
interleaving, escapes and padding (Sec. IV-B, IV-F) against an implementation
whose per-lane arithmetic is pinned to the paper's worked examples.

Container layout (little endian), version 1:

  header (256 bytes): magic "CSRDTANS", u32 version=1, u32 dtype (1 FP32,
    2 FP64), u32 layout (1: lane = one row, 2: lane = T nonzeros), u32 T,
    i64 m, n, nnz, num_lanes, num_waves, n_words, n_esc_delta, n_esc_value,
    u64 perm_seed, u64 FNV-1a-64 checksum of every byte after the header,
    u32 first-delta mode at byte 104, u32 escape mode at byte 108 (0: raw
    bits of escaped symbols in the esc_delta / esc_value regions; 1: in the
    word stream, a step's escaped deltas then values, (position, lane) order,
    FP64 values as two words low first, between the words read before that
    step and the words its checks read; Sec. IV-F), u32 row-sort window sigma
    at byte 112 (0: rows in CSR order; else the encoded rows are the original
    ones sorted by descending length within windows of sigma rows, a
    SELL-C-sigma base, and an (m) x i32 section after esc_value holds the
    original row of every encoded row);
  delta table, value table: 4096 entries of 16 bytes each
    (u64 symbol, u8 digit, u8 base-1, u8 flags: bit0 used, bit1 escape);
  row_ptr: (m+1) x i32;  word_off, esc_delta_off, esc_value_off:
    (num_waves+1) x u64 each;  words: u32;  esc_delta: u32;
    esc_value: u32 (FP32) or u64 (FP64).  Every section starts 8-aligned.
"""
from __future__ import annotations

import random
import struct
from dataclasses import dataclass
from typing import List, Optional

import numpy as np

from . import toy

K = 4096
M = 256
WAVE = 64
DELTA_LIMIT = 1 << 30
FIRST_BIAS = 1 << 29  # first-delta mode 1 (an extension of the paper's format)
HEADER = 256
ESC = "ESC"


def _fnv1a64_np(buf: np.ndarray) -> int:
    """FNV-1a, 64-bit (Fowler, Noll, Vo), one byte at a time."""
    h = 0xCBF29CE484222325
    for b in buf.tobytes():
        h ^= b
        h = (h * 0x100000001B3) & 0xFFFFFFFFFFFFFFFF
    return h


@dataclass
class Container:
    dtype: int
    layout: int
    lane_nnz: int
    m: int
    n: int
    nnz: int
    num_lanes: int
    num_waves: int
    seed: int
    dtab: toy.Tables
    vtab: toy.Tables
    row_ptr: np.ndarray
    word_off: np.ndarray
    escd_off: np.ndarray
    escv_off: np.ndarray
    words: np.ndarray
    escd: np.ndarray
    escv: np.ndarray
    first_mode: int = 0  # first delta of a row: 0 its column, 1 column - row + 2^29
    esc_mode: int = 0    # escaped symbols: 0 separate regions, 1 in the word stream
    sigma: int = 0       # row-sort window (0: CSR order)
    perm: Optional[np.ndarray] = None  # original row of each encoded row (sigma > 0)


def _al8(x: int) -> int:
    return (x + 7) & ~7


def _table_from_bytes(b: bytes) -> toy.Tables:
    sym, dig, base = [], [], []
    for i in range(K):
        key, d, bm1, fl = struct.unpack_from("<QBBB", b, 16 * i)
        if fl & 1:
            sym.append(ESC if fl & 2 else key)
            dig.append(d)
            base.append(bm1 + 1)
        else:
            sym.append(None)
            dig.append(0)
            base.append(0)
    return toy.Tables(sym, dig, base)


def _table_to_bytes(t: toy.Tables) -> bytes:
    out = bytearray(16 * K)
    for i in range(K):
        if t.symbol[i] is None:
            continue
        esc = t.symbol[i] == ESC
        struct.pack_into("<QBBB", out, 16 * i, 0 if esc else int(t.symbol[i]),
                         t.digit[i], t.base[i] - 1, 1 | (2 if esc else 0))
    return bytes(out)


def read(path: str, verify: bool = True) -> Container:
    data = open(path, "rb").read()
    if data[:8] != b"CSRDTANS":
        raise ValueError("bad magic")
    (ver, dtype, layout, T) = struct.unpack_from("<IIII", data, 8)
    (m, n, nnz, lanes, waves, nw, nd, nv, seed, chk) = struct.unpack_from("<qqqqqqqqQQ", data, 24)
    if ver != 1:
        raise ValueError("bad version")
    if verify and _fnv1a64_np(np.frombuffer(data, np.uint8, offset=HEADER)) != chk:
        raise ValueError("checksum mismatch")
    o = HEADER
    dtab = _table_from_bytes(data[o:o + 16 * K]); o = _al8(o + 16 * K)
    vtab = _table_from_bytes(data[o:o + 16 * K]); o = _al8(o + 16 * K)

    def take(dt, count):
        nonlocal o
        arr = np.frombuffer(data, dtype=dt, count=count, offset=o).copy()
        o = _al8(o + arr.nbytes)
        return arr

    row_ptr = take("<i4", m + 1)
    woff = take("<u8", waves + 1)
    doff = take("<u8", waves + 1)
    voff = take("<u8", waves + 1)
    words = take("<u4", nw)
    escd = take("<u4", nd)
    escv = take("<u8" if dtype == 2 else "<u4", nv)
    (first_mode, esc_mode, sigma) = struct.unpack_from("<III", data, 104)
    perm = take("<i4", m) if sigma else None
    if o != len(data):
        raise ValueError("size mismatch")
    if sigma % WAVE or (sigma and layout != 1):
        raise ValueError("bad row-sort window")
    if first_mode > 1:
        raise ValueError("bad first-delta mode")
    if esc_mode > 1 or (esc_mode == 1 and (nd or nv)):
        raise ValueError("bad escape mode")
    return Container(dtype, layout, T, m, n, nnz, lanes, waves, seed, dtab, vtab,
                     row_ptr, woff, doff, voff, words, escd, escv, first_mode, esc_mode, sigma, perm)


def write(path: str, c: Container) -> None:
    body = bytearray()

    def put(b: bytes):
        body.extend(b)
        while (len(body) + HEADER) % 8:
            body.append(0)

    put(_table_to_bytes(c.dtab))
    put(_table_to_bytes(c.vtab))
    put(np.asarray(c.row_ptr, "<i4").tobytes())
    put(np.asarray(c.word_off, "<u8").tobytes())
    put(np.asarray(c.escd_off, "<u8").tobytes())
    put(np.asarray(c.escv_off, "<u8").tobytes())
    put(np.asarray(c.words, "<u4").tobytes())
    put(np.asarray(c.escd, "<u4").tobytes())
    put(np.asarray(c.escv, "<u8" if c.dtype == 2 else "<u4").tobytes())
    if c.sigma:
        put(np.asarray(c.perm, "<i4").tobytes())
    hdr = bytearray(HEADER)
    hdr[:8] = b"CSRDTANS"
    struct.pack_into("<IIII", hdr, 8, 1, c.dtype, c.layout, c.lane_nnz)
    struct.pack_into("<qqqqqqqqQQ", hdr, 24, c.m, c.n, c.nnz, c.num_lanes, c.num_waves,
                     len(c.words), len(c.escd), len(c.escv), c.seed,
                     _fnv1a64_np(np.frombuffer(bytes(body), np.uint8)))
    struct.pack_into("<III", hdr, 104, c.first_mode, c.esc_mode, c.sigma)
    with open(path, "wb") as f:
        f.write(bytes(hdr) + bytes(body))


# --------------------------------------------------------------------------
# lanes and symbols
# --------------------------------------------------------------------------
def lane_ranges(layout: int, lane_nnz: int, m: int, nnz: int, row_ptr) -> List[tuple]:
    if layout == 1:
        return [(int(row_ptr[i]), int(row_ptr[i + 1] - row_ptr[i])) for i in range(m)]
    lanes = (nnz + lane_nnz - 1) // lane_nnz
    return [(l * lane_nnz, min(lane_nnz, nnz - l * lane_nnz)) for l in range(lanes)]


def row_of(row_ptr, g: int) -> int:
    """The row holding nonzero g (the last i with row_ptr[i] <= g)."""
    return int(np.searchsorted(np.asarray(row_ptr), g, side="right")) - 1


def first_base(first_mode: int, row: int) -> int:
    """Start value of a row's column accumulation: 0 (mode 0, the paper's form)
    or row - 2^29 modulo 2^32 (mode 1)."""
    return (row - FIRST_BIAS) % (1 << 32) if first_mode else 0


def delta_keys(row_ptr, col, ranges, first_mode: int = 0) -> List[int]:
    """Column delta per nonzero: for the first nonzero of a row or of a lane
    stream the column itself (mode 0, Sec. IV-A) or column - row + 2^29 modulo
    2^32 (mode 1), else the difference to the previous column (rows are
    delta-encoded separately)."""
    first = set(int(row_ptr[i]) for i in range(len(row_ptr) - 1) if row_ptr[i] < row_ptr[i + 1])
    d = [0] * len(col)
    for g0, c in ranges:
        for t in range(c):
            g = g0 + t
            if t == 0 or g in first:
                d[g] = (int(col[g]) - first_base(first_mode, row_of(row_ptr, g))) % (1 << 32)
            else:
                d[g] = int(col[g]) - int(col[g - 1])
    return d


def value_keys(vals, dtype: int) -> List[int]:
    a = np.ascontiguousarray(vals)
    return [int(x) for x in a.view(np.uint64 if dtype == 2 else np.uint32)]


# --------------------------------------------------------------------------
# whole-container decode, lanes of a wave in lockstep (Alg. 3)
# --------------------------------------------------------------------------
def decode(c: Container):
    p = toy.CSR_DTANS
    nnz = c.nnz
    col = np.zeros(nnz, np.int64)
    keys = [0] * nnz
    ranges = lane_ranges(c.layout, c.lane_nnz, c.m, c.nnz, c.row_ptr)
    first = set(int(c.row_ptr[i]) for i in range(c.m) if c.row_ptr[i] < c.row_ptr[i + 1])
    tabs = (c.dtab, c.vtab)
    for w in range(c.num_waves):
        wp, wend = int(c.word_off[w]), int(c.word_off[w + 1])
        dp, dend = int(c.escd_off[w]), int(c.escd_off[w + 1])
        vp, vend = int(c.escv_off[w]), int(c.escv_off[w + 1])
        lanes = ranges[w * WAVE:(w + 1) * WAVE]
        S = [(cnt + 3) // 4 for _, cnt in lanes]
        words = [[0, 0, 0] for _ in lanes]
        st = [[0, 1] for _ in lanes]
        colv = [0] * len(lanes)

        def nxt():
            nonlocal wp
            if wp >= wend:
                raise ValueError("stream exhausted")
            x = int(c.words[wp]); wp += 1
            return x

        for k in range(3):
            for q in range(len(lanes)):
                if S[q] > 0:
                    words[q][k] = nxt()
        for j in range(max(S, default=0)):
            slots = {q: toy.unpack(words[q], p) for q in range(len(lanes)) if j < S[q]}
            for pos in range(4):
                for q in slots:
                    t = 4 * j + pos
                    if t >= lanes[q][1]:
                        continue
                    s = c.dtab.symbol[slots[q][2 * pos]]
                    if s is None:
                        raise ValueError("unused slot")
                    if s == ESC and c.esc_mode == 1:
                        s = nxt()
                    elif s == ESC:
                        s = int(c.escd[dp]); dp += 1
                    g = lanes[q][0] + t
                    if t == 0 or g in first:
                        colv[q] = (first_base(c.first_mode, row_of(c.row_ptr, g)) + s) % (1 << 32)
                    else:
                        colv[q] = colv[q] + s
                    col[g] = colv[q]
            for pos in range(4):
                for q in slots:
                    t = 4 * j + pos
                    if t >= lanes[q][1]:
                        continue
                    s = c.vtab.symbol[slots[q][2 * pos + 1]]
                    if s is None:
                        raise ValueError("unused slot")
                    if s == ESC and c.esc_mode == 1:
                        s = nxt()
                        if c.dtype == 2:
                            s |= nxt() << 32
                    elif s == ESC:
                        s = int(c.escv[vp]); vp += 1
                    keys[lanes[q][0] + t] = s
            for g in range(2):
                for q in slots:
                    if j >= S[q] - 1:
                        continue
                    d, r = st[q]
                    for t in range(4 * g, 4 * g + 4):
                        T = tabs[t % 2]
                        i = slots[q][t]
                        d = d * T.base[i] + T.digit[i]
                        r = r * T.base[i]
                    if r >= p.W:
                        words[q][g] = d % p.W
                        d, r = d // p.W, r // p.W
                    else:
                        words[q][g] = nxt()
                    st[q] = [d, r]
            for q in slots:
                if j < S[q] - 1:
                    words[q][2] = nxt()
        if wp != wend or dp != dend or vp != vend:
            raise ValueError("wave %d: stored and consumed words differ" % w)
    vdt = np.uint64 if c.dtype == 2 else np.uint32
    vals = np.array(keys, dtype=vdt).view(np.float64 if c.dtype == 2 else np.float32)
    if not c.sigma:
        return c.row_ptr.copy(), col.astype(np.int32), vals
    # rows back into their original order; the stored order must be the
    # canonical one for these row lengths
    lens = np.diff(c.row_ptr.astype(np.int64))
    orig_len = np.zeros(c.m, np.int64)
    orig_len[c.perm] = lens
    if sorted(c.perm.tolist()) != list(range(c.m)) or list(sigma_order(orig_len, c.sigma)) != c.perm.tolist():
        raise ValueError("bad row order")
    rp = np.zeros(c.m + 1, np.int64)
    rp[1:] = np.cumsum(orig_len)
    col2, vals2 = np.zeros_like(col), np.zeros_like(vals)
    for r in range(c.m):
        i = int(c.perm[r])
        col2[rp[i]:rp[i + 1]] = col[c.row_ptr[r]:c.row_ptr[r + 1]]
        vals2[rp[i]:rp[i + 1]] = vals[c.row_ptr[r]:c.row_ptr[r + 1]]
    return rp.astype(np.int32), col2.astype(np.int32), vals2


def sigma_order(lengths, sigma: int) -> List[int]:
    """SELL-C-sigma row order (Kreutzer et al. 2014): within each window of
    sigma rows, rows by descending length, ties in their original order."""
    m = len(lengths)
    out = []
    for w0 in range(0, m, sigma):
        out.extend(sorted(range(w0, min(m, w0 + sigma)), key=lambda i: -int(lengths[i])))
    return out


# --------------------------------------------------------------------------
# whole-container encode with given tables (two-pass encoder, Sec. IV-E)
# --------------------------------------------------------------------------
def simple_tables(dkeys, vkeys, seed: int):
    """A valid pair of tables for small inputs: keys seen once are escaped
    (deltas at or above 2^30 always are), every other key gets a
    multiplicity equal to its count capped at M, slots shuffled."""
    rng = random.Random(seed)
    out = []
    for keys, is_delta in ((dkeys, True), (vkeys, False)):
        cnt = {}
        for k in keys:
            cnt[k] = cnt.get(k, 0) + 1
        table = sorted(k for k, v in cnt.items() if v > 1 and (not is_delta or k < DELTA_LIMIT))
        if not table and cnt:
            cand = sorted(k for k in cnt if not is_delta or k < DELTA_LIMIT)
            table = cand[:1] if cand else [0]
        esc = sum(v for k, v in cnt.items() if k not in set(table))
        mult = [(k, min(M, cnt.get(k, 1))) for k in table]
        if esc:
            mult.append((ESC, min(M, esc)))
        assert sum(mm for _, mm in mult) <= K
        sym, dig, base = [None] * K, [0] * K, [0] * K
        order = list(range(K))
        rng.shuffle(order)
        it = iter(order)
        for s, mm in mult:
            for d in range(mm):
                slot = next(it)
                sym[slot], dig[slot], base[slot] = s, d, mm
        out.append(toy.Tables(sym, dig, base))
    return out[0], out[1]


def encode(m, n, row_ptr, col, vals, dtype: int, layout: int = 1, lane_nnz: int = 0,
           tables: Optional[tuple] = None, seed: int = 1, first_mode: int = 0,
           esc_mode: int = 0, sigma: int = 0) -> Container:
    p = toy.CSR_DTANS
    row_ptr = np.asarray(row_ptr, np.int64)
    perm = None
    if sigma:  # encode the rows in SELL-C-sigma order
        assert layout == 1 and sigma % WAVE == 0
        perm = np.array(sigma_order(np.diff(row_ptr), sigma), np.int32)
        col = np.asarray(col)
        vals = np.asarray(vals)
        rows = [np.arange(row_ptr[i], row_ptr[i + 1]) for i in perm]
        idx = np.concatenate(rows) if rows else np.zeros(0, np.int64)
        col, vals = col[idx], vals[idx]
        row_ptr = np.concatenate([[0], np.cumsum([len(r) for r in rows])]).astype(np.int64)
    nnz = int(row_ptr[-1])
    ranges = lane_ranges(layout, lane_nnz, m, nnz, row_ptr)
    dk = delta_keys(row_ptr, col, ranges, first_mode)
    vk = value_keys(vals, dtype)
    dtab, vtab = tables if tables is not None else simple_tables(dk, vk, seed)
    tabs = (dtab, vtab)
    dset = set(s for s in dtab.symbol if s is not None and s != ESC)
    vset = set(s for s in vtab.symbol if s is not None and s != ESC)
    # padding: the symbol on the lowest-numbered used non-escape slot
    dpad = next((s for s in dtab.symbol if s is not None and s != ESC), None)
    vpad = next((s for s in vtab.symbol if s is not None and s != ESC), None)
    words, escd, escv = [], [], []
    woff, doff, voff = [0], [0], [0]
    waves = (len(ranges) + WAVE - 1) // WAVE
    for w in range(waves):
        lanes = ranges[w * WAVE:(w + 1) * WAVE]
        per = []
        for g0, cnt in lanes:
            S = (cnt + 3) // 4
            if S == 0:
                per.append(None)
                continue
            u = []
            for t in range(4 * S):
                if t < cnt:
                    dkey, vkey = dk[g0 + t], vk[g0 + t]
                    u.append(dkey if dkey in dset else ESC)
                    u.append(vkey if vkey in vset else ESC)
                else:
                    u.extend([dpad, vpad])
            lw = toy.dtans_encode(u, tabs, p, skip_tail=True)
            flags = toy.dtans_base_pass(u, tabs, p, skip_tail=True)
            init, rest = lw[:3], lw[3:]
            steps, i = [], 0
            for fj in flags:
                c1 = None if fj[0] else rest[i]; i += (0 if fj[0] else 1)
                c2 = None if fj[1] else rest[i]; i += (0 if fj[1] else 1)
                steps.append((c1, c2, rest[i])); i += 1
            assert i == len(rest)
            per.append((init, steps))
        for r in range(3):
            for e in per:
                if e is not None:
                    words.append(e[0][r])
        maxS = max(((cnt + 3) // 4 for _, cnt in lanes), default=0)

        def escapes(j, out_d, out_v):
            for pos in range(4):
                for g0, cnt in lanes:
                    t = 4 * j + pos
                    if t < cnt and dk[g0 + t] not in dset:
                        out_d.append(dk[g0 + t])
            for pos in range(4):
                for g0, cnt in lanes:
                    t = 4 * j + pos
                    if t < cnt and vk[g0 + t] not in vset:
                        if esc_mode == 1:  # one or two words, low first
                            out_v.append(vk[g0 + t] & 0xFFFFFFFF)
                            if dtype == 2:
                                out_v.append(vk[g0 + t] >> 32)
                        else:
                            out_v.append(vk[g0 + t])

        for j in range(maxS):
            if esc_mode == 1:
                escapes(j, words, words)
            if j == maxS - 1:
                break
            for k in range(3):
                for e in per:
                    if e is None or j >= len(e[1]):
                        continue
                    x = e[1][j][k]
                    if x is not None:
                        words.append(x)
        if esc_mode == 0:
            for j in range(maxS):
                escapes(j, escd, [])
            for j in range(maxS):
                escapes(j, [], escv)
        woff.append(len(words)); doff.append(len(escd)); voff.append(len(escv))
    return Container(dtype, layout, lane_nnz if layout == 2 else 0, m, n, nnz, len(ranges), waves,
                     seed, dtab, vtab, row_ptr.astype(np.int32), np.array(woff, np.uint64),
                     np.array(doff, np.uint64), np.array(voff, np.uint64),
                     np.array(words, np.uint32), np.array(escd, np.uint32),
                     np.array(escv, np.uint64 if dtype == 2 else np.uint32), first_mode, esc_mode,
                     sigma, perm)
