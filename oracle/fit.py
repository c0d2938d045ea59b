"""Exact alphabet fit of a CSR-dtANS coding table (oracle side).

TEST INFRASTRUCTURE ONLY.  Only ``tests/`` may import this module.

Sec. IV-F says the symbols kept in a table and their multiplicities are chosen
so that the expected total size is smallest, without giving the algorithm.
The reading used here (and in the design notes): a table of K slots holds t
ordinary symbols with multiplicities 1 <= m_i <= cap (cap <= M = 256,
Sec. IV-C) and, when some symbol is left out, one escape symbol with its own
multiplicity (Sec. IV-F, "Escaping rare values"); the sum of all
multiplicities is at most K (unused slots are allowed).  A symbol coded
through a table slot of base m costs log2(K / m) bits (the ideal ANS cost,
Eq. 2 summed over the data), an escaped symbol the escape symbol's cost plus
its raw bits (32 for a column delta and an FP32 value, 64 for an FP64 value).
The expected total size of an alphabet with counts c is therefore

    sum_{i in table} c_i log2(K / m_i) + E (log2(K / m_E) + raw_bits),

E being the count of escaped symbols (keys the table cannot hold, such as
column deltas >= 2^30, are always escaped).  At least one ordinary symbol is
kept (the padding of a lane's last segment needs one, Sec. IV-F).

The minimum is found without any search heuristic:

  * for a fixed number t of table symbols the t most frequent admissible keys
    are an optimal choice (exchanging a kept symbol for a more frequent
    escaped one moves count from a cost of at most log2(K) = 12 bits per
    symbol to one of at least raw_bits >= 32, so it never increases the size);
  * for each t the multiplicities are optimised exactly by dynamic
    programming over the number of slots used, A_t[s] = the least coded bits
    of the first t symbols using exactly s slots, built from A_{t-1} by one
    min-plus step over m = 1..cap; the escape symbol then takes
    min(cap, K - s) slots, since its cost falls with its multiplicity;
  * every t from 1 to the number of admissible keys (at most K, or K - 1 when
    something is escaped) is evaluated.

``brute_force`` enumerates every subset and every multiplicity vector and
pins the dynamic programme on tiny K.
"""
from __future__ import annotations

import itertools
import math
from typing import Dict, Iterable, List, Optional, Sequence, Tuple

import numpy as np

K_SLOTS = 4096
M_CAP = 256
DELTA_LIMIT = 1 << 30


def size_of(counts: Sequence[int], mult: Sequence[int], esc_count: int, esc_mult: int, raw_bits: int,
            K: int = K_SLOTS) -> float:
    """Expected total size in bits of one alphabet coded with the given table
    (the objective above)."""
    bits = 0.0
    for c, m in zip(counts, mult):
        if c:
            bits += c * math.log2(K / m)
    if esc_count:
        bits += esc_count * (math.log2(K / esc_mult) + raw_bits)
    return bits


def _candidates(hist: Dict[int, int], is_delta: bool) -> Tuple[List[int], int]:
    """Admissible keys' counts, most frequent first, and the forced escapes."""
    forced = sum(c for k, c in hist.items() if is_delta and k >= DELTA_LIMIT)
    cand = sorted((c for k, c in hist.items() if not (is_delta and k >= DELTA_LIMIT) and c > 0),
                  reverse=True)
    return cand, forced


def exact_fit(hist: Dict[int, int], raw_bits: int, is_delta: bool = False, K: int = K_SLOTS,
              cap: int = 255) -> Tuple[float, int]:
    """Smallest expected total size (bits) of an alphabet with histogram
    ``hist`` (key -> count) and the number of table symbols that reaches it
    (the smallest such number)."""
    if raw_bits < math.log2(K):
        raise ValueError("the top-t argument needs raw_bits >= log2(K)")
    cand, forced = _candidates(hist, is_delta)
    total = forced + sum(cand)
    if total == 0:
        return 0.0, 0
    if not cand:
        # only escapes: one (unused) ordinary symbol keeps a slot
        return size_of([], [], forced, min(cap, K - 1), raw_bits, K), 1
    suffix = np.concatenate([np.cumsum(np.asarray(cand[::-1], np.float64))[::-1], [0.0]])
    inf = np.inf
    A = np.full(K + 1, inf)
    A[0] = 0.0
    mvals = np.arange(1, cap + 1)
    w = np.log2(K / mvals)  # cost per occurrence at multiplicity m
    best, best_t = inf, 0
    tmax = min(len(cand), K)
    for t in range(1, tmax + 1):
        c = cand[t - 1]
        new = np.full(K + 1, inf)
        for m in range(1, cap + 1):
            if m > K:
                break
            np.minimum(new[m:], A[:K + 1 - m] + c * w[m - 1], out=new[m:])
        A = new
        esc = forced + float(suffix[t])
        if esc > 0:
            if t > K - 1:
                continue
            s = np.arange(K + 1)
            room = np.minimum(cap, K - s)
            ok = room >= 1
            tot = np.where(ok, A + esc * (np.log2(K / np.maximum(room, 1)) + raw_bits), inf)
            cost = float(tot.min())
        else:
            cost = float(A.min())
        if cost < best:
            best, best_t = cost, t
    return best, best_t


def brute_force(hist: Dict[int, int], raw_bits: int, is_delta: bool = False, K: int = 16,
                cap: int = 6) -> float:
    """The same minimum by enumeration of every subset of admissible keys
    and every multiplicity vector (tiny K and alphabets only)."""
    cand, forced = _candidates(hist, is_delta)
    if forced + sum(cand) == 0:
        return 0.0
    best = math.inf
    idx = range(len(cand))
    for t in range(1, len(cand) + 1):
        for kept in itertools.combinations(idx, t):
            esc = forced + sum(cand[i] for i in idx if i not in kept)
            syms = [cand[i] for i in kept] + ([esc] if esc else [])
            for mult in itertools.product(range(1, cap + 1), repeat=len(syms)):
                if sum(mult) > K:
                    continue
                bits = size_of(syms[:t], mult[:t], esc, mult[t] if esc else 1, raw_bits, K)
                best = min(best, bits)
    if not cand:
        best = size_of([], [], forced, min(cap, K - 1), raw_bits, K)
    return best


def table_size(hist: Dict[int, int], symbols: Iterable, base_of: Dict, esc_base: Optional[int],
               raw_bits: int, is_delta: bool = False, K: int = K_SLOTS) -> float:
    """Expected total size of ``hist`` coded by a given table: ``base_of``
    maps each table key to its multiplicity, ``esc_base`` is the escape
    symbol's multiplicity (None: no escape symbol).  Keys outside the table
    are escaped; it is an error for one to occur without an escape symbol."""
    keys = set(symbols)
    counts, mult, esc = [], [], 0
    for k, c in hist.items():
        if k in keys and not (is_delta and k >= DELTA_LIMIT):
            counts.append(c)
            mult.append(base_of[k])
        else:
            esc += c
    if esc and esc_base is None:
        raise ValueError("escaped keys but the table has no escape symbol")
    return size_of(counts, mult, esc, esc_base or 1, raw_bits, K)
