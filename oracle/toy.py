"""Generic big-integer tANS / dtANS codec for small examples.

TEST INFRASTRUCTURE ONLY: this module belongs to the oracle. Only tests,
``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may use it.
It shares no code with the HIP path.

Everything here follows the paper (Schaetzle, Pegolotti, Pueschel, "Fast
Entropy Decoding for Sparse MVM on GPUs", 2026) with Python integers, so that
any word size W, table size K, multiplicity cap M, segment length l, words per
segment o and check count f can be run by hand:

* mixed-radix states and tANS encode/decode: Sec. III-C..E, Alg. 1 and Alg. 2;
* dtANS unpack/pack, decoding with conditional and unconditional loads:
  Sec. IV-D, Alg. 3 and its worked example (W=4, K=8, M=4, l=2, o=3, f=2);
* the two-pass dtANS encoder (forward base pass, backward digit pass):
  Sec. IV-E;
* skipping the trailing loads of a stream whose length is known: Sec. IV-F.

Readings of the text that this module takes (each one is exercised by a test):

* Check placement.  Alg. 3 as printed appends all l digits and then performs
  the f checks; the worked example of Sec. IV-D instead performs check g right
  after digit group g (groups of l/f consecutive symbols).  Only the latter
  reproduces the printed stream, so it is the default (``order="grouped"``);
  the literal order is kept as ``order="after_all"`` for the test that shows
  the difference.
* Digit order.  A returned digit is appended as the new least significant
  digit of the decoder state (d <- d*base + digit); an extraction takes the
  least significant word (d mod W).
* unpack/pack.  The o words form one number with w_1 most significant; the l
  slots are its base-K digits with i_1 least significant.
"""
from __future__ import annotations

from dataclasses import dataclass
from fractions import Fraction
import math
from typing import Dict, List, Sequence, Tuple


# --------------------------------------------------------------------------
# coding tables (Sec. III-D "Constructing the coding table")
# --------------------------------------------------------------------------
@dataclass
class Tables:
    """Per-slot ``symbol``, ``digit`` and ``base`` tables over K slots."""

    symbol: List[object]
    digit: List[int]
    base: List[int]

    @property
    def K(self) -> int:
        return len(self.symbol)

    def _index(self):
        # (symbol, digit) -> slot and symbol -> base, built once by a scan
        idx = getattr(self, "_idx", None)
        if idx is None:
            slot, base = {}, {}
            for j in range(self.K):
                if self.symbol[j] is None:
                    continue
                slot[(self.symbol[j], self.digit[j])] = j
                base[self.symbol[j]] = self.base[j]
            idx = self._idx = (slot, base)
        return idx

    def slot_of(self, sym, dig: int) -> int:
        return self._index()[0][(sym, dig)]

    def base_of(self, sym) -> int:
        return self._index()[1][sym]

    @staticmethod
    def from_multiplicities(mult: Sequence[Tuple[object, int]]) -> "Tables":
        """Symbols in the given order, each on consecutive slots, digits
        numbered consecutively, base = multiplicity (Sec. III-D)."""
        sym, dig, base = [], [], []
        for s, m in mult:
            for t in range(m):
                sym.append(s)
                dig.append(t)
                base.append(m)
        return Tables(sym, dig, base)


def paper_example_tables() -> Tables:
    """The tables of the tANS example (Fig. 3 is an image; reconstructed from
    the text of Sec. III-D/E): a on slot 0; b on slots 1-4 with digits 0-3 and
    base 4; c on slots 5-7 with digits 0-2 and base 3.  Every number in the
    text (slot 0 for a, slot 1 for (b, digit 0), slot 7 -> (c, 2_3), P' =
    (1/8, 4/8, 3/8)) is consistent with this layout."""
    return Tables.from_multiplicities([("a", 1), ("b", 4), ("c", 3)])


# --------------------------------------------------------------------------
# entropy and cross entropy (Eq. 1 and Eq. 2)
# --------------------------------------------------------------------------
def entropy(counts: Dict[object, int]) -> float:
    n = sum(counts.values())
    return -sum(c / n * math.log2(c / n) for c in counts.values() if c)


def cross_entropy(counts: Dict[object, int], q: Dict[object, Fraction]) -> float:
    n = sum(counts.values())
    return -sum(c / n * math.log2(float(q[s])) for s, c in counts.items() if c)


# --------------------------------------------------------------------------
# tANS (Alg. 1 and Alg. 2)
# --------------------------------------------------------------------------
def _bits(value: int, k: int) -> str:
    return format(value, "0%db" % k) if k else ""


def tans_encode_step(s: int, u, tab: Tables, L: int) -> Tuple[int, str]:
    """One step of Alg. 1: s = x_inf b_2 d_r  ->  s' = x_inf j_K."""
    K = tab.K
    r = tab.base_of(u)
    d = s % r
    j = tab.slot_of(u, d)
    q = s // r  # = x * 2^k + b
    k = 0
    while not (L <= (q >> k) * K + j <= 2 * L - 1):
        k += 1
        if (q >> k) == 0:
            raise ValueError("no renormalisation found")
    x, b = q >> k, q & ((1 << k) - 1)
    return x * K + j, _bits(b, k)


def tans_encode(u: Sequence, tab: Tables, L: int):
    """Alg. 1: encode from right to left starting in state L.  Returns the
    final state s_0, the bit strings v_0..v_{n-1} and the states s_0..s_n."""
    n = len(u)
    s = L
    states = [None] * (n + 1)
    states[n] = s
    v = [None] * n
    for i in range(n - 1, -1, -1):
        s, v[i] = tans_encode_step(s, u[i], tab, L)
        states[i] = s
    return s, v, states


def tans_decode(s0: int, v: Sequence[str], tab: Tables, L: int, n: int):
    """Alg. 2: decode left to right.  Step i reads the bit string v_i; its
    length is the one that brings the state back into [L, 2L-1]."""
    K = tab.K
    s = s0
    bitstream = "".join(v)
    pos = 0
    out, states = [], [s0]
    for _ in range(n):
        j = s % K
        d, r, sym = tab.digit[j], tab.base[j], tab.symbol[j]
        x = s // K
        for k in range(0, 64):
            b = int(bitstream[pos:pos + k], 2) if k else 0
            cand = (x * (1 << k) + b) * r + d
            if L <= cand <= 2 * L - 1 and pos + k <= len(bitstream):
                # the encoder chose the k for which x = q >> k; that is the k
                # where (x*2^k + b) keeps x as its leading part
                if ((x * (1 << k) + b) >> k) == x:
                    break
        else:
            raise ValueError("tANS decode: no valid bit length")
        pos += k
        s = cand
        out.append(sym)
        states.append(s)
    return out, states, pos


# --------------------------------------------------------------------------
# dtANS (Sec. IV-C..F, Alg. 3)
# --------------------------------------------------------------------------
@dataclass(frozen=True)
class Params:
    W: int  # radix of a stream word
    K: int  # slots per table
    M: int  # multiplicity cap (largest base)
    l: int  # symbols per segment
    o: int  # words unpacked per segment
    f: int  # conditional checks per segment

    def check(self) -> None:
        # unpack is a bijection between o words and l slots (Sec. IV-D)
        assert self.K ** self.l == self.W ** self.o, "K^l must equal W^o"
        # every returned digit can replace a conditional load (Sec. IV-D)
        assert self.M ** self.l <= self.W ** self.f, "M^l must be <= W^f"
        assert self.f <= self.o and self.l % self.f == 0

    @property
    def group(self) -> int:
        return self.l // self.f


PAPER_TOY = Params(W=4, K=8, M=4, l=2, o=3, f=2)
CSR_DTANS = Params(W=2 ** 32, K=2 ** 12, M=2 ** 8, l=8, o=3, f=2)


def unpack(words: Sequence[int], p: Params) -> List[int]:
    """i_l ... i_1 (base K) = w_1 ... w_o (base W)."""
    V = 0
    for w in words:
        assert 0 <= w < p.W
        V = V * p.W + w
    slots = []
    for _ in range(p.l):
        slots.append(V % p.K)
        V //= p.K
    return slots


def pack(slots: Sequence[int], p: Params) -> List[int]:
    V = 0
    for i in reversed(slots):
        assert 0 <= i < p.K
        V = V * p.K + i
    words = []
    for _ in range(p.o):
        words.append(V % p.W)
        V //= p.W
    return words[::-1]


def _tab(tab, t: int) -> Tables:
    """Table for segment position t: a single table, or alternating tables
    (CSR-dtANS interleaves a delta table and a value table, Sec. IV-B)."""
    if isinstance(tab, Tables):
        return tab
    return tab[t % len(tab)]


class Stream:
    def __init__(self, words: Sequence[int]):
        self.words = list(words)
        self.pos = 0

    def read(self) -> int:
        w = self.words[self.pos]
        self.pos += 1
        return w


def dtans_decode(v: Sequence[int], tab: Tables, n: int, p: Params,
                 skip_tail: bool = True, order: str = "grouped", trace=None):
    """Alg. 3.  ``n`` symbols, n a multiple of l.  With ``skip_tail`` the last
    segment performs no checks and no loads (Sec. IV-F).  ``trace``, if a
    list, receives one dict per check with the state before and after."""
    p.check()
    assert n % p.l == 0
    st = Stream(v)
    w = [st.read() for _ in range(p.o)]
    d, r = 0, 1
    out = []
    nseg = n // p.l
    for j in range(nseg):
        slots = unpack(w, p)
        last = (j == nseg - 1)
        if last and skip_tail:
            out.extend(_tab(tab, t).symbol[i] for t, i in enumerate(slots))
            break
        new_w = list(w)
        if order == "grouped":
            for g in range(p.f):
                for t in range(g * p.group, (g + 1) * p.group):
                    T, i = _tab(tab, t), slots[t]
                    out.append(T.symbol[i])
                    d = d * T.base[i] + T.digit[i]
                    r = r * T.base[i]
                d, r, new_w[g] = _check(d, r, st, p, trace, j, g)
        elif order == "after_all":
            for t, i in enumerate(slots):
                T = _tab(tab, t)
                out.append(T.symbol[i])
                d = d * T.base[i] + T.digit[i]
                r = r * T.base[i]
            for g in range(p.f):
                d, r, new_w[g] = _check(d, r, st, p, trace, j, g)
        else:
            raise ValueError(order)
        for k in range(p.f, p.o):
            new_w[k] = st.read()
        w = new_w
    return out, st.pos


def _check(d, r, st, p, trace, j, g):
    before = (d, r)
    if r >= p.W:
        wk = d % p.W
        d, r = d // p.W, r // p.W
        kind = "extract"
    else:
        wk = st.read()
        kind = "load"
    if trace is not None:
        trace.append(dict(segment=j, check=g + 1, kind=kind, before=before,
                          after=(d, r), word=wk))
    return d, r, wk


def dtans_base_pass(u: Sequence, tab: Tables, p: Params,
                    skip_tail: bool = True) -> List[List[bool]]:
    """Forward pass over the bases only (Sec. IV-E): flags[j][g] is True when
    check g of segment j extracts a word from the state (r >= W) and False
    when it loads one from the stream."""
    nseg = len(u) // p.l
    r = 1
    flags = []
    for j in range(nseg):
        if j == nseg - 1 and skip_tail:
            break
        fj = []
        for g in range(p.f):
            for t in range(g * p.group, (g + 1) * p.group):
                r *= _tab(tab, t).base_of(u[j * p.l + t])
            if r >= p.W:
                fj.append(True)
                r //= p.W
            else:
                fj.append(False)
        flags.append(fj)
    return flags


def dtans_encode(u: Sequence, tab: Tables, p: Params, skip_tail: bool = True,
                 final_digit: int = 0) -> List[int]:
    """Backward digit pass (Sec. IV-E).  Walks the decoder's steps in reverse
    order, un-appending digits, choosing the slot that carries each digit and
    emitting the stream words the decoder will load.  The decoder's state
    after its last step is taken as 0, and the words it would hold after the
    last segment are 0 (they are never stored: Sec. IV-F)."""
    p.check()
    assert len(u) % p.l == 0 and len(u) > 0
    nseg = len(u) // p.l
    flags = dtans_base_pass(u, tab, p, skip_tail)
    rev: List[int] = []  # emitted words in reverse stream order
    d = 0
    if skip_tail:
        # the last segment appends nothing: its digits are free; take 0
        slots = [_tab(tab, t).slot_of(s, final_digit)
                 for t, s in enumerate(u[(nseg - 1) * p.l:])]
        first_checked = nseg - 2
    else:
        slots = None
        first_checked = nseg - 1
    for j in range(first_checked, -1, -1):
        nxt = pack(slots, p) if slots is not None else [0] * p.o
        for k in range(p.o - 1, p.f - 1, -1):
            rev.append(nxt[k])  # unconditional loads
        seg_syms = u[j * p.l:(j + 1) * p.l]
        seg_slots = [None] * p.l
        for g in range(p.f - 1, -1, -1):
            if flags[j][g]:
                d = d * p.W + nxt[g]
            else:
                rev.append(nxt[g])
            for t in range((g + 1) * p.group - 1, g * p.group - 1, -1):
                T = _tab(tab, t)
                b = T.base_of(seg_syms[t])
                dig = d % b
                d //= b
                seg_slots[t] = T.slot_of(seg_syms[t], dig)
        slots = seg_slots
    assert d == 0, "digit pass must end in the initial state"
    first = pack(slots, p)
    return first + rev[::-1]


def dtans_word_count(u: Sequence, tab: Tables, p: Params,
                     skip_tail: bool = True) -> int:
    flags = dtans_base_pass(u, tab, p, skip_tail)
    return p.o + sum(p.o - p.f + sum(1 for x in fj if not x) for fj in flags)
