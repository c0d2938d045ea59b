"""Pins of the oracle's toy codec against the numbers the paper prints.

Sec. III-C (mixed radix), III-D/E (tANS example, Alg. 1/2), IV-D (dtANS
example, Alg. 3), IV-E (two-pass encoder) and IV-F (skipped trailing loads).
"""
import json
import os
from fractions import Fraction

import pytest

from oracle import toy


def load(golden_dir, name):
    with open(os.path.join(golden_dir, name)) as f:
        return json.load(f)


def test_mixed_radix_example():
    # Sec. III-C: 10 days, 5 hours, 30 minutes = 10*24*60 + 5*60 + 30.  The
    # text prints the total as 11370; the right-hand side it prints evaluates
    # to 14730, so the printed total is a typo and the formula is what is
    # pinned.  Appending a digit with d <- d*base + digit (the rule the toy
    # decoder uses for Alg. 3) makes the digit appended last the least
    # significant one.
    d = 10  # the infinite-radix (most significant) digit
    for digit, base in ((5, 24), (30, 60)):
        d = d * base + digit
    assert d == 10 * 24 * 60 + 5 * 60 + 30 == 14730
    # and peeling digits off in reverse order recovers them
    assert (d % 60, (d // 60) % 24, d // (60 * 24)) == (30, 5, 10)


def test_tans_tables_and_entropies(golden_dir):
    g = load(golden_dir, "tans_example.json")
    tab = toy.Tables.from_multiplicities([tuple(x) for x in g["multiplicities"]])
    assert tab.K == g["K"]
    counts = {s: g["u"].count(s) for s in "abc"}
    assert toy.entropy(counts) == pytest.approx(g["entropy_H"], abs=5e-4)
    q = {s: Fraction(tab.base_of(s), tab.K) for s in "abc"}
    assert q == {"a": Fraction(1, 8), "b": Fraction(4, 8), "c": Fraction(3, 8)}
    assert toy.cross_entropy(counts, q) == pytest.approx(g["cross_entropy_Hprime"], abs=5e-4)
    q2 = {s: Fraction(v).limit_denominator() for s, v in g["Pdoubleprime"].items()}
    assert toy.cross_entropy(counts, q2) == pytest.approx(g["cross_entropy_Pdoubleprime"], abs=1e-12)
    # slot numbers quoted in the text
    assert tab.slot_of("a", 0) == 0 and tab.slot_of("b", 0) == 1
    assert (tab.symbol[7], tab.digit[7], tab.base[7]) == ("c", 2, 3)


def test_tans_example_states(golden_dir):
    g = load(golden_dir, "tans_example.json")
    tab = toy.Tables.from_multiplicities([tuple(x) for x in g["multiplicities"]])
    s0, v, states = toy.tans_encode(g["u"], tab, g["L"])
    assert states[10] == g["s10"]
    assert states[9] == g["s9"] and v[9] == g["v9"]
    assert states[8] == g["s8"] and v[8] == g["v8"]
    assert states[1] == g["s1"]
    assert s0 == g["s0"]
    assert sum(len(b) for b in v) == g["total_bits"]
    # every printed chunk except v_4 (bit order garbled in the text)
    for i, b in enumerate(g["printed_v"]):
        if i != 4:
            assert v[i] == b
    assert sorted(v[4]) == sorted(g["printed_v"][4])
    out, dstates, used = toy.tans_decode(s0, v, tab, g["L"], len(g["u"]))
    assert out == g["u"] and dstates == states and used == g["total_bits"]


def test_dtans_parameters_closed_forms():
    # Sec. IV-D: K^l = W^o (3 words <-> 8 slots) and M^l = W^f
    p = toy.CSR_DTANS
    assert p.K ** p.l == p.W ** p.o == 2 ** 96
    assert p.M ** p.l == p.W ** p.f == 2 ** 64
    toy.PAPER_TOY.check()
    assert 8 ** 2 == 4 ** 3


def test_dtans_example_unpack(golden_dir):
    g = load(golden_dir, "dtans_example.json")
    p = toy.Params(g["W"], g["K"], g["M"], g["l"], g["o"], g["f"])
    w = g["first_unpack_words"]
    assert w[0] * 16 + w[1] * 4 + w[2] == g["first_unpack_value"]
    assert toy.unpack(w, p) == g["first_unpack_slots"]
    assert toy.pack(g["first_unpack_slots"], p) == w
    tab = toy.paper_example_tables()
    pairs = [[tab.digit[i], tab.base[i]] for i in g["first_unpack_slots"]]
    assert pairs == g["first_returned_pairs"]


def test_dtans_example_decode_trace(golden_dir):
    g = load(golden_dir, "dtans_example.json")
    p = toy.Params(g["W"], g["K"], g["M"], g["l"], g["o"], g["f"])
    tab = toy.paper_example_tables()
    trace = []
    out, used = toy.dtans_decode(g["v"], tab, len(g["u"]), p, skip_tail=False, trace=trace)
    assert out == g["u"]
    assert used == len(g["v"])
    c1, c2 = trace[0], trace[1]
    assert list(c1["before"]) == g["first_check"]["state_before"]
    assert c1["kind"] == g["first_check"]["kind"] and c1["word"] == g["first_check"]["word"]
    assert list(c2["before"]) == g["second_check"]["state_before"]
    assert c2["kind"] == g["second_check"]["kind"] and c2["word"] == g["second_check"]["word"]
    assert list(c2["after"]) == g["second_check"]["state_after"]
    # the unconditional load is the next stream word after the first
    # conditional load: v = 1,1,1 | 2 (load) | 3 (unconditional)
    assert g["v"][4] == g["first_unconditional_word"]
    # invariants of every check: 0 <= d < r, r < W afterwards
    for t in trace:
        d, r = t["after"]
        assert 0 <= d < r < p.W
        d0, r0 = t["before"]
        assert 0 <= d0 < r0 < p.W * p.M ** (p.l // p.f)


def test_dtans_example_literal_order_differs(golden_dir):
    """Alg. 3 as printed (all digits, then the checks) does not reproduce the
    worked example; checking after each digit group does (reading used by
    the oracle and the library)."""
    g = load(golden_dir, "dtans_example.json")
    p = toy.PAPER_TOY
    tab = toy.paper_example_tables()
    out, _ = toy.dtans_decode(g["v"], tab, len(g["u"]), p, skip_tail=False, order="after_all")
    assert out != g["u"]
    assert "".join(out) == "cbbbbcbacb"


def test_dtans_example_encode(golden_dir):
    g = load(golden_dir, "dtans_example.json")
    p = toy.PAPER_TOY
    tab = toy.paper_example_tables()
    assert toy.dtans_encode(g["u"], tab, p, skip_tail=False) == g["v"]
    # Sec. IV-F: with the length known, the known-zero trailing loads are
    # skipped: the same stream minus the words after the last segment
    short = toy.dtans_encode(g["u"], tab, p, skip_tail=True)
    assert short == g["v"][:9]
    out, used = toy.dtans_decode(short, tab, len(g["u"]), p, skip_tail=True)
    assert out == g["u"] and used == 9


def test_base_pass_matches_decoder(golden_dir):
    g = load(golden_dir, "dtans_example.json")
    p = toy.PAPER_TOY
    tab = toy.paper_example_tables()
    flags = toy.dtans_base_pass(g["u"], tab, p, skip_tail=False)
    trace = []
    toy.dtans_decode(g["v"], tab, len(g["u"]), p, skip_tail=False, trace=trace)
    assert [t["kind"] == "extract" for t in trace] == [x for fj in flags for x in fj]
    assert toy.dtans_word_count(g["u"], tab, p, skip_tail=False) == len(g["v"])
