"""Pins of the oracle's Bounded Integer Sequence Encoding (Sec. 3.3; C9-C11).

* bit counts against ASTC's published closed forms (S*m, S*m + ceil(8S/5),
  S*m + ceil(7S/3));
* hand-derived known-answer words (tests/golden/bise_vectors.txt);
* brute force over every trit 5-tuple and every quint 3-tuple with
  m = 0..6, round trip, digit-field bounds and injectivity;
* zigzag bijection and the quantiser's error bound.
"""
import math
import os

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "bise_vectors.txt")


def bits_of(words, nbits, start=0):
    """The bit string start..start+nbits-1 as a python int (LSB = first bit)."""
    w = [int(x) for x in words]
    acc = sum(v << (32 * i) for i, v in enumerate(w))
    return (acc >> start) & ((1 << nbits) - 1)


@pytest.mark.parametrize("S", list(range(1, 65)))
def test_bit_counts_closed_form(S):
    for code in range(26):
        kind, m, n = oracle.bise_range(code)
        expect = S * m + {"bits": 0, "trit": math.ceil(8 * S / 5), "quint": math.ceil(7 * S / 3)}[kind]
        assert oracle.bise_bits(code, S) == expect
        assert n == {"bits": 2 ** m, "trit": 3 * 2 ** m, "quint": 5 * 2 ** m}[kind]


def test_range_table():
    assert [oracle.bise_range(k)[2] for k in range(12)] == [2 ** m for m in range(1, 13)]
    assert [oracle.bise_range(k)[2] for k in range(12, 19)] == [3 * 2 ** m for m in range(7)]
    assert [oracle.bise_range(k)[2] for k in range(19, 26)] == [5 * 2 ** m for m in range(7)]
    with pytest.raises(oracle.OracleError):
        oracle.bise_range(26)


@pytest.mark.parametrize("S", [4, 16, 64])
def test_cost_strictly_increasing_in_range(S):
    # the encoder picks the smallest range that fits; for block sizes 2, 4, 8
    # that is also the cheapest choice because cost grows with N
    by_n = sorted((oracle.bise_range(k)[2], oracle.bise_bits(k, S)) for k in range(26))
    costs = [c for _, c in by_n]
    assert all(a < b for a, b in zip(costs, costs[1:]))


def test_known_answer_vectors():
    rows = [l for l in open(GOLDEN) if l.strip() and not l.startswith("#")]
    assert len(rows) == 6
    for row in rows:
        code, pos, vals, words, nbits = [f.strip() for f in row.split("|")]
        code, pos, nbits = int(code), int(pos), int(nbits)
        vals = [int(v) for v in vals.split()]
        expect = [int(w, 16) for w in words.split()]
        assert oracle.bise_bits(code, len(vals)) == nbits
        got = oracle.bise_encode(vals, code, bitpos=pos)
        first = pos // 32
        assert [int(x) for x in got[first:first + len(expect)]] == expect, row
        assert not np.any(got[first + len(expect):]), row
        assert list(oracle.bise_decode(got, len(vals), code, bitpos=pos)) == vals


def _brute(kind_codes, radix, glen):
    rng = np.random.default_rng(5)
    for code in kind_codes:
        _, m, n = oracle.bise_range(code)
        seen = {}
        for tup in np.ndindex(*([radix] * glen)):
            digits = np.array(tup, dtype=np.int64)
            for lowpat in ("zero", "ones", "rand"):
                if lowpat == "zero":
                    low = np.zeros(glen, dtype=np.int64)
                elif lowpat == "ones":
                    low = np.full(glen, (1 << m) - 1, dtype=np.int64)
                else:
                    low = rng.integers(0, 1 << m, glen) if m else np.zeros(glen, dtype=np.int64)
                vals = (digits << m) | low
                assert vals.max() < n
                words = oracle.bise_encode(vals, code)
                nbits = oracle.bise_bits(code, glen)
                field_bits = nbits - glen * m
                number = bits_of(words, field_bits)
                assert number < radix ** glen
                # the digit field is the base-radix number of the digits
                assert number == sum(int(d) * radix ** r for r, d in enumerate(tup))
                assert bits_of(words, 32 * len(words)) >> nbits == 0
                back = oracle.bise_decode(words, glen, code)
                assert np.array_equal(back.astype(np.int64), vals)
                key = bits_of(words, nbits)
                assert seen.setdefault(key, tuple(vals)) == tuple(vals)


def test_brute_force_all_trit_tuples():
    _brute(range(12, 19), 3, 5)


def test_brute_force_all_quint_tuples():
    _brute(range(19, 26), 5, 3)


@pytest.mark.parametrize("code", [12, 13, 19, 20, 25])
def test_partial_groups_sizes(code):
    kind, m, n = oracle.bise_range(code)
    glen = 5 if kind == "trit" else 3
    part = {1: 2, 2: 4, 3: 5, 4: 7} if kind == "trit" else {1: 3, 2: 5}
    for k, extra in part.items():
        S = glen * 2 + k
        full = 2 * (8 if kind == "trit" else 7)
        assert oracle.bise_bits(code, S) == S * m + full + extra
        vals = np.random.default_rng(k).integers(0, n, S)
        w = oracle.bise_encode(vals, code)
        assert np.array_equal(oracle.bise_decode(w, S, code).astype(np.int64), vals)


def test_decode_rejects_out_of_range_digit_field():
    # a trit field of 243 or more, and a single-trit field of 3, are not valid
    w = np.array([250, 0], dtype=np.uint32)
    with pytest.raises(oracle.OracleError):
        oracle.bise_decode(w, 5, 12)
    w = np.array([3, 0], dtype=np.uint32)
    with pytest.raises(oracle.OracleError):
        oracle.bise_decode(w, 1, 12)


def test_zigzag_bijection():
    vals = list(range(-4096, 4096))
    z = [oracle.zigzag(v) for v in vals]
    assert sorted(z) == list(range(8192))
    assert [oracle.zigzag(v) for v in (0, -1, 1, -2, 2)] == [0, 1, 2, 3, 4]
    assert all(oracle.unzigzag(oracle.zigzag(v)) == v for v in vals)


def test_quantiser_error_bound():
    for q in range(5):
        for r in range(-700, 701):
            qv = oracle.quantize(r, q)
            if q == 0:
                assert qv == r
            else:
                assert abs(qv * (1 << q) - r) <= 1 << (q - 1)
                assert oracle.quantize(-r, q) == -qv
    # exact halves round away from zero
    assert oracle.quantize(2, 2) == 1 and oracle.quantize(-2, 2) == -1
    assert oracle.quantize(1, 2) == 0 and oracle.quantize(6, 2) == 2
