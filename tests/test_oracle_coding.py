"""Pins of the oracle's coding layer (not gpu).

Negabinary (Sec. 4.4.2), the 2-prefix-bit XOR code (Sec. 4.4.1), truncation
uncertainty (Sec. 4.4.2, Eq. uncertainty), bitplane packing (Sec. 4.3) and the
delta-y table (Thm. 1), each checked against the paper's printed values or an
independent construction.
"""

import json
import os

import numpy as np
import pytest

from oracle import coding
from oracle.brute import negabinary_digits, planes_brute

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_examples.json")))


def test_negabinary_paper_8bit_example():
    for case in GOLDEN["negabinary_8bit"]["cases"]:
        v = int(coding.to_negabinary(np.array([case["value"]]))[0])
        assert format(v & 0xFF, "08b") == case["negabinary"]
        assert v >> 8 == 0
        # the other two encodings of the same sentence, as a sanity check of the fixture
        assert format(case["value"] & 0xFF, "08b") == case["twos_complement"]
        sm = (0x80 if case["value"] < 0 else 0) | abs(case["value"])
        assert format(sm, "08b") == case["sign_magnitude"]


def test_negabinary_equals_division_by_minus_two():
    rng = np.random.default_rng(0)
    qs = np.concatenate([np.arange(-70000, 70001, 7), rng.integers(-2**30, 2**30, 2000),
                         [2**30, -2**30, 1431655765, -2863311530 + 1]])
    v = coding.to_negabinary(qs)
    for q, w in zip(qs.tolist(), v.tolist()):
        d = negabinary_digits(int(q))
        assert w == sum(bit << k for k, bit in enumerate(d)), q
    assert np.array_equal(coding.from_negabinary(v), qs)


def test_negabinary_extreme_range():
    # 32 digits cover [-0xAAAAAAAA, 0x55555555]
    ends = np.array([-0xAAAAAAAA, 0x55555555])
    assert np.array_equal(coding.from_negabinary(coding.to_negabinary(ends)), ends)


def test_xor_code_inverse_and_prefix_property():
    rng = np.random.default_rng(1)
    v = rng.integers(0, 2**32, 200000, dtype=np.uint64).astype(np.uint32)
    e = coding.xor_encode(v)
    assert np.array_equal(coding.xor_decode(e), v)
    # bit k of e is bit k of v xor its two more-significant bits (Sec. 4.4.1)
    for k in (0, 5, 29, 30, 31):
        vk = (v >> k) & 1
        v1 = (v >> (k + 1)) & 1 if k < 31 else 0
        v2 = (v >> (k + 2)) & 1 if k < 30 else 0
        assert np.array_equal((e >> k) & 1, vk ^ v1 ^ v2)
    # a decoder that has planes b..31 recovers digits b..31 exactly
    for b in range(33):
        m = coding.keep_mask(b)
        assert np.array_equal(coding.xor_decode(e & m) & m, v & m)


def _brute_max_low(d):
    best_nb = 0
    for pattern in range(1 << d):
        val = sum(((pattern >> k) & 1) * (-2) ** k for k in range(d))
        best_nb = max(best_nb, abs(val))
    return best_nb


@pytest.mark.parametrize("d", list(range(1, 15)))
def test_truncation_uncertainty_matches_paper(d):
    g = GOLDEN["truncation_uncertainty"]
    form = g["negabinary_odd"] if d % 2 else g["negabinary_even"]
    paper = form["a"] * 2 ** d + form["b"]
    assert _brute_max_low(d) == round(paper)
    sm = g["sign_magnitude"]["a"] * 2 ** d + g["sign_magnitude"]["b"]
    assert (1 << d) - 1 == round(sm)
    # and the oracle's delta-y of a code set covering every d-digit pattern
    qs = np.array([sum(((p >> k) & 1) * (-2) ** k for k in range(d)) for p in range(1 << d)])
    assert int(coding.errq_table(qs)[d]) == round(paper)


def test_pack_planes_matches_packbits_and_bitwise():
    rng = np.random.default_rng(2)
    for n in (1, 31, 32, 33, 100, 1000):
        e = rng.integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)
        planes = coding.pack_planes(e)
        W = -(-n // 32)
        assert planes.shape == (32, W)
        bits = ((e[:, None] >> np.arange(32, dtype=np.uint32)[None, :]) & 1).astype(np.uint8)
        padded = np.zeros((W * 32, 32), dtype=np.uint8)
        padded[:n] = bits
        for k in range(32):
            pk = np.packbits(padded[:, k].reshape(W, 32), axis=1, bitorder="little")
            words = pk.view("<u4").reshape(W)
            assert np.array_equal(words, planes[k])
        if n <= 100:
            assert np.array_equal(np.array(planes_brute(e.tolist())), planes)
        assert np.array_equal(coding.unpack_planes(planes, n), e)


def test_errq_brute_and_invariants():
    rng = np.random.default_rng(3)
    for trial in range(20):
        scale = [3, 100, 5000, 2**20][trial % 4]
        q = rng.integers(-scale, scale + 1, rng.integers(1, 300))
        t = coding.errq_table(q)
        e = coding.xor_encode(coding.to_negabinary(q))
        for b in range(33):
            qb = coding.truncated_codes(e, b)
            assert int(t[b]) == int(np.max(np.abs(q - qb)))
        assert t[0] == 0
        assert int(t[32]) == int(np.max(np.abs(q)))
        # the loss of b discarded digits never exceeds the b-digit uncertainty
        for b in range(33):
            assert int(t[b]) <= ((1 << (b + 1)) - 1) // 3
    assert np.array_equal(coding.errq_table(np.zeros(0, dtype=np.int64)), np.zeros(33))


def test_errq_bound_table_is_the_paper_uncertainty():
    """The bound form of delta-y (IPC_ERRQ_BOUND) is Sec. 4.4.2's Eq.
    uncertainty for every number of discarded digits, and a code set holding
    every b-digit pattern attains it (so it is the least bound)."""
    g = GOLDEN["truncation_uncertainty"]
    t = coding.errq_bound_table()
    assert t[0] == 0
    for b in range(1, 33):
        form = g["negabinary_odd"] if b % 2 else g["negabinary_even"]
        assert int(t[b]) == round(form["a"] * 2 ** b + form["b"]), b
    for b in range(1, 12):
        qs = np.array([sum(((p >> k) & 1) * (-2) ** k for k in range(b)) for p in range(1 << b)])
        assert int(coding.errq_table(qs)[b]) == int(t[b])


def test_errq_bound_table_dominates_measured_tables():
    rng = np.random.default_rng(5)
    t = coding.errq_bound_table().astype(np.int64)
    for hi in (3, 100, 5000, 1 << 20, (1 << 30) - 1):
        q = rng.integers(-hi, hi + 1, 2000)
        m = coding.errq_table(q).astype(np.int64)
        assert np.all(m <= t), hi
