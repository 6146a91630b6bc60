"""Pins of the oracle's entropy stage for stored bitplanes (CPU).

The coder's bytes are pinned by hand-worked cases (the interval arithmetic
done on paper from the coder's definition), by decoding (any dropped term or
wrong branch breaks the round trip), and by the code length staying within a
few bytes of the model's ideal length (sum of -log2 of the probabilities,
computed without the coder).  The stage is lossless, so every retrieval from a
coded stream must equal the retrieval from the raw stream with the same plan,
and the planner must charge each plane exactly what the coded stream stores.
"""

import numpy as np
import pytest

import fieldgen
from oracle import codec, entropy, planner
from oracle.stream import (CODING_ENTROPY, StreamError, entropy_code_stream, parse_stream,
                           stream_chunk_counts)


# (bits, bytes) worked by hand:
#  [1]: bound = (2^32-1 >> 12) * 2048 = 0x7FFFF800 -> low = 0x7FFFF800, range
#       0x800007FF; the one-byte value 0x80000000 lies inside.
#  [1, 1]: p0 = 1920, bound = 0x80000 * 1920 = 0x3C000000 -> low 0xBBFFF800,
#       range 0x440007FF; 0xBC000000 lies inside.
#  [0, 1]: range 0x7FFFF800, p0 = 2176, bound = 0x7FFFF * 2176 = 0x43FFF780 ->
#       low 0x43FFF780, range 0x3C000080; 0x44000000 lies inside.
#  zeros only: low stays 0, every output byte is zero and is dropped.
HAND = [([], b""), ([0], b""), ([1], b"\x80"), ([1, 1], b"\xbc"), ([0, 1], b"\x44"),
        ([0] * 4096, b"")]


@pytest.mark.parametrize("bits,expected", HAND, ids=range(len(HAND)))
def test_hand_worked_codes(bits, expected):
    assert entropy.encode_bits(bits) == expected
    assert np.array_equal(entropy.decode_bits(expected, len(bits)), np.array(bits, dtype=np.uint8))


@pytest.mark.parametrize("n", [1, 31, 32, 33, 1000, 4096])
@pytest.mark.parametrize("density", [0.0005, 0.03, 0.3, 0.5, 0.9, 0.999])
def test_round_trip_and_length(n, density):
    rng = np.random.default_rng(int(n * 1000 + density * 1e4))
    bits = (rng.random(n) < density).astype(np.uint8)
    data = entropy.encode_bits(bits)
    assert np.array_equal(entropy.decode_bits(data, n), bits)
    ideal = entropy.ideal_cost_bits(bits)
    # truncating bound loses at most 2^-11 bits per bit; the end adds <= 1 byte
    assert len(data) <= (ideal + n * 2.0 ** -11) / 8 + 2
    assert len(data) >= ideal / 8 - 5


def test_carry_propagation():
    """Runs that push low past 2^32 after 0xFF bytes were output: the round
    trip holds only if the carry reaches the bytes already written."""
    rng = np.random.default_rng(7)
    stats = {}
    for t in range(300):
        bits = (rng.random(600) < rng.uniform(0.5, 0.999)).astype(np.uint8)
        data = entropy.encode_bits(bits, stats)
        assert np.array_equal(entropy.decode_bits(data, bits.size), bits)
    assert stats.get("carries", 0) > 10


def test_block_stored_raw_when_not_smaller():
    rng = np.random.default_rng(3)
    words = rng.integers(0, 2 ** 32, size=4, dtype=np.uint64).astype(np.uint32)
    stored, nw = entropy.code_block(words, 128)
    assert nw == 4 and np.array_equal(stored, words)
    sparse = np.zeros(100, dtype=np.uint32)
    sparse[[3, 50]] = [1 << 7, 1 << 30]
    stored, nw = entropy.code_block(sparse, 3190)
    assert 0 < nw < 100
    assert np.array_equal(entropy.decode_block(stored, nw, 3190), sparse)


def _coded_pair(x, eb):
    raw = codec.compress(x, eb)
    return raw, entropy_code_stream(raw)


@pytest.fixture(scope="module")
def smooth_pair():
    x = fieldgen.climate_2d(1)[700:760, 1000:1200].copy()
    return x, _coded_pair(x, 1e-3 * fieldgen.value_range(x))


@pytest.fixture(scope="module")
def rough_pair():
    x = fieldgen.grf((20, 24, 70), -5.0 / 6.0, seed=5, dtype=np.float32)
    return x, _coded_pair(x, 1e-5 * fieldgen.value_range(x))


def test_coded_stream_round_trip(smooth_pair, rough_pair):
    for _, (raw, coded) in (smooth_pair, rough_pair):
        pr, pc = parse_stream(raw), parse_stream(coded)
        assert pc.header.coding == CODING_ENTROPY
        assert np.array_equal(pr.payload, pc.payload)
        assert np.array_equal(pr.masks, pc.masks) and np.array_equal(pr.errq, pc.errq)
        assert entropy_code_stream(coded) == coded
        assert len(coded) < len(raw)


def test_coded_tables_charge_stored_words(smooth_pair):
    _, (raw, coded) = smooth_pair
    pc = parse_stream(coded)
    t = planner.tables_from_stream(pc)
    assert int(t.sizes.sum()) == 4 * pc.header.payload_words == 4 * int(pc.block_words.sum())
    assert t.fixed_bytes + int(t.sizes[t.progressive].sum()) == len(coded)
    # per plane: the coded stream never charges more than the raw one
    tr = planner.tables_from_stream(parse_stream(raw))
    assert np.all(t.sizes <= tr.sizes)


@pytest.mark.parametrize("which", ["smooth", "rough"])
def test_coded_retrieval_equals_raw(which, smooth_pair, rough_pair):
    x, (raw, coded) = smooth_pair if which == "smooth" else rough_pair
    _, _, t = codec.open_stream(coded)
    rng = np.random.default_rng(11)
    for trial in range(4):
        plan = [0 if not t.progressive[s] else int(rng.integers(0, 20)) for s in range(t.n_passes)]
        a = codec.retrieve_with_plan(raw, plan)
        b = codec.retrieve_with_plan(coded, plan)
        assert a.field.tobytes() == b.field.tobytes()
        assert b.bytes_read <= a.bytes_read
    # bitrate plans on the coded stream: within budget (counted in coded
    # bytes) and within their reported bound
    for br in (0.5, 1.0, 2.0):
        b = codec.retrieve(coded, "bitrate", br)
        assert planner.loaded_bytes(b.tables, b.plan) <= br * x.size / 8 or b.flags
        err = float(np.max(np.abs(b.field.astype(np.float64) - x)))
        assert err <= b.bound


def test_refine_on_coded_stream(rough_pair):
    x, (raw, coded) = rough_pair
    r = fieldgen.value_range(x)
    st = codec.retrieve(coded, "eb", 1e-2 * r)
    total = st.bytes_read
    for e in (1e-3, 1e-4):
        st = codec.refine(st, "eb", e * r)
        total += st.bytes_read
    fresh = codec.retrieve(coded, "eb", 1e-4 * r)
    assert np.array_equal(st.plan, fresh.plan)
    assert st.field.tobytes() == fresh.field.tobytes()
    assert total == fresh.bytes_read


def test_corrupt_block_lengths_rejected(smooth_pair):
    _, (_, coded) = smooth_pair
    pc = parse_stream(coded)
    off = pc.payload_offset - ((pc.block_words.size + 7) & ~7)
    bad = bytearray(coded)
    bad[off] = 200  # longer than any block can be
    with pytest.raises(StreamError):
        parse_stream(bytes(bad))
    counts = stream_chunk_counts(pc.header)
    assert len(entropy.blocks(pc.masks, counts)) == pc.block_words.size
