"""Entropy stage for stored bitplanes (oracle; test infrastructure only).

The paper hands every independently loadable block to a general-purpose
lossless compressor (zstd) before it is stored (experimental setup, Sec. 6).
This implementation codes each block -- one stored bitplane of one chunk --
with an adaptive binary range coder instead, so that a GPU can code every block
on its own thread and a retrieval still reads only the blocks of its plan.

Coder (a binary arithmetic coder in the range-coder form of Martin, 1979, with
byte output and carry propagation, and the shift-update probability estimate
used by LZMA-style coders):

* The bits of a block are the plane's bits in code order: bit j of the block is
  bit k of code j of the chunk (word j >> 5, bit j & 31 of the raw plane), for
  j = 0 .. count - 1.
* State: a 32-bit ``range`` (initially 2^32 - 1), the interval base ``low`` and
  a 12-bit probability ``p0`` that the next bit is 0 (initially 2048).
* Bit b: ``bound = (range >> 12) * p0``; a 0 keeps ``[low, low + bound)`` and
  raises p0 by ``(4096 - p0) >> 4``; a 1 keeps ``[low + bound, low + range)``
  and lowers p0 by ``p0 >> 4``.  While ``range < 2^24`` the top byte of low is
  output and low and range are shifted left by 8 bits; a carry out of low adds
  one to the bytes already output.
* End: the shortest run of whole bytes whose value, followed by zero bytes,
  lies inside the final interval (at most one byte, since the final range is
  at least 2^24); trailing zero bytes are dropped.
* The decoder mirrors these steps and reads zero bytes past the end.

Stored form: a block whose code takes fewer 32-bit words than the raw plane
(``W = ceil(count / 32)``) is stored coded (bytes little-endian in words, zero
padded); otherwise it is stored raw.  The per-block word count, in payload
order, is a byte array (``W`` means raw), so a loader finds every block with a
prefix sum and the planner charges each plane what it occupies.
"""

from __future__ import annotations

import numpy as np

PROB_BITS = 12
PROB_ONE = 1 << PROB_BITS
ADAPT_SHIFT = 4
TOP = 1 << 24
MASK32 = (1 << 32) - 1


def encode_bits(bits, stats=None) -> bytes:
    """Code a sequence of 0/1 values; returns the coded bytes.  `stats`, a
    dict, receives the number of carries into output bytes."""
    low = 0
    rng = MASK32
    p0 = PROB_ONE // 2
    out = bytearray()

    def carry():
        i = len(out) - 1
        while out[i] == 0xFF:
            out[i] = 0
            i -= 1
        assert i >= 0, "carry past the first byte"
        out[i] += 1
        if stats is not None:
            stats["carries"] = stats.get("carries", 0) + 1

    for b in bits:
        bound = (rng >> PROB_BITS) * p0
        if b:
            low += bound
            rng -= bound
            p0 -= p0 >> ADAPT_SHIFT
        else:
            rng = bound
            p0 += (PROB_ONE - p0) >> ADAPT_SHIFT
        if low > MASK32:
            low -= 1 << 32
            carry()
        while rng < TOP:
            out.append(low >> 24)
            low = (low << 8) & MASK32
            rng <<= 8
    # shortest byte string (then zeros) inside [low, low + range)
    for n in range(5):
        unit = 1 << (8 * (4 - n))
        v = -(-low // unit) * unit
        if v < low + rng:
            break
    if v > MASK32:
        v -= 1 << 32
        carry()
    for i in range(n):
        out.append((v >> (24 - 8 * i)) & 0xFF)
    # the decoder reads zeros past the end: trailing zero bytes carry nothing
    return bytes(out).rstrip(b"\0")


def decode_bits(data: bytes, n: int) -> np.ndarray:
    """The first n bits coded in `data` (uint8 0/1 array)."""
    def byte(i):
        return data[i] if i < len(data) else 0

    code = (byte(0) << 24) | (byte(1) << 16) | (byte(2) << 8) | byte(3)
    pos = 4
    rng = MASK32
    p0 = PROB_ONE // 2
    out = np.zeros(n, dtype=np.uint8)
    for j in range(n):
        bound = (rng >> PROB_BITS) * p0
        if code < bound:
            rng = bound
            p0 += (PROB_ONE - p0) >> ADAPT_SHIFT
        else:
            code -= bound
            rng -= bound
            p0 -= p0 >> ADAPT_SHIFT
            out[j] = 1
        while rng < TOP:
            code = ((code << 8) | byte(pos)) & MASK32
            pos += 1
            rng <<= 8
    return out


def ideal_cost_bits(bits) -> float:
    """Code length in bits that the adaptive model assigns to `bits`:
    the sum of -log2 of the probability of every bit (used by the pins)."""
    p0 = PROB_ONE // 2
    tot = 0.0
    for b in bits:
        pb = (PROB_ONE - p0) if b else p0
        tot -= np.log2(pb / PROB_ONE)
        if b:
            p0 -= p0 >> ADAPT_SHIFT
        else:
            p0 += (PROB_ONE - p0) >> ADAPT_SHIFT
    return tot


def plane_bits(words: np.ndarray, count: int) -> np.ndarray:
    """Bits of a raw plane in code order (bit j = word j >> 5, bit j & 31)."""
    w = np.asarray(words, dtype=np.uint32)
    b = (w[:, None] >> np.arange(32, dtype=np.uint32)) & np.uint32(1)
    return b.reshape(-1)[:count].astype(np.uint8)


def bits_to_words(bits: np.ndarray, W: int) -> np.ndarray:
    padded = np.zeros(32 * W, dtype=np.uint64)
    padded[:bits.size] = bits
    return (padded.reshape(W, 32) << np.arange(32, dtype=np.uint64)).sum(axis=1).astype(np.uint32)


def bytes_to_words(data: bytes) -> np.ndarray:
    pad = (-len(data)) % 4
    return np.frombuffer(data + b"\0" * pad, dtype="<u4").astype(np.uint32)


def words_to_bytes(words: np.ndarray) -> bytes:
    return np.ascontiguousarray(words, dtype="<u4").tobytes()


def code_block(words: np.ndarray, count: int):
    """(stored words, stored word count) of one raw plane block."""
    W = words.size
    data = encode_bits(plane_bits(words, count))
    cw = bytes_to_words(data)
    if cw.size < W:
        return cw, cw.size
    return np.asarray(words, dtype=np.uint32), W


def decode_block(stored: np.ndarray, n_words: int, count: int) -> np.ndarray:
    """The raw plane block (W words) back from its stored form."""
    W = -(-count // 32)
    if n_words == W:
        return np.asarray(stored, dtype=np.uint32).copy()
    return bits_to_words(decode_bits(words_to_bytes(stored), count), W)


def blocks(masks: np.ndarray, chunk_counts):
    """(count, plane) of every stored block in payload order: chunks in
    order, the stored planes of a chunk from 31 down to 0.  `chunk_counts`
    lists the codes of every chunk of the stream, in chunk order."""
    out = []
    for c, n in enumerate(chunk_counts):
        m = int(masks[c])
        for k in range(31, -1, -1):
            if (m >> k) & 1:
                out.append((int(n), k))
    return out


def code_payload(masks: np.ndarray, chunk_counts, payload: np.ndarray):
    """(per-block stored word counts uint8, stored payload uint32)."""
    lens = []
    parts = []
    pos = 0
    for n, _ in blocks(masks, chunk_counts):
        W = -(-n // 32)
        stored, nw = code_block(payload[pos:pos + W], n)
        pos += W
        lens.append(nw)
        parts.append(stored)
    assert pos == payload.size
    stored = np.concatenate(parts).astype(np.uint32) if parts else np.zeros(0, np.uint32)
    return np.asarray(lens, dtype=np.uint8), stored


def decode_payload(masks: np.ndarray, chunk_counts, lens: np.ndarray, stored: np.ndarray):
    """The raw payload back from the stored form."""
    parts = []
    pos = 0
    for i, (n, _) in enumerate(blocks(masks, chunk_counts)):
        nw = int(lens[i])
        parts.append(decode_block(stored[pos:pos + nw], nw, n))
        pos += nw
    if pos != stored.size:
        raise ValueError("block lengths do not cover the payload")
    return np.concatenate(parts).astype(np.uint32) if parts else np.zeros(0, np.uint32)
