"""Predictive negabinary bitplane coding (oracle).

Sec. 4.4.2: signed codes are written in base -2 (negabinary), so small values of
either sign keep their high digits zero (the paper's 8-bit example: 1 is
00000001 and -1 is 00000011).
Sec. 4.4.1: each bit is XORed with the two next-more-significant bits of the
same code before it is stored; the two prefix bits are already known to a
decoder that loads planes from the top.
Sec. 4.3 / Fig. "overwrite": the 32 bits of the codes of one group form 32
bitplanes that are stored independently, most significant first.
Thm. 1: delta-y, the information lost by not loading the low planes, is
computed once at compression time; here it is the exact max over the pass of
|q - q'_b|, q'_b being the code rebuilt from planes b..31, in code units.

Readings used:
* 32-bit negabinary through the mask identity v = (q + A) xor A with
  A = 0xAAAAAAAA (mod 2^32); bits above bit 31 are zero for the XOR prefix.
* Discarded digits are read back as zero (no mid-point bias).
"""

from __future__ import annotations

import numpy as np

NB_MASK = np.uint32(0xAAAAAAAA)
U32 = np.uint32


def to_negabinary(q) -> np.ndarray:
    """Signed codes -> 32-digit negabinary words (uint32)."""
    q = np.asarray(q, dtype=np.int64)
    v = (q.astype(np.uint64) + np.uint64(0xAAAAAAAA)) & np.uint64(0xFFFFFFFF)
    return (v.astype(U32) ^ NB_MASK).astype(U32)


def from_negabinary(v) -> np.ndarray:
    """32-digit negabinary words -> signed codes (int64)."""
    v = np.asarray(v, dtype=U32)
    w = (v ^ NB_MASK).astype(np.int64)
    return w - 0xAAAAAAAA


def xor_encode(v) -> np.ndarray:
    """e = v xor (v >> 1) xor (v >> 2): each bit predicted from its 2 prefix bits."""
    v = np.asarray(v, dtype=U32)
    return (v ^ (v >> U32(1)) ^ (v >> U32(2))).astype(U32)


def xor_decode(e) -> np.ndarray:
    """Inverse of :func:`xor_encode`, recovering bits from the top down."""
    e = np.asarray(e, dtype=U32)
    v = np.zeros_like(e)
    # v_k = e_k ^ v_{k+1} ^ v_{k+2}, with v_32 = v_33 = 0
    for k in range(31, -1, -1):
        ek = (e >> U32(k)) & U32(1)
        v1 = (v >> U32(k + 1)) & U32(1) if k + 1 < 32 else np.zeros_like(e)
        v2 = (v >> U32(k + 2)) & U32(1) if k + 2 < 32 else np.zeros_like(e)
        v |= ((ek ^ v1 ^ v2) & U32(1)) << U32(k)
    return v


def keep_mask(b: int) -> np.uint32:
    """Digits b..31 kept, 0..b-1 discarded."""
    if b >= 32:
        return U32(0)
    return U32((0xFFFFFFFF << b) & 0xFFFFFFFF)


def truncated_codes(e, b: int) -> np.ndarray:
    """Codes rebuilt from the stored (XOR-coded) planes b..31 only."""
    e = np.asarray(e, dtype=U32)
    m = keep_mask(b)
    v = xor_decode(e & m) & m
    return from_negabinary(v)


def errq_table(q) -> np.ndarray:
    """delta-y per number of discarded planes b = 0..32, in code units."""
    q = np.asarray(q, dtype=np.int64)
    out = np.zeros(33, dtype=np.uint32)
    if q.size == 0:
        return out
    v = to_negabinary(q)
    for b in range(33):
        qb = from_negabinary(v & keep_mask(b))
        out[b] = np.uint32(np.max(np.abs(q - qb)))
    return out


def errq_bound_table() -> np.ndarray:
    """delta-y fixed before compression (the bound reading of Thm. 1): for
    b = 0..32 discarded digits, the largest |value| the b low negabinary
    digits can take, which Sec. 4.4.2's Eq. uncertainty gives as
    2/3 2^b - 1/3 (b odd) and 2/3 2^b - 2/3 (b even).  Written here as the
    larger of the two digit sums (even positions carry +2^k, odd ones -2^k),
    so the formula is checked against it rather than restated."""
    out = np.zeros(33, dtype=np.uint32)
    for b in range(33):
        pos = sum(1 << k for k in range(0, b, 2))
        neg = sum(1 << k for k in range(1, b, 2))
        out[b] = np.uint32(max(pos, neg))
    return out


def pack_planes(e_chunk: np.ndarray) -> np.ndarray:
    """Bitplanes of one chunk: array [32, W] of uint32, W = ceil(n / 32).

    Plane k, word w, bit j holds bit k of code 32 w + j; padding bits are 0.
    """
    e_chunk = np.asarray(e_chunk, dtype=U32)
    n = e_chunk.size
    W = -(-n // 32)
    padded = np.zeros(W * 32, dtype=U32)
    padded[:n] = e_chunk
    rows = padded.reshape(W, 32)
    shifts = np.arange(32, dtype=U32)
    planes = np.zeros((32, W), dtype=U32)
    for k in range(32):
        bits = ((rows >> U32(k)) & U32(1)).astype(np.uint64) << shifts.astype(np.uint64)
        planes[k] = bits.sum(axis=1).astype(U32)
    return planes


def unpack_planes(planes: np.ndarray, n: int) -> np.ndarray:
    """Inverse of :func:`pack_planes` (absent planes given as zero rows)."""
    planes = np.asarray(planes, dtype=U32)
    W = planes.shape[1]
    j = np.arange(32, dtype=U32)
    e = np.zeros((W, 32), dtype=U32)
    for k in range(32):
        bits = (planes[k][:, None] >> j[None, :]) & U32(1)
        e |= bits << U32(k)
    return e.reshape(-1)[:n]
