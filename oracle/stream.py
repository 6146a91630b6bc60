"""Serialized stream of independently loadable blocks (oracle).

Fig. "overall-design": the compressed data is a set of blocks that can be
decompressed independently; the data loader (Sec. 3.2, Sec. 5) fetches only the
blocks a request needs.  Here a block is one bitplane of one chunk of one pass.

Layout (all little endian; every section is zero-padded to a multiple of 8
bytes):

  header      128 bytes (see HEADER_FMT)
  errq        n_passes x 33 uint32       delta-y table (Thm. 1), code units
  masks       n_chunks uint32            bit k set <=> plane k of the chunk stored
  out_keys    n_outliers x 3 uint32      (pass, chunk, local index), sorted
  out_vals    n_outliers x T             exact values of the outliers
  block_words n_blocks uint8             only in entropy-coded streams: the
                                         stored words of every block
  payload     payload_words uint32       per pass, per chunk (tile order), the
                                         stored planes from 31 down to 0, each
                                         ceil(count / 32) words raw, or its
                                         entropy-coded form (oracle/entropy.py)

Header byte 11 is the coding: 0 raw blocks, 1 entropy-coded blocks.

Everything before the payload plus the planes of non-progressive passes is
always loaded ("fixed bytes").
"""

from __future__ import annotations

import struct
from dataclasses import dataclass

import numpy as np

from . import entropy
from .schedule import make_schedule

MAGIC = 0x4D435049  # bytes "IPCM"
VERSION = 1
HEADER_SIZE = 128
# magic, version, dtype, ndim, interp, coding, nonprog_levels, dims[3], eb,
# K, qmax, chunk_log2[3], reserved, n_passes, n_chunks, n_outliers,
# payload_words, maxabs, reserved[32]
HEADER_FMT = "<IIBBBBI3QdII3BBIQQQd32x"
assert struct.calcsize(HEADER_FMT) == HEADER_SIZE

DTYPES = {0: np.dtype(np.float32), 1: np.dtype(np.float64)}
DTYPE_CODES = {np.dtype(np.float32): 0, np.dtype(np.float64): 1}


def pad8(n: int) -> int:
    return (n + 7) & ~7


@dataclass
class StreamHeader:
    dtype: np.dtype
    ndim: int
    interp: int
    nonprog_levels: int
    dims: tuple
    eb: float
    K: int
    qmax: int
    chunk_log2: tuple
    n_passes: int
    n_chunks: int
    n_outliers: int
    payload_words: int
    maxabs: float
    coding: int = 0


CODING_RAW = 0
CODING_ENTROPY = 1


@dataclass
class ParsedStream:
    header: StreamHeader
    errq: np.ndarray          # [n_passes, 33] uint32
    masks: np.ndarray         # [n_chunks] uint32
    out_keys: np.ndarray      # [n_outliers, 3] uint32
    out_vals: np.ndarray      # [n_outliers] T
    payload: np.ndarray       # raw payload (entropy-coded blocks decoded)
    payload_offset: int       # byte offset of the payload in the stream
    total_bytes: int
    block_words: np.ndarray = None  # stored words per block (coded streams)


def section_sizes(n_passes, n_chunks, n_outliers, itemsize, payload_words, n_blocks=None):
    """Padded section sizes; `n_blocks` is given for entropy-coded streams
    (their block-length section sits before the payload)."""
    s = [HEADER_SIZE, pad8(4 * 33 * n_passes), pad8(4 * n_chunks),
         pad8(12 * n_outliers), pad8(itemsize * n_outliers)]
    if n_blocks is not None:
        s.append(pad8(n_blocks))
    return s + [pad8(4 * payload_words)]


def stream_chunk_counts(h: StreamHeader) -> np.ndarray:
    """Codes of every chunk of the stream, in chunk order."""
    sched = make_schedule(h.dims, h.chunk_log2)
    return np.concatenate([p.chunk_counts for p in sched.passes]).astype(np.int64)


def n_blocks_of(masks: np.ndarray) -> int:
    return int(sum(bin(int(v)).count("1") for v in masks))


def write_stream(h: StreamHeader, errq, masks, out_keys, out_vals, payload,
                 block_words=None) -> bytes:
    """Serialize; with `block_words` the payload is the entropy-coded one."""
    D = h.ndim
    dims3 = tuple(h.dims) + (1,) * (3 - D)
    cl3 = tuple(h.chunk_log2) + (0,) * (3 - D)
    head = struct.pack(HEADER_FMT, MAGIC, VERSION, DTYPE_CODES[np.dtype(h.dtype)], D,
                       h.interp, h.coding, h.nonprog_levels, *dims3, float(h.eb), h.K, h.qmax,
                       *cl3, 0, h.n_passes, h.n_chunks, h.n_outliers, h.payload_words,
                       float(h.maxabs))
    parts = [head]

    def add(arr_bytes: bytes):
        parts.append(arr_bytes + b"\0" * (pad8(len(arr_bytes)) - len(arr_bytes)))

    add(np.ascontiguousarray(errq, dtype="<u4").tobytes())
    add(np.ascontiguousarray(masks, dtype="<u4").tobytes())
    add(np.ascontiguousarray(out_keys, dtype="<u4").reshape(-1).tobytes())
    add(np.ascontiguousarray(out_vals, dtype=np.dtype(h.dtype).newbyteorder("<")).tobytes())
    if h.coding == CODING_ENTROPY:
        add(np.ascontiguousarray(block_words, dtype=np.uint8).tobytes())
    add(np.ascontiguousarray(payload, dtype="<u4").tobytes())
    return b"".join(parts)


class StreamError(ValueError):
    pass


def parse_stream(buf: bytes) -> ParsedStream:
    if len(buf) < HEADER_SIZE:
        raise StreamError("stream shorter than its header")
    f = struct.unpack(HEADER_FMT, buf[:HEADER_SIZE])
    (magic, version, dcode, D, interp, cod, nonprog, d0, d1, d2, eb, K, qmax,
     c0, c1, c2, _r1, n_passes, n_chunks, n_out, pw, maxabs) = f
    if magic != MAGIC or version != VERSION:
        raise StreamError("bad magic or version")
    if dcode not in DTYPES or not 1 <= D <= 3 or interp not in (0, 1) or cod not in (0, 1):
        raise StreamError("bad header field")
    dt = DTYPES[dcode]
    h = StreamHeader(dtype=dt, ndim=D, interp=interp, nonprog_levels=nonprog,
                     dims=(d0, d1, d2)[:D], eb=eb, K=K, qmax=qmax,
                     chunk_log2=(c0, c1, c2)[:D], n_passes=n_passes, n_chunks=n_chunks,
                     n_outliers=n_out, payload_words=pw, maxabs=maxabs, coding=cod)
    nb = None
    if cod == CODING_ENTROPY:
        off_m = HEADER_SIZE + pad8(4 * 33 * n_passes)
        if off_m + 4 * n_chunks > len(buf):
            raise StreamError("stream shorter than its tables")
        nb = n_blocks_of(np.frombuffer(buf, dtype="<u4", count=n_chunks, offset=off_m))
    sizes = section_sizes(n_passes, n_chunks, n_out, dt.itemsize, pw, nb)
    if sum(sizes) != len(buf):
        raise StreamError("stream size does not match its header")
    off = HEADER_SIZE
    errq = np.frombuffer(buf, dtype="<u4", count=33 * n_passes, offset=off).reshape(n_passes, 33)
    off += sizes[1]
    masks = np.frombuffer(buf, dtype="<u4", count=n_chunks, offset=off)
    off += sizes[2]
    keys = np.frombuffer(buf, dtype="<u4", count=3 * n_out, offset=off).reshape(n_out, 3)
    off += sizes[3]
    vals = np.frombuffer(buf, dtype=dt.newbyteorder("<"), count=n_out, offset=off).astype(dt)
    off += sizes[4]
    bw = None
    if nb is not None:
        bw = np.frombuffer(buf, dtype=np.uint8, count=nb, offset=off).copy()
        off += sizes[5]
    payload = np.frombuffer(buf, dtype="<u4", count=pw, offset=off).astype(np.uint32)
    masks = masks.astype(np.uint32)
    if bw is not None:
        counts = stream_chunk_counts(h)
        W = [-(-n // 32) for n, _ in entropy.blocks(masks, counts)]
        if any(int(b) > w for b, w in zip(bw, W)) or int(bw.astype(np.int64).sum()) != pw:
            raise StreamError("block lengths do not match the payload")
        payload = entropy.decode_payload(masks, counts, bw, payload)
    return ParsedStream(header=h, errq=errq.astype(np.uint32), masks=masks,
                        out_keys=keys.astype(np.uint32), out_vals=vals,
                        payload=payload, payload_offset=off,
                        total_bytes=len(buf), block_words=bw)


def entropy_code_stream(buf: bytes) -> bytes:
    """The same stream with every stored block entropy coded (a coded stream
    is returned unchanged)."""
    ps = parse_stream(buf)
    h = ps.header
    if h.coding == CODING_ENTROPY:
        return buf
    bw, stored = entropy.code_payload(ps.masks, stream_chunk_counts(h), ps.payload)
    h2 = StreamHeader(**{**h.__dict__, "coding": CODING_ENTROPY, "payload_words": int(stored.size)})
    return write_stream(h2, ps.errq, ps.masks, ps.out_keys, ps.out_vals, stored, bw)
