"""Level schedule, pass lattices and chunk grouping (oracle).

Sec. 4.1 and Fig. "interp-design": the field is split into levels by a shrinking
stride; inside a level the interpolation runs once along each dimension in turn.
Sec. 4.2.2: the prediction P_l of a level is driven from the already
reconstructed coarser data, and the top level is predicted from zero (Alg. 1,
second step).

Readings used (the paper does not fix these):

* Number of levels: with M the largest dimension, K = 0 if M == 1, else
  max(1, ceil(log2(M - 1))).  Anchors are the points whose every coordinate is a
  multiple of 2^K; they form pass 0 and are predicted from zero.
* Level l (K down to 1) has stride h = 2^(l-1).  In level coordinates c = i / h
  (the grid of points whose coordinates are multiples of h, with extent
  d'_j = (d_j - 1) // h + 1) the level's pass along dimension k (k = 0 first, the
  contiguous dimension last) targets c_j any for j < k, c_k odd, c_j even for
  j > k, and predicts along k from c_k -+ 1 and c_k -+ 3.
* Codes of a pass are grouped in chunks: level-coordinate boxes of shape
  C = 2^chunk_log2 (every extent even).  Chunks are numbered in lexicographic
  tile order over the full tile grid ceil(d'_j / C_j) (a chunk may be empty);
  codes inside a chunk are in lexicographic order of their coordinates.
  The anchors form a single chunk.
"""

from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Tuple

import numpy as np

DEFAULT_CHUNK_LOG2 = {1: (12,), 2: (4, 6), 3: (1, 4, 6)}

ANY, ODD, EVEN = 0, 1, 2


def ceil_log2(v: int) -> int:
    """Smallest e with 2**e >= v, for v >= 1."""
    if v < 1:
        raise ValueError("ceil_log2 needs v >= 1")
    return (v - 1).bit_length()


def num_levels(dims) -> int:
    m = max(dims)
    if m == 1:
        return 0
    return max(1, ceil_log2(m - 1))


def level_dims(dims, h: int) -> Tuple[int, ...]:
    return tuple((d - 1) // h + 1 for d in dims)


def parity_count(extent: int, kind: int) -> int:
    """Number of coordinates in [0, extent) of the given parity kind."""
    if kind == ANY:
        return extent
    if kind == ODD:
        return extent // 2
    return (extent + 1) // 2


def parity_count_range(lo: int, hi: int, kind: int) -> int:
    """Number of coordinates in [lo, hi) (lo even) of the given parity kind."""
    n = max(0, hi - lo)
    if kind == ANY:
        return n
    if kind == ODD:
        return n // 2
    return (n + 1) // 2


@dataclass
class Pass:
    index: int                 # position in stream order (0 = anchors)
    level: int                 # l (0 for the anchors)
    dim: int                   # k (-1 for the anchors)
    h: int                     # stride in fine coordinates (2^K for the anchors)
    ldims: Tuple[int, ...]     # level-grid extent d'
    kinds: Tuple[int, ...]     # ANY / ODD / EVEN per dimension
    tdims: Tuple[int, ...]     # target-lattice extent per dimension
    chunk: Tuple[int, ...]     # chunk extent in level coordinates
    tiles: Tuple[int, ...]     # tile grid extent
    ctarget: Tuple[int, ...]   # chunk extent in target-lattice coordinates
    chunk_counts: np.ndarray = field(repr=False, default=None)  # codes per chunk

    @property
    def n_targets(self) -> int:
        return int(np.prod(self.tdims, dtype=np.int64))

    @property
    def n_chunks(self) -> int:
        return int(np.prod(self.tiles, dtype=np.int64))

    def target_coords(self, axis: int) -> np.ndarray:
        """Level coordinate of every target-lattice index along ``axis``."""
        m = np.arange(self.tdims[axis], dtype=np.int64)
        kind = self.kinds[axis]
        if kind == ANY:
            return m
        if kind == ODD:
            return 2 * m + 1
        return 2 * m


@dataclass
class Schedule:
    dims: Tuple[int, ...]
    K: int
    chunk_log2: Tuple[int, ...]
    passes: List[Pass]

    @property
    def ndim(self) -> int:
        return len(self.dims)

    @property
    def n_passes(self) -> int:
        return len(self.passes)


def _chunk_counts(tiles, ctarget, tdims) -> np.ndarray:
    """Codes per chunk over the full tile grid (lexicographic)."""
    per_dim = []
    for t, c, n in zip(tiles, ctarget, tdims):
        starts = np.arange(t, dtype=np.int64) * c
        per_dim.append(np.clip(n - starts, 0, c))
    out = per_dim[0]
    for e in per_dim[1:]:
        out = np.multiply.outer(out, e)
    return np.asarray(out, dtype=np.int64).reshape(-1)


def make_schedule(dims, chunk_log2=None) -> Schedule:
    dims = tuple(int(d) for d in dims)
    D = len(dims)
    if D < 1 or D > 3 or min(dims) < 1:
        raise ValueError("dims must have 1..3 entries, each >= 1")
    if chunk_log2 is None:
        chunk_log2 = DEFAULT_CHUNK_LOG2[D]
    chunk_log2 = tuple(int(c) for c in chunk_log2)
    if len(chunk_log2) != D or min(chunk_log2) < 1 or max(chunk_log2) > 16:
        raise ValueError("chunk_log2 needs one entry in [1, 16] per dimension")
    C = tuple(1 << c for c in chunk_log2)
    K = num_levels(dims)

    passes: List[Pass] = []
    # pass 0: the anchor grid, one chunk
    sa = 1 << K
    adims = tuple((d - 1) // sa + 1 for d in dims)
    p0 = Pass(index=0, level=0, dim=-1, h=sa, ldims=adims, kinds=(ANY,) * D,
              tdims=adims, chunk=adims, tiles=(1,) * D, ctarget=adims)
    p0.chunk_counts = np.array([int(np.prod(adims))], dtype=np.int64)
    passes.append(p0)

    for lev in range(K, 0, -1):
        h = 1 << (lev - 1)
        ld = level_dims(dims, h)
        for k in range(D):
            kinds = tuple(ANY if j < k else (ODD if j == k else EVEN) for j in range(D))
            tdims = tuple(parity_count(ld[j], kinds[j]) for j in range(D))
            tiles = tuple(-(-ld[j] // C[j]) for j in range(D))
            ctarget = tuple(C[j] if kinds[j] == ANY else C[j] // 2 for j in range(D))
            p = Pass(index=len(passes), level=lev, dim=k, h=h, ldims=ld, kinds=kinds,
                     tdims=tdims, chunk=C, tiles=tiles, ctarget=ctarget)
            p.chunk_counts = _chunk_counts(tiles, ctarget, tdims)
            passes.append(p)
    return Schedule(dims=dims, K=K, chunk_log2=chunk_log2, passes=passes)


def fine_index_grids(sched: Schedule, p: Pass):
    """Per-dimension fine coordinates of the pass's targets (for np.ix_)."""
    return [p.target_coords(j) * p.h for j in range(sched.ndim)]


def stream_positions(p: Pass):
    """(chunk id, local index) of every target, as arrays shaped like the lattice.

    Chunk id is the lexicographic tile number; the local index is the
    lexicographic position inside the (possibly ragged) chunk.
    """
    D = len(p.tdims)
    chunk_id = None
    local = None
    # extents of the chunk each target falls in, per dimension
    tile_of = []
    off_of = []
    ext_of = []
    for j in range(D):
        m = np.arange(p.tdims[j], dtype=np.int64)
        t = m // p.ctarget[j]
        o = m % p.ctarget[j]
        e = np.minimum(p.ctarget[j], p.tdims[j] - t * p.ctarget[j])
        tile_of.append(t)
        off_of.append(o)
        ext_of.append(e)
    shape = p.tdims
    for j in range(D):
        sh = [1] * D
        sh[j] = shape[j]
        t = tile_of[j].reshape(sh)
        stride_t = int(np.prod(p.tiles[j + 1:], dtype=np.int64))
        chunk_id = t * stride_t if chunk_id is None else chunk_id + t * stride_t
    # local = sum_j o_j * prod_{i>j} e_i
    for j in range(D):
        sh = [1] * D
        sh[j] = shape[j]
        term = off_of[j].reshape(sh)
        for i in range(j + 1, D):
            shi = [1] * D
            shi[i] = shape[i]
            term = term * ext_of[i].reshape(shi)
        local = term if local is None else local + term
    chunk_id = np.broadcast_to(chunk_id, shape)
    local = np.broadcast_to(local, shape)
    return chunk_id, local


def canonical_order(p: Pass) -> np.ndarray:
    """Flat lattice index of the code at each stream position of the pass."""
    if p.n_targets == 0:
        return np.zeros(0, dtype=np.int64)
    chunk_id, local = stream_positions(p)
    starts = np.concatenate([[0], np.cumsum(p.chunk_counts)[:-1]]).astype(np.int64)
    pos = (starts[chunk_id] + local).reshape(-1)
    order = np.empty(p.n_targets, dtype=np.int64)
    order[pos] = np.arange(p.n_targets, dtype=np.int64)
    return order
