"""Compress, retrieve and refine (oracle).

Compression (Sec. 3.2 workflow, Sec. 4.2.2 prediction model, Sec. 4.3-4.4
coding): anchors predicted from zero, then every pass of every level, coarse to
fine, predicts its targets from the current reconstruction, quantizes, and
writes the reconstruction back in place before any later pass reads it.  Codes
are negabinary, XOR-coded with their two prefix bits, and split into 32 planes
per chunk; all-zero planes are not stored.

Retrieval (Alg. 1): decode the loaded planes of every pass (missing planes read
as zero), dequantize, and predict in the same order with the same arithmetic.
The retrieval reads only the stream.

Refinement (Alg. 2, recompute form): merge the newly loaded planes into the
codes already held and recompute every pass from the first one whose codes
changed; coarser values are reused.  The result is bit-identical to a fresh
retrieval with the same plan.  The paper's additive form (a difference field
predicted from itself and added to the current reconstruction) is the variant
``refine_additive``; it agrees with a fresh retrieval only up to rounding.
"""

from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

from . import coding, planner, predict
from .schedule import Schedule, make_schedule, canonical_order, stream_positions
from .stream import (ParsedStream, StreamHeader, parse_stream, write_stream, DTYPES)


# --------------------------------------------------------------------------- #
# pass geometry helpers
# --------------------------------------------------------------------------- #

def _level_view(a: np.ndarray, h: int) -> np.ndarray:
    return a[tuple(slice(None, None, h) for _ in range(a.ndim))]


def _pass_slices(p, D):
    """(neighbour-lattice slices, target slices) inside the level grid."""
    nb = [slice(None)] * D
    for j in range(p.dim + 1, D):
        nb[j] = slice(0, None, 2)
    tg = list(nb)
    tg[p.dim] = slice(1, None, 2)
    return tuple(nb), tuple(tg)


def _anchor_index(dims, K):
    s = 1 << K
    return np.ix_(*[np.arange(0, d, s) for d in dims])


def _pass_prediction(work: np.ndarray, p, interp: int) -> np.ndarray:
    G = _level_view(work, p.h)
    nb, _ = _pass_slices(p, work.ndim)
    return predict.predict_along(G[nb], p.dim, interp)


def _store_pass(work: np.ndarray, p, values: np.ndarray):
    G = _level_view(work, p.h)
    _, tg = _pass_slices(p, work.ndim)
    G[tg] = values


def _pass_inputs(x: np.ndarray, p) -> np.ndarray:
    G = _level_view(x, p.h)
    _, tg = _pass_slices(p, x.ndim)
    return G[tg]


# --------------------------------------------------------------------------- #
# chunk encoding
# --------------------------------------------------------------------------- #

def _encode_pass_chunks(p, e_lattice: np.ndarray):
    """(masks [n_chunks] uint32, payload words) of one pass."""
    counts = p.chunk_counts.astype(np.int64)
    nch = counts.size
    W = -(-counts // 32)
    total_words = int(W.sum())
    masks = np.zeros(nch, dtype=np.uint32)
    if total_words == 0:
        return masks, np.zeros(0, dtype=np.uint32)
    order = canonical_order(p)
    e_stream = e_lattice.reshape(-1)[order]
    starts = np.concatenate([[0], np.cumsum(counts)[:-1]])
    wstart = np.concatenate([[0], np.cumsum(W)[:-1]])
    chunk_of = np.repeat(np.arange(nch), counts)
    padpos = wstart[chunk_of] * 32 + (np.arange(e_stream.size) - starts[chunk_of])
    padded = np.zeros(total_words * 32, dtype=np.uint32)
    padded[padpos] = e_stream
    rows = padded.reshape(total_words, 32)
    shifts = np.arange(32, dtype=np.uint64)
    planes = np.zeros((32, total_words), dtype=np.uint32)
    for k in range(32):
        bits = ((rows >> np.uint32(k)) & np.uint32(1)).astype(np.uint64) << shifts
        planes[k] = bits.sum(axis=1).astype(np.uint32)
    nz = planes != 0
    anyk = np.zeros((32, nch), dtype=bool)
    ne = np.nonzero(W > 0)[0]
    anyk[:, ne] = np.logical_or.reduceat(nz, wstart[ne], axis=1)
    for k in range(32):
        masks |= anyk[k].astype(np.uint32) << np.uint32(k)
    # payload: chunk-major, planes 31 -> 0
    cs, krev = np.nonzero(anyk.T[:, ::-1])
    ks = 31 - krev
    lens = W[cs]
    base = ks * total_words + wstart[cs]
    seg0 = np.concatenate([[0], np.cumsum(lens)[:-1]])
    idx = np.repeat(base - seg0, lens) + np.arange(int(lens.sum()))
    payload = planes.reshape(-1)[idx]
    return masks, payload


# --------------------------------------------------------------------------- #
# compress
# --------------------------------------------------------------------------- #

@dataclass
class CompressDebug:
    xhat: np.ndarray
    codes: List[np.ndarray]      # per pass, lattice shaped int64
    outlier_masks: List[np.ndarray]


def compress(x: np.ndarray, eb: float, interp: int = predict.CUBIC, chunk_log2=None,
             nonprog_levels: int = 0, debug: bool = False, errq_mode: str = "exact"):
    """Compress a float32/float64 field with absolute error bound eb.

    errq_mode "exact" stores each pass's measured delta-y (Thm. 1); "bound"
    stores the fixed table of coding.errq_bound_table for every pass."""
    if errq_mode not in ("exact", "bound"):
        raise ValueError("errq_mode is 'exact' or 'bound'")
    x = np.ascontiguousarray(x)
    if x.dtype not in (np.float32, np.float64):
        raise TypeError("only float32 and float64 fields")
    if not (np.isfinite(eb) and eb > 0):
        raise ValueError("eb must be finite and > 0")
    dims = x.shape
    D = x.ndim
    sched = make_schedule(dims, chunk_log2)
    if not (0 <= nonprog_levels <= sched.K):
        raise ValueError("nonprog_levels out of range")
    work = x.copy()
    all_masks = []
    payload_parts = []
    errq = np.zeros((sched.n_passes, 33), dtype=np.uint32)
    keys = []
    vals = []
    dbg_codes = []
    dbg_out = []
    for p in sched.passes:
        if p.index == 0:
            idx = _anchor_index(dims, sched.K)
            xt = x[idx]
            pred = np.zeros_like(xt)
            q, xh, out = predict.quantize(xt, pred, eb)
            work[idx] = xh
        else:
            pred = _pass_prediction(work, p, interp)
            xt = _pass_inputs(x, p)
            q, xh, out = predict.quantize(xt, pred, eb)
            _store_pass(work, p, xh)
        errq[p.index] = coding.errq_table(q) if errq_mode == "exact" else coding.errq_bound_table()
        e = coding.xor_encode(coding.to_negabinary(q))
        masks, payload = _encode_pass_chunks(p, e)
        all_masks.append(masks)
        payload_parts.append(payload)
        if out.any():
            cid, loc = stream_positions(p)
            sel = np.nonzero(out.reshape(-1))[0]
            c = np.asarray(cid).reshape(-1)[sel]
            lo = np.asarray(loc).reshape(-1)[sel]
            srt = np.lexsort((lo, c))
            keys.append(np.stack([np.full(sel.size, p.index), c[srt], lo[srt]], axis=1))
            vals.append(xt.reshape(-1)[sel][srt])
        if debug:
            dbg_codes.append(q.copy())
            dbg_out.append(out.copy())
    masks = np.concatenate(all_masks).astype(np.uint32)
    payload = np.concatenate(payload_parts).astype(np.uint32)
    if keys:
        out_keys = np.concatenate(keys).astype(np.uint32)
        out_vals = np.concatenate(vals).astype(x.dtype)
    else:
        out_keys = np.zeros((0, 3), dtype=np.uint32)
        out_vals = np.zeros(0, dtype=x.dtype)
    fin = work[np.isfinite(work)]
    maxabs = float(np.max(np.abs(fin))) if fin.size else 0.0
    h = StreamHeader(dtype=x.dtype, ndim=D, interp=interp, nonprog_levels=nonprog_levels,
                     dims=tuple(dims), eb=float(eb), K=sched.K,
                     qmax=predict.QMAX[x.dtype], chunk_log2=sched.chunk_log2,
                     n_passes=sched.n_passes, n_chunks=int(masks.size),
                     n_outliers=int(out_vals.size), payload_words=int(payload.size),
                     maxabs=maxabs)
    buf = write_stream(h, errq, masks, out_keys, out_vals, payload)
    if debug:
        return buf, CompressDebug(xhat=work, codes=dbg_codes, outlier_masks=dbg_out)
    return buf


# --------------------------------------------------------------------------- #
# retrieve / refine
# --------------------------------------------------------------------------- #

@dataclass
class PassData:
    """Loaded (truncated, XOR-coded) codes of one pass, in stream order."""
    e: np.ndarray
    b: int


@dataclass
class State:
    stream: bytes
    parsed: ParsedStream
    sched: Schedule
    tables: planner.PlanTables
    plan: np.ndarray
    passes: List[PassData]
    field: np.ndarray
    bound: float
    bytes_read: int = 0          # payload bytes read by the last call
    flags: int = 0


def _chunk_word_offsets(ps: ParsedStream, sched: Schedule):
    """Per pass: (first chunk index, word offset of every chunk's data in the
    raw payload, index of every chunk's first stored block)."""
    out = []
    c0 = 0
    off = 0
    blk = 0
    for p in sched.passes:
        n = p.n_chunks
        m = ps.masks[c0:c0 + n]
        W = -(-p.chunk_counts // 32)
        pc = np.array([bin(int(v)).count("1") for v in m], dtype=np.int64)
        sizes = pc * W
        starts = off + np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64)
        bstarts = blk + np.concatenate([[0], np.cumsum(pc)[:-1]]).astype(np.int64)
        out.append((c0, starts, bstarts))
        off += int(sizes.sum())
        blk += int(pc.sum())
        c0 += n
    return out


def _load_planes(ps: ParsedStream, p, c0, starts, b_lo: int, b_hi: int, bstarts=None):
    """XOR-coded codes of the pass built from planes k with b_lo <= k < b_hi.

    Returns (e in stream order, payload bytes read); a block of an
    entropy-coded stream counts the bytes it occupies there.
    """
    counts = p.chunk_counts
    e = np.zeros(int(counts.sum()), dtype=np.uint32)
    nread = 0
    pos = 0
    for ci in range(p.n_chunks):
        n = int(counts[ci])
        if n == 0:
            continue
        W = -(-n // 32)
        mask = int(ps.masks[c0 + ci])
        planes = np.zeros((32, W), dtype=np.uint32)
        w = int(starts[ci])
        blk = int(bstarts[ci]) if bstarts is not None else 0
        for k in range(31, -1, -1):
            if not (mask >> k) & 1:
                continue
            if b_lo <= k < b_hi:
                planes[k] = ps.payload[w:w + W]
                nread += 4 * (W if ps.block_words is None else int(ps.block_words[blk]))
            w += W
            blk += 1
        e[pos:pos + n] = coding.unpack_planes(planes, n)
        pos += n
    return e, nread


def _reconstruct_from(state: State, s_min: int):
    """Recompute every pass s >= s_min from the loaded codes (Alg. 1)."""
    ps, sched = state.parsed, state.sched
    h = ps.header
    dt = h.dtype
    two_eb, _ = predict.quant_constants(dt, h.eb)
    keys = ps.out_keys
    work = state.field
    for p in sched.passes:
        if p.index < s_min:
            continue
        pdat = state.passes[p.index]
        m = coding.keep_mask(pdat.b)
        v = coding.xor_decode(pdat.e & m) & m
        qs = coding.from_negabinary(v)
        q = np.zeros(p.n_targets, dtype=np.int64)
        if p.n_targets:
            q[canonical_order(p)] = qs
        q = q.reshape(p.tdims)
        with np.errstate(all="ignore"):
            if p.index == 0:
                idx = _anchor_index(h.dims, h.K)
                pred = np.zeros(p.tdims, dtype=dt)
                vals = pred + q.astype(dt) * two_eb
            else:
                pred = _pass_prediction(work, p, h.interp)
                vals = pred + q.astype(dt) * two_eb
        sel = np.nonzero(keys[:, 0] == p.index)[0] if keys.size else np.zeros(0, np.int64)
        if sel.size:
            order = canonical_order(p)
            cstart = np.concatenate([[0], np.cumsum(p.chunk_counts)[:-1]]).astype(np.int64)
            pos = cstart[keys[sel, 1].astype(np.int64)] + keys[sel, 2].astype(np.int64)
            flat = vals.reshape(-1).copy()
            flat[order[pos]] = ps.out_vals[sel]
            vals = flat.reshape(vals.shape)
        if p.index == 0:
            work[idx] = vals
        else:
            _store_pass(work, p, vals)


def open_stream(buf: bytes):
    ps = parse_stream(buf)
    sched = make_schedule(ps.header.dims, ps.header.chunk_log2)
    tables = planner.tables_from_stream(ps)
    return ps, sched, tables


def make_plan(tables, mode: str, value: float, limit=None, level_groups: bool = False):
    if mode == "eb":
        plan, flags = planner.plan_error_bound(tables, value, limit, level_groups)
    elif mode == "bitrate":
        plan, flags = planner.plan_bitrate(tables, value, limit, level_groups)
    else:
        raise ValueError("mode must be 'eb' or 'bitrate'")
    return plan, flags


def retrieve_with_plan(buf: bytes, plan, mode: str = "eb", target: Optional[float] = None,
                       flags: int = 0) -> State:
    ps, sched, tables = open_stream(buf)
    plan = np.asarray(plan, dtype=np.int64)
    offs = _chunk_word_offsets(ps, sched)
    passes = []
    nread = 0
    for p in sched.passes:
        c0, starts, bstarts = offs[p.index]
        b = int(plan[p.index])
        e, nb = _load_planes(ps, p, c0, starts, b, 32, bstarts)
        nread += nb
        passes.append(PassData(e=e, b=b))
    fld = np.zeros(ps.header.dims, dtype=ps.header.dtype)
    if target is None:
        b0 = planner.bound_of(tables, plan, tables.maxabs)
        bound = planner.bound_of(tables, plan, 2.0 * (tables.maxabs + b0))
    else:
        bound = planner.reported_bound(tables, plan, mode, target)
    st = State(stream=buf, parsed=ps, sched=sched, tables=tables, plan=plan.copy(),
               passes=passes, field=fld, bound=bound, bytes_read=nread, flags=flags)
    _reconstruct_from(st, 0)
    return st


def retrieve(buf: bytes, mode: str = "eb", value: float = 0.0,
             level_groups: bool = False) -> State:
    """Alg. 1 with the plan chosen by the Sec. 5 planner for (mode, value);
    ``level_groups`` plans with one discarded-plane count per level."""
    _, _, tables = open_stream(buf)
    plan, flags = make_plan(tables, mode, value, level_groups=level_groups)
    return retrieve_with_plan(buf, plan, mode, value, flags)


def refine(state: State, mode: str, value: float, level_groups: bool = False) -> State:
    """Alg. 2 (recompute form): load only new planes, recompute from s_min."""
    tables = state.tables
    if mode == "eb" and value >= state.bound:
        state.flags = planner.FLAG_NOOP
        state.bytes_read = 0
        return state
    plan, flags = make_plan(tables, mode, value, limit=state.plan, level_groups=level_groups)
    if np.array_equal(plan, state.plan):
        state.flags = flags | planner.FLAG_NOOP
        state.bytes_read = 0
        return state
    offs = _chunk_word_offsets(state.parsed, state.sched)
    s_min = None
    nread = 0
    for p in state.sched.passes:
        b_new, b_old = int(plan[p.index]), int(state.plan[p.index])
        if b_new < b_old:
            c0, starts, bstarts = offs[p.index]
            e_new, nb = _load_planes(state.parsed, p, c0, starts, b_new, b_old, bstarts)
            nread += nb
            state.passes[p.index].e = state.passes[p.index].e | e_new
            state.passes[p.index].b = b_new
            if s_min is None:
                s_min = p.index
    state.plan = plan.copy()
    state.bound = planner.reported_bound(tables, plan, mode, value)
    state.bytes_read = nread
    state.flags = flags
    if s_min is not None:
        _reconstruct_from(state, s_min)
    return state


def _add_delta_from(state: State, s_min: int, old_plan):
    """Additive form of Alg. 2: the difference field Delta is predicted pass
    by pass from Delta itself (interpolation is linear) plus the dequantized
    code difference of the pass, outliers contributing nothing; then
    x_new = x_old + Delta wherever Delta is not zero."""
    ps, sched = state.parsed, state.sched
    h = ps.header
    dt = h.dtype
    two_eb, _ = predict.quant_constants(dt, h.eb)
    keys = ps.out_keys
    delta = np.zeros_like(state.field)
    for p in sched.passes:
        if p.index < s_min:
            continue
        assert p.index > 0, "the anchors are always fully loaded"
        pdat = state.passes[p.index]
        mn = coding.keep_mask(int(state.plan[p.index]))
        mo = coding.keep_mask(int(old_plan[p.index]))
        qn = coding.from_negabinary(coding.xor_decode(pdat.e & mn) & mn)
        qo = coding.from_negabinary(coding.xor_decode(pdat.e & mo) & mo)
        dq = np.zeros(p.n_targets, dtype=np.int64)
        if p.n_targets:
            dq[canonical_order(p)] = qn - qo
        dq = dq.reshape(p.tdims)
        with np.errstate(all="ignore"):
            pred = _pass_prediction(delta, p, h.interp)
            vals = pred + dq.astype(dt) * two_eb
        sel = np.nonzero(keys[:, 0] == p.index)[0] if keys.size else np.zeros(0, np.int64)
        if sel.size:
            order = canonical_order(p)
            cstart = np.concatenate([[0], np.cumsum(p.chunk_counts)[:-1]]).astype(np.int64)
            pos = cstart[keys[sel, 1].astype(np.int64)] + keys[sel, 2].astype(np.int64)
            flat = vals.reshape(-1).copy()
            flat[order[pos]] = 0
            vals = flat.reshape(vals.shape)
        _store_pass(delta, p, vals)
    nz = delta != 0
    with np.errstate(all="ignore"):
        state.field[nz] = state.field[nz] + delta[nz]


def refine_additive(state: State, mode: str, value: float, level_groups: bool = False) -> State:
    """Alg. 2 in the paper's additive form (a variant): plan and load the new
    planes as :func:`refine` does, then add the difference field to the
    current reconstruction instead of recomputing it.  The result agrees with
    a fresh retrieval only up to rounding; its bound is
    :func:`planner.additive_bound`."""
    tables = state.tables
    if mode == "eb" and value >= state.bound:
        state.flags = planner.FLAG_NOOP
        state.bytes_read = 0
        return state
    plan, flags = make_plan(tables, mode, value, limit=state.plan, level_groups=level_groups)
    if np.array_equal(plan, state.plan):
        state.flags = flags | planner.FLAG_NOOP
        state.bytes_read = 0
        return state
    old_plan = state.plan.copy()
    offs = _chunk_word_offsets(state.parsed, state.sched)
    s_min = None
    nread = 0
    for p in state.sched.passes:
        b_new, b_old = int(plan[p.index]), int(old_plan[p.index])
        if b_new < b_old:
            c0, starts, bstarts = offs[p.index]
            e_new, nb = _load_planes(state.parsed, p, c0, starts, b_new, b_old, bstarts)
            nread += nb
            state.passes[p.index].e = state.passes[p.index].e | e_new
            state.passes[p.index].b = b_new
            if s_min is None:
                s_min = p.index
    state.plan = plan.copy()
    state.bound = planner.additive_bound(tables, plan, old_plan, mode, value)
    state.bytes_read = nread
    state.flags = flags
    if s_min is not None:
        _add_delta_from(state, s_min, old_plan)
    return state


def stream_dtype(buf: bytes):
    return parse_stream(buf).header.dtype


__all__ = ["compress", "retrieve", "retrieve_with_plan", "refine", "refine_additive", "open_stream",
           "make_plan", "State", "DTYPES"]
