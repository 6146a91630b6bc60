"""Error bound of a partial load and the two loading planners (oracle).

Thm. 1 bounds the L-infinity error of a reconstruction from a subset of
bitplanes by eb plus the truncation losses delta-y of every group, each
amplified by the interpolation norm p (1 linear, 1.25 cubic) once per later
prediction step.  Sec. 5.2 turns "load the least data for an error bound E" into
a knapsack solved by dynamic programming over (level, error budget); Sec. 5.3
does the same for "least error within a byte budget".

Readings used:

* Groups are passes, not levels.  In D > 1 dimensions a level runs D cascaded
  one-dimensional predictions, so a loss in an earlier pass of the same level
  is amplified again by every later pass; the per-level factor of Thm. 1 is
  not an upper bound there (see the counterexample test).  With passes
  s = 1..S in stream order, loss delta_s reaches the final error through at most
  S - s further predictions: A_s = p^(S - s).
* delta_s(b) = errq[s][b] * T(2 eb) (the actual quantization bin).
* Floating-point slack: a reconstruction from truncated codes is computed in the
  field's dtype, so the difference to the full-precision reconstruction picks
  up rounding.  One stencil plus the add of the dequantized code rounds by at
  most 7 u M per evaluation (u the unit roundoff, M a bound on the magnitudes
  involved), so the difference gains at most r = 14 u M per pass once any
  earlier or current pass is lossy.  Choosing b > 0 in pass s is charged
  T_s * r with T_s = sum_{s' >= s} A_s'; this over-counts when several passes
  are lossy and is exactly zero for a full load (which reproduces the
  compressor's reconstruction bit for bit).  M = maxabs + E in error-bound
  mode; in bitrate mode the plan is chosen with M = maxabs and the reported
  bound uses M = 2 (maxabs + B0), B0 being that plan's bound at M = maxabs.
* Error budget discretised into G = 1024 units of (E - eb) / G; a pass's cost is
  floor(term / unit) + 1 units for a non-zero term (never below the exact
  ratio), 0 for a zero term.  Ties go to the smallest number of discarded
  planes.  Byte budgets are discretised into at most 1024 units, costs rounded
  up, so the plan never exceeds the budget; a budget of at least the whole
  stream loads everything.
* Anchors (pass 0) and the passes of the first ``nonprog_levels`` levels are
  always fully loaded.

Variant (the paper's own grouping, Sec. 4.3): with ``level_groups`` every pass
of a level discards the same number of planes, so the dynamic programs choose
one b per level.  The bound of such a plan is still the per-pass bound above
(the per-level factor of Thm. 1 is not an upper bound in D > 1); a level's
term and bytes are the sums over its passes.  Its plans are a subset of the
per-pass ones, so up to the discretization of the budget it loads at least as
much for the same bound.
"""

from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from .schedule import make_schedule
from .stream import ParsedStream

G_UNITS = 1024
FLAG_CLAMPED_TO_EB = 1
FLAG_BUDGET_BELOW_MIN = 2
FLAG_NOOP = 4

UNIT_ROUNDOFF = {4: 2.0 ** -24, 8: 2.0 ** -53}


@dataclass
class PlanTables:
    """Everything the planner needs, read from a stream's fixed part."""
    n_passes: int
    errq: np.ndarray        # [P, 33] uint32
    sizes: np.ndarray       # [P, 32] int64 bytes of plane k of pass s
    progressive: np.ndarray  # [P] bool
    amp: np.ndarray         # [P] float64, A_s (0 for the anchors)
    tail: np.ndarray        # [P] float64, T_s
    two_eb: float
    eb: float
    unit_roundoff: float
    maxabs: float
    n_points: int
    total_bytes: int
    fixed_bytes: int
    levels: np.ndarray = None   # [P] level of every pass (pass 0: the anchors)


def tables_from_stream(ps: ParsedStream) -> PlanTables:
    h = ps.header
    sched = make_schedule(h.dims, h.chunk_log2)
    P = h.n_passes
    sizes = np.zeros((P, 32), dtype=np.int64)
    c0 = 0
    blk = 0
    for p in sched.passes:
        n = p.n_chunks
        m = ps.masks[c0:c0 + n].astype(np.uint64)
        if ps.block_words is None:
            W = (-(-p.chunk_counts // 32)).astype(np.int64)
            for k in range(32):
                bit = ((m >> np.uint64(k)) & np.uint64(1)).astype(np.int64)
                sizes[p.index, k] = int(np.sum(bit * W)) * 4
        else:
            # entropy-coded blocks: every plane costs the words it occupies
            for mk in m:
                for k in range(31, -1, -1):
                    if (int(mk) >> k) & 1:
                        sizes[p.index, k] += 4 * int(ps.block_words[blk])
                        blk += 1
        c0 += n
    prog = np.ones(P, dtype=bool)
    prog[0] = False
    for p in sched.passes[1:]:
        if p.level > h.K - h.nonprog_levels:
            prog[p.index] = False
    pval = 1.0 if h.interp == 0 else 1.25
    amp = np.zeros(P, dtype=np.float64)
    tail = np.zeros(P, dtype=np.float64)
    a = 1.0
    t = 0.0
    for s in range(P - 1, 0, -1):
        amp[s] = a
        t = t + a
        tail[s] = t
        a = a * pval
    two_eb = float(h.dtype.type(2.0 * h.eb))
    prog_bytes = int(np.sum(sizes[prog]))
    return PlanTables(n_passes=P, errq=ps.errq.copy(), sizes=sizes, progressive=prog,
                      amp=amp, tail=tail, two_eb=two_eb, eb=float(h.eb),
                      unit_roundoff=UNIT_ROUNDOFF[h.dtype.itemsize],
                      maxabs=float(h.maxabs),
                      n_points=int(np.prod(h.dims, dtype=np.int64)),
                      total_bytes=ps.total_bytes, fixed_bytes=ps.total_bytes - prog_bytes,
                      levels=np.array([p.level for p in sched.passes], dtype=np.int64))


def rounding_step(t: PlanTables, M: float) -> float:
    return 14.0 * t.unit_roundoff * M


def term(t: PlanTables, s: int, b: int, r: float) -> float:
    """Contribution of pass s with b discarded planes to the bound."""
    v = (float(t.errq[s][b]) * t.two_eb) * t.amp[s]
    if b > 0:
        v = v + t.tail[s] * r
    return v


def bound_of(t: PlanTables, plan, M: float) -> float:
    r = rounding_step(t, M)
    tot = t.eb
    for s in range(t.n_passes):
        if t.progressive[s]:
            tot = tot + term(t, s, int(plan[s]), r)
    return tot


def loaded_bytes(t: PlanTables, plan) -> int:
    tot = t.fixed_bytes
    for s in range(t.n_passes):
        if t.progressive[s]:
            tot += int(np.sum(t.sizes[s, int(plan[s]):]))
    return tot


def plan_groups(t: PlanTables, level_groups: bool = False):
    """Passes that share one discarded-plane count, in stream order: every
    pass alone, or (level_groups) the anchors alone and then one group per
    level."""
    if not level_groups:
        return [[s] for s in range(t.n_passes)]
    groups = [[0]]
    for s in range(1, t.n_passes):
        if len(groups) > 1 and t.levels[groups[-1][0]] == t.levels[s]:
            groups[-1].append(s)
        else:
            groups.append([s])
    return groups


def _allowed(t: PlanTables, g, limit) -> range:
    """Choices of b for a group (a list of passes) or a single pass."""
    if isinstance(g, (int, np.integer)):
        g = [int(g)]
    if not t.progressive[g[0]]:
        return range(0, 1)
    hi = 32 if limit is None else min(int(limit[s]) for s in g)
    return range(0, hi + 1)


def _group_term(t: PlanTables, g, b: int, r: float) -> float:
    v = 0.0
    for s in g:
        if t.progressive[s]:
            v = v + term(t, s, b, r)
    return v


def _group_bytes(t: PlanTables, g, lo: int, hi: int) -> int:
    """Bytes of planes lo <= k < hi over the group's progressive passes."""
    return int(sum(int(np.sum(t.sizes[s, lo:hi])) for s in g if t.progressive[s]))


def plan_error_bound(t: PlanTables, E: float, limit=None, level_groups: bool = False):
    """Sec. 5.2: most bytes left unloaded subject to bound <= E.

    ``limit`` (refine) caps b per pass at the planes not yet loaded.
    Returns (plan, flags).
    """
    P = t.n_passes
    R = E - t.eb
    if not (R >= 0.0):
        return np.zeros(P, dtype=np.int64), FLAG_CLAMPED_TO_EB
    r = rounding_step(t, t.maxabs + E)
    u = R / G_UNITS
    NEG = np.iinfo(np.int64).min // 4
    groups = plan_groups(t, level_groups)
    NG = len(groups)
    F = np.zeros(G_UNITS + 1, dtype=np.int64)        # F_0[r] = 0
    choices = np.zeros((NG, G_UNITS + 1), dtype=np.int64)
    costs = np.zeros((NG, 33), dtype=np.int64)
    for gi, g in enumerate(groups):
        newF = np.full(G_UNITS + 1, NEG, dtype=np.int64)
        ch = np.zeros(G_UNITS + 1, dtype=np.int64)
        for b in _allowed(t, g, limit):
            tv = _group_term(t, g, b, r)
            if tv == 0.0:
                c = 0
            else:
                qv = tv / u if u > 0.0 else math.inf
                c = math.floor(qv) + 1 if qv < G_UNITS else G_UNITS + 1
            costs[gi, b] = c
            if c > G_UNITS:
                continue
            saved = _group_bytes(t, g, 0, b)
            prev = F[:G_UNITS + 1 - c]
            cand = np.full(G_UNITS + 1, NEG, dtype=np.int64)
            cand[c:] = np.where(prev == NEG, NEG, prev + saved)
            better = cand > newF
            newF = np.where(better, cand, newF)
            ch = np.where(better, b, ch)
        F = newF
        choices[gi] = ch
    plan = np.zeros(P, dtype=np.int64)
    rr = G_UNITS
    for gi in range(NG - 1, -1, -1):
        b = int(choices[gi, rr])
        plan[groups[gi]] = b
        rr -= int(costs[gi, b])
    return plan, 0


def plan_bitrate(t: PlanTables, bitrate: float, limit=None, level_groups: bool = False):
    """Sec. 5.3: least bound subject to loaded bytes <= bitrate * n / 8.

    Returns (plan, flags).  With ``limit`` (refine) and a budget below the
    bytes already loaded, the current plan is returned with FLAG_NOOP.
    """
    P = t.n_passes
    bt = bitrate * t.n_points / 8.0
    if bt >= t.total_bytes:
        # everything fits
        return np.zeros(P, dtype=np.int64), 0
    budget = math.floor(bt) - t.fixed_bytes
    if limit is not None:
        cur = np.asarray(limit, dtype=np.int64)
        if budget < loaded_bytes(t, cur) - t.fixed_bytes:
            return cur.copy(), FLAG_NOOP
    if budget < 0:
        plan = np.zeros(P, dtype=np.int64)
        for s in range(P):
            if t.progressive[s]:
                plan[s] = 32
        return plan, FLAG_BUDGET_BELOW_MIN
    ub = max(1, -(-budget // G_UNITS))
    cap = budget // ub
    r = rounding_step(t, t.maxabs)
    INF = math.inf
    groups = plan_groups(t, level_groups)
    NG = len(groups)
    F = np.zeros(cap + 1, dtype=np.float64)          # F_0[r] = 0
    choices = np.zeros((NG, cap + 1), dtype=np.int64)
    lcs = np.zeros((NG, 33), dtype=np.int64)
    for gi, g in enumerate(groups):
        newF = np.full(cap + 1, INF, dtype=np.float64)
        ch = np.zeros(cap + 1, dtype=np.int64)
        for b in _allowed(t, g, limit):
            lc = -(-_group_bytes(t, g, b, 32) // ub)
            tv = _group_term(t, g, b, r)
            lcs[gi, b] = lc
            if lc > cap:
                continue
            cand = np.full(cap + 1, INF, dtype=np.float64)
            cand[lc:] = F[:cap + 1 - lc] + tv
            better = cand < newF
            newF = np.where(better, cand, newF)
            ch = np.where(better, b, ch)
        F = newF
        choices[gi] = ch
    if not math.isfinite(F[cap]):
        # only reachable with a limit: nothing fits, keep what is loaded
        return np.asarray(limit, dtype=np.int64).copy(), FLAG_NOOP
    plan = np.zeros(P, dtype=np.int64)
    rr = cap
    for gi in range(NG - 1, -1, -1):
        b = int(choices[gi, rr])
        plan[groups[gi]] = b
        rr -= int(lcs[gi, b])
    return plan, 0


def reported_bound(t: PlanTables, plan, mode: str, target: float) -> float:
    """Bound reported with a plan.

    Error-bound mode uses M = maxabs + E (valid by induction over the passes
    whenever the bound stays below E); bitrate mode uses
    M = 2 (maxabs + B0), B0 the bound at M = maxabs.
    """
    if mode == "eb":
        if target < t.eb:
            return bound_of(t, plan, t.maxabs)
        return bound_of(t, plan, t.maxabs + target)
    b0 = bound_of(t, plan, t.maxabs)
    return bound_of(t, plan, 2.0 * (t.maxabs + b0))


def reported_magnitude(t: PlanTables, plan, mode: str, target: float) -> float:
    """The magnitude bound M that reported_bound uses."""
    if mode == "eb":
        return t.maxabs if target < t.eb else t.maxabs + target
    return 2.0 * (t.maxabs + bound_of(t, plan, t.maxabs))


def additive_bound(t: PlanTables, plan, old_plan, mode: str, target: float) -> float:
    """Bound reported by the additive form of Alg. 2 (x_new = x_old + Delta).

    Reading: the reported bound of the new plan plus what the additive form
    rounds where a fresh reconstruction does not -- the old reconstruction's
    own rounding (the rounding terms T_s r of the old plan's lossy passes), the
    rounding of the difference field (charged as if every progressive pass
    were lossy: T_s1 r, s1 the first progressive pass) and the final addition
    (u M).
    """
    M = reported_magnitude(t, plan, mode, target)
    r = rounding_step(t, M)
    a = reported_bound(t, plan, mode, target)
    first = None
    for s in range(t.n_passes):
        if not t.progressive[s]:
            continue
        if first is None:
            first = s
        if int(old_plan[s]) > 0:
            a = a + t.tail[s] * r
    if first is not None:
        a = a + t.tail[first] * r
    return a + t.unit_roundoff * M


def fixed_section_bytes(ps: ParsedStream) -> int:
    """Bytes before the payload (with the block lengths of a coded stream)."""
    return ps.payload_offset
