"""Pins of the oracle's refinement planner (not gpu).

Alg. 2 refines a resident reconstruction by loading planes it does not hold
yet; the Sec. 5.2 (error bound) and Sec. 5.3 (bitrate) programs then choose
among plans that never drop a loaded plane (b <= b_cur per pass).  These tests
pin that restricted program, independently of the implementation:

* on streams of three passes (anchors + two progressive passes, 33^2 plans)
  the program's plan equals an exhaustive enumeration of every plan under a
  random limit, with the same tie-break in error-bound mode and the same least
  bound in bitrate mode;
* a bitrate refinement counts every loaded byte (old planes included) against
  bitrate * n / 8, and it is a no-op exactly when that budget is below what is
  already loaded (or when the best plan is the current one);
* when the fresh optimum for the new target already lies under the limit, the
  refined plan saves exactly as many bytes as that fresh plan.
"""

import itertools

import numpy as np
import pytest

import fieldgen
from oracle import codec, planner, predict

G = planner.G_UNITS


def _choices(t, limit):
    """Every allowed b per pass: 0 for the fixed passes, 0..limit[s] else."""
    out = []
    for s in range(t.n_passes):
        if not t.progressive[s]:
            out.append([0])
        else:
            hi = 32 if limit is None else int(limit[s])
            out.append(list(range(hi + 1)))
    return out


def _saved(t, plan):
    return sum(int(np.sum(t.sizes[s, :plan[s]])) for s in range(t.n_passes) if t.progressive[s])


def _loaded(t, plan):
    return t.fixed_bytes + sum(int(np.sum(t.sizes[s, plan[s]:]))
                               for s in range(t.n_passes) if t.progressive[s])


def _enum_eb(t, E, limit):
    """Largest saved bytes over all plans under `limit` whose integer costs fit
    the 1024 units; ties to the smallest b of the last pass, then of the one
    before (the enumeration runs with the last pass slowest)."""
    u = (E - t.eb) / G
    r = planner.rounding_step(t, t.maxabs + E)

    def cost(s, b):
        tv = planner.term(t, s, b, r) if t.progressive[s] else 0.0
        if tv == 0.0:
            return 0
        q = tv / u if u > 0 else np.inf
        return int(np.floor(q)) + 1 if q < G else G + 1

    ch = _choices(t, limit)
    best = None
    for rc in itertools.product(*reversed(ch)):
        plan = list(rc[::-1])
        if sum(cost(s, plan[s]) for s in range(t.n_passes)) > G:
            continue
        sv = _saved(t, plan)
        if best is None or sv > best[0]:
            best = (sv, plan)
    return best


def _enum_br(t, bitrate, limit):
    """Least bound over all plans under `limit` whose rounded-up byte costs
    fit the budget; None when none fits."""
    budget = int(np.floor(bitrate * t.n_points / 8.0)) - t.fixed_bytes
    ub = max(1, -(-budget // G))
    cap = budget // ub
    r = planner.rounding_step(t, t.maxabs)
    best = None
    for plan in itertools.product(*_choices(t, limit)):
        lc = sum(-(-int(np.sum(t.sizes[s, plan[s]:])) // ub) for s in range(t.n_passes)
                 if t.progressive[s])
        if lc > cap:
            continue
        err = 0.0
        for s in range(t.n_passes):
            if t.progressive[s]:
                err = err + planner.term(t, s, plan[s], r)
        if best is None or err < best[0]:
            best = (err, list(plan))
    return best


def _tiny_streams(interp):
    # 5 points in 1-D: anchors, level 2, level 1; 3 x 2 in 2-D: anchors and
    # the two passes of level 1
    for shape, seed in (((5,), 1), ((3, 2), 2)):
        x = fieldgen.random_field(shape, seed=seed, dtype=np.float64, scale=50.0, smooth=False)
        buf = codec.compress(x, 1e-3, interp=interp)
        _, _, t = codec.open_stream(buf)
        assert t.n_passes == 3
        yield buf, t


def _random_limits(t, rng, n):
    yield np.array([0, 32, 32])
    yield np.array([0, 0, 0])
    for _ in range(n):
        lim = rng.integers(0, 33, t.n_passes)
        lim[0] = 0
        yield lim


@pytest.mark.parametrize("interp", [predict.LINEAR, predict.CUBIC])
def test_refine_error_bound_program_equals_enumeration(interp):
    rng = np.random.default_rng(21)
    for buf, t in _tiny_streams(interp):
        for limit in _random_limits(t, rng, 12):
            for E in (1e-3, 1.5e-3, 1e-2, 0.1, 1.0, 10.0, 1e3):
                plan, flags = planner.plan_error_bound(t, E, limit=limit)
                assert flags == 0
                assert np.all(plan <= limit)
                best = _enum_eb(t, E, limit)
                assert best is not None        # b = 0 everywhere always fits
                assert _saved(t, plan) == best[0]
                assert list(plan) == best[1]   # same tie-break
                assert planner.bound_of(t, plan, t.maxabs + E) <= E


@pytest.mark.parametrize("interp", [predict.LINEAR, predict.CUBIC])
def test_refine_bitrate_program_equals_enumeration(interp):
    rng = np.random.default_rng(22)
    for buf, t in _tiny_streams(interp):
        for limit in _random_limits(t, rng, 12):
            held = _loaded(t, limit)
            for br in (0.5, 2.0, 8.0, 16.0, 24.0, 40.0, 64.0, 200.0):
                plan, flags = planner.plan_bitrate(t, br, limit=limit)
                bt = br * t.n_points / 8.0
                if bt >= t.total_bytes:
                    # everything fits: load everything
                    assert flags == 0 and np.all(plan == 0)
                    continue
                budget = int(np.floor(bt)) - t.fixed_bytes
                if budget < held - t.fixed_bytes:
                    # the budget is below what is already loaded: no-op
                    assert flags == planner.FLAG_NOOP
                    assert list(plan) == list(limit)
                    continue
                assert np.all(plan <= limit)
                best = _enum_br(t, br, limit)
                if best is None:
                    # byte units rounded up leave no plan under the cap
                    assert flags == planner.FLAG_NOOP and list(plan) == list(limit)
                    continue
                assert flags == 0
                err = 0.0
                r = planner.rounding_step(t, t.maxabs)
                for s in range(t.n_passes):
                    if t.progressive[s]:
                        err = err + planner.term(t, s, int(plan[s]), r)
                assert abs(err - best[0]) <= 1e-12 * max(1.0, best[0])
                # every loaded byte counts, the planes loaded before included
                assert _loaded(t, plan) <= np.floor(bt)


def test_bitrate_refinement_budget_and_noop_rule():
    x = fieldgen.grf((24, 40, 33), -5.0 / 6.0, seed=3, dtype=np.float32)
    eb = 1e-5 * fieldgen.value_range(x)
    buf = codec.compress(x, eb)
    _, _, t = codec.open_stream(buf)
    n = x.size
    st0 = codec.retrieve(buf, "bitrate", 2.0)
    held = _loaded(t, st0.plan)
    assert held <= 2.0 * n / 8.0
    seen_noop = seen_refined = 0
    # budgets just around the loaded bytes, then well above them
    for br in [8.0 * (held + d) / n for d in (-4096, -64, -1, 0, 1, 64, 4096)] + [3.0, 4.0, 6.0]:
        st = codec.retrieve_with_plan(buf, st0.plan, "bitrate", 2.0)
        old = st.plan.copy()
        st = codec.refine(st, "bitrate", br)
        budget = int(np.floor(br * n / 8.0))
        if budget < held:
            assert st.flags & planner.FLAG_NOOP and st.bytes_read == 0
            assert np.array_equal(st.plan, old)
            seen_noop += 1
            continue
        assert np.all(st.plan <= old)
        if np.array_equal(st.plan, old):
            assert st.flags & planner.FLAG_NOOP and st.bytes_read == 0
        else:
            assert not st.flags & planner.FLAG_NOOP
            seen_refined += 1
            # total loaded bytes within the budget; only the new planes read
            assert _loaded(t, st.plan) <= budget
            assert st.bytes_read == _loaded(t, st.plan) - held
            fresh = codec.retrieve_with_plan(buf, st.plan)
            assert st.field.tobytes() == fresh.field.tobytes()
    assert seen_noop >= 3 and seen_refined >= 2


def test_refinement_matches_fresh_optimum_when_it_fits_the_limit():
    x = fieldgen.grf((24, 40, 33), -5.0 / 6.0, seed=5, dtype=np.float32)
    r = fieldgen.value_range(x)
    buf = codec.compress(x, 1e-6 * r)
    _, _, t = codec.open_stream(buf)
    hits = 0
    for e1, e2 in [(1e-2, 1e-3), (1e-2, 1e-4), (1e-3, 1e-4), (1e-3, 1e-5), (1e-4, 1e-5)]:
        p1, _ = planner.plan_error_bound(t, e1 * r)
        p2, _ = planner.plan_error_bound(t, e2 * r)
        pr, _ = planner.plan_error_bound(t, e2 * r, limit=p1)
        assert np.all(pr <= p1)
        assert planner.bound_of(t, pr, t.maxabs + e2 * r) <= e2 * r
        # the restricted optimum never saves more than the unrestricted one
        assert _saved(t, pr) <= _saved(t, p2)
        if np.all(p2 <= p1):
            assert _saved(t, pr) == _saved(t, p2)
            hits += 1
    assert hits >= 2
