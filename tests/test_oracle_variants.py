"""Pins of the oracle's variants of the paper (CPU): the planner with the
paper's per-level plane groups (Sec. 4.3).

The grouped dynamic programs are checked against exhaustive enumeration of
every per-level plan on a stream small enough to enumerate, and the plans
they return must meet the per-pass bound of Thm. 1 on real retrievals."""

import itertools

import numpy as np
import pytest

import fieldgen
from oracle import codec, planner, predict


def _small_stream(interp):
    x = fieldgen.random_field((9, 9), seed=12, dtype=np.float64)
    eb = 1e-6 * fieldgen.value_range(x)
    return x, codec.compress(x, eb, interp=interp)


def _enumerate(t, groups, choose):
    """Every per-level plan, as (plan, per-group b) pairs."""
    opts = [list(planner._allowed(t, g, None)) for g in groups]
    for bs in itertools.product(*reversed(opts)):
        bs = bs[::-1]
        plan = np.zeros(t.n_passes, dtype=np.int64)
        for g, b in zip(groups, bs):
            plan[g] = b
        yield plan, bs


@pytest.mark.parametrize("interp", [predict.LINEAR, predict.CUBIC])
def test_level_groups_error_bound_exhaustive(interp):
    x, buf = _small_stream(interp)
    _, _, t = codec.open_stream(buf)
    groups = planner.plan_groups(t, True)
    assert len(groups) == 4 and [len(g) for g in groups] == [1, 2, 2, 2]
    for rel in (1e-5, 1e-4, 1e-3, 1e-2):
        E = rel * fieldgen.value_range(x)
        u = (E - t.eb) / planner.G_UNITS
        r = planner.rounding_step(t, t.maxabs + E)
        best = None
        for plan, bs in _enumerate(t, groups, None):
            cost = 0
            for g, b in zip(groups, bs):
                tv = sum(planner.term(t, s, b, r) for s in g if t.progressive[s])
                cost += 0 if tv == 0.0 else int(np.floor(tv / u)) + 1
            if cost > planner.G_UNITS:
                continue
            saved = sum(int(np.sum(t.sizes[s, :plan[s]])) for s in range(t.n_passes)
                        if t.progressive[s])
            if best is None or saved > best[0]:
                best = (saved, plan)
        plan, _ = planner.plan_error_bound(t, E, level_groups=True)
        assert np.array_equal(plan, best[1])
        assert planner.bound_of(t, plan, t.maxabs + E) <= E
        st = codec.retrieve_with_plan(buf, plan)
        assert float(np.max(np.abs(st.field - x))) <= planner.bound_of(t, plan, t.maxabs + E)


@pytest.mark.parametrize("interp", [predict.LINEAR, predict.CUBIC])
def test_level_groups_bitrate_exhaustive(interp):
    x, buf = _small_stream(interp)
    _, _, t = codec.open_stream(buf)
    groups = planner.plan_groups(t, True)
    for br in (4.0, 8.0, 16.0, 24.0):
        bt = br * t.n_points / 8.0
        if bt >= t.total_bytes:
            continue
        budget = int(np.floor(bt)) - t.fixed_bytes
        if budget < 0:
            continue
        ub = max(1, -(-budget // planner.G_UNITS))
        cap = budget // ub
        r = planner.rounding_step(t, t.maxabs)
        best = None
        for plan, bs in _enumerate(t, groups, None):
            lc = sum(-(-sum(int(np.sum(t.sizes[s, b:])) for s in g if t.progressive[s]) // ub)
                     for g, b in zip(groups, bs))
            if lc > cap:
                continue
            err = 0.0
            for g, b in zip(groups, bs):
                err = err + sum(planner.term(t, s, b, r) for s in g if t.progressive[s])
            if best is None or err < best[0]:
                best = (err, plan)
        plan, flags = planner.plan_bitrate(t, br, level_groups=True)
        assert flags == 0
        assert np.array_equal(plan, best[1])
        assert planner.loaded_bytes(t, plan) <= bt


def test_level_groups_cost_at_least_per_pass():
    """On a larger stream: at the same error bound the per-level plan is
    uniform within every level, meets the bound, and loads at least about as
    many bytes as the per-pass plan (within the budget's discretization)."""
    x = fieldgen.grf((24, 40, 64), -5.0 / 6.0, seed=8, dtype=np.float32)
    r = fieldgen.value_range(x)
    buf = codec.compress(x, 1e-6 * r)
    _, _, t = codec.open_stream(buf)
    for rel in (1e-5, 1e-4, 1e-3, 1e-2):
        E = rel * r
        pp, _ = planner.plan_error_bound(t, E)
        pl, _ = planner.plan_error_bound(t, E, level_groups=True)
        for g in planner.plan_groups(t, True):
            assert len(set(int(pl[s]) for s in g)) == 1
        assert planner.bound_of(t, pl, t.maxabs + E) <= E
        assert planner.loaded_bytes(t, pl) >= 0.97 * planner.loaded_bytes(t, pp)
