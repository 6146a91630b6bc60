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


# ---------------------------------------------------------------------------
# Alg. 2 in its additive form


@pytest.mark.parametrize("interp", [predict.LINEAR, predict.CUBIC])
@pytest.mark.parametrize("shape", [(17, 33, 20), (65, 90), (700,)])
def test_additive_refine_exact_on_dyadic_data(interp, shape):
    """Integer data, eb = 1/2 (2 eb = 1), float64: every prediction, code and
    reconstruction is a short dyadic fraction, so all arithmetic is exact and
    the additive form must equal a fresh reconstruction bit for bit (any
    dropped or misplaced term of the difference field breaks this)."""
    rng = np.random.default_rng(len(shape) * 7 + interp)
    x = np.cumsum(rng.integers(-40, 41, size=shape), axis=-1).astype(np.float64)
    buf = codec.compress(x, 0.5, interp=interp)
    _, _, t = codec.open_stream(buf)
    plan = np.where(t.progressive, 20, 0)
    st = codec.retrieve_with_plan(buf, plan)
    for b in (14, 9, 5, 2, 0):
        target = np.where(t.progressive, np.minimum(plan, b), 0)
        # refine to an explicit plan through the error-bound planner's limit
        E = planner.bound_of(t, target, t.maxabs + 1e9)
        st = codec.refine_additive(st, "eb", E)
        fresh = codec.retrieve_with_plan(buf, st.plan)
        assert st.field.tobytes() == fresh.field.tobytes()
        plan = st.plan


@pytest.mark.parametrize("dt,rel", [(np.float32, 1e-6), (np.float64, 1e-10)])
def test_additive_refine_within_its_bound(dt, rel):
    x = fieldgen.grf((24, 40, 64), -5.0 / 6.0, seed=9, dtype=dt)
    r = fieldgen.value_range(x)
    buf = codec.compress(x, rel * r)
    st = codec.retrieve(buf, "eb", 1e-2 * r)
    total = st.bytes_read
    for e in (1e-3, 1e-4, 1e-5, rel):
        prev = st.bound
        st = codec.refine_additive(st, "eb", e * r)
        total += st.bytes_read
        fresh = codec.retrieve_with_plan(buf, st.plan, "eb", e * r)
        err = float(np.max(np.abs(st.field.astype(np.float64) - x)))
        assert err <= st.bound
        # the additive form differs from the fresh one by rounding only
        gap = float(np.max(np.abs(st.field.astype(np.float64) - fresh.field)))
        assert gap <= st.bound - fresh.bound
        assert st.bound >= fresh.bound and (st.bound < prev or st.flags)
    assert total == codec.retrieve_with_plan(buf, st.plan).bytes_read


def test_additive_refine_noop_and_outliers():
    """Outliers (NaN, inf, huge) keep their exact values through additive
    refinements; a target already met loads nothing."""
    x = fieldgen.random_field((30, 41), seed=4, dtype=np.float32)
    r = fieldgen.value_range(x)
    f = x.reshape(-1)
    f[10], f[500], f[900] = np.nan, np.inf, 3e37
    buf = codec.compress(x, 1e-6 * r)
    st = codec.retrieve(buf, "eb", 1e-2 * r)
    st = codec.refine_additive(st, "eb", 1e-5 * r)
    g = st.field.reshape(-1)
    assert np.isnan(g[10]) and g[500] == np.inf and g[900] == np.float32(3e37)
    b = st.bound
    st = codec.refine_additive(st, "eb", 2 * b)
    assert st.flags & planner.FLAG_NOOP and st.bytes_read == 0 and st.bound == b
