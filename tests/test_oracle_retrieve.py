"""Pins of the oracle's retrieval, planner and refinement (not gpu).

* Full retrieval reproduces the compressor's reconstruction bit for bit
  (Alg. 1 with every plane; Sec. 4.2.2).
* Thm. 1 (per-pass reading): the measured error of random partial plans stays
  within the bound; the per-level reading of the printed theorem fails on a
  two-dimensional counterexample.
* Sec. 5.2 / 5.3 planners equal an exhaustive search over every plan on tiny
  instances, including tie-breaks; retrievals meet their targets.
* Alg. 2 refinement reads only new planes and equals a fresh retrieval.
"""

import itertools

import numpy as np
import pytest

import fieldgen
from oracle import codec, coding, planner, predict, schedule
from oracle.stream import StreamError, parse_stream


def _field(shape, dtype, seed=0):
    return fieldgen.random_field(shape, seed=seed, dtype=dtype)


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("interp", [predict.LINEAR, predict.CUBIC])
@pytest.mark.parametrize("shape", [(200,), (30, 41), (9, 17, 33), (1, 1, 1)])
def test_full_retrieval_is_bit_identical(shape, interp, dtype):
    x = _field(shape, dtype)
    eb = max(1e-4 * fieldgen.value_range(x), 1e-6)
    buf, dbg = codec.compress(x, eb, interp=interp, debug=True)
    st = codec.retrieve(buf, "eb", eb)
    assert np.all(st.plan == 0)
    assert st.field.tobytes() == dbg.xhat.tobytes()
    assert st.bound == eb
    ps = parse_stream(buf)
    assert st.bytes_read == 4 * ps.payload.size


def _random_plans(P, rng, n):
    for _ in range(n):
        plan = rng.integers(0, 33, P)
        plan[0] = 0
        yield plan


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("interp", [predict.LINEAR, predict.CUBIC])
def test_bound_holds_for_random_plans(interp, dtype):
    rng = np.random.default_rng(4)
    for shape in [(65,), (17, 33), (9, 9, 17)]:
        x = _field(shape, dtype, seed=len(shape))
        eb = 1e-4 * fieldgen.value_range(x)
        buf = codec.compress(x, eb, interp=interp)
        _, _, t = codec.open_stream(buf)
        for plan in _random_plans(t.n_passes, rng, 40):
            plan = np.minimum(plan, rng.integers(0, 12, plan.size))
            st = codec.retrieve_with_plan(buf, plan)
            err = np.max(np.abs(st.field.astype(np.float64) - x.astype(np.float64)))
            bound = planner.bound_of(t, plan, t.maxabs + 2 * err + 1.0)
            assert err <= bound


def test_per_level_reading_of_theorem_fails_in_2d():
    """The printed bound with one group per level is not an upper bound in 2-D.

    Level 1 of a 3 x 3 grid with linear interpolation: pass along dim 0 predicts
    (1,0) and (1,2); pass along dim 1 then predicts (1,1) from them.  Codes of 1
    at those three points with the least significant plane dropped give a
    centre error of about 2 * (2 eb), above the per-level bound eb + 2 eb; the
    per-pass bound (amplification p per later pass) holds.
    """
    eb = 0.5
    x = np.zeros((3, 3), dtype=np.float64)
    x[1, 0] = 1.0
    x[1, 2] = 1.0
    x[1, 1] = 2.0
    buf, dbg = codec.compress(x, eb, interp=predict.LINEAR, debug=True)
    assert dbg.codes[1].tolist() == [[1, 1]]            # level 1, pass along dim 0
    assert dbg.codes[2].tolist() == [[0], [1], [0]]     # level 1, pass along dim 1
    _, _, t = codec.open_stream(buf)
    assert t.n_passes == 3
    plan = np.array([0, 1, 1])
    st = codec.retrieve_with_plan(buf, plan)
    err = float(np.max(np.abs(st.field - x)))
    assert err == 2.0
    # one group for the whole level, p^0 = 1: eb + 2 eb * max delta-y
    per_level = eb + 1 * (2 * eb) * max(t.errq[1][1], t.errq[2][1])
    assert err > per_level
    assert err <= planner.bound_of(t, plan, t.maxabs + 3.0)


def _exhaustive_eb(t, E, limit=None):
    """Best plan by enumeration under the planner's own integer costs."""
    R = E - t.eb
    u = R / planner.G_UNITS
    r = planner.rounding_step(t, t.maxabs + E)
    choices = []
    for s in range(t.n_passes):
        opts = []
        for b in planner._allowed(t, s, limit):
            tv = planner.term(t, s, b, r) if t.progressive[s] else 0.0
            qv = tv / u if u > 0 else np.inf
            c = 0 if tv == 0.0 else (int(np.floor(qv)) + 1 if qv < planner.G_UNITS else planner.G_UNITS + 1)
            if c > planner.G_UNITS:
                continue
            saved = int(np.sum(t.sizes[s, :b])) if t.progressive[s] else 0
            opts.append((b, c, saved))
        choices.append(opts)
    best = None
    # enumerate with the last pass slowest: the first optimum found is the
    # plan with the smallest b in the last pass, then the one before, ...
    for rcombo in itertools.product(*reversed(choices)):
        combo = rcombo[::-1]
        cost = sum(o[1] for o in combo)
        if cost > planner.G_UNITS:
            continue
        saved = sum(o[2] for o in combo)
        if best is None or saved > best[0]:
            best = (saved, [o[0] for o in combo])
    return best


def _exhaustive_br(t, bitrate):
    bt = bitrate * t.n_points / 8.0
    if bt >= t.total_bytes:
        return (0.0, [0] * t.n_passes)
    budget = int(np.floor(bt)) - t.fixed_bytes
    ub = max(1, -(-budget // planner.G_UNITS))
    cap = budget // ub
    r = planner.rounding_step(t, t.maxabs)
    choices = []
    for s in range(t.n_passes):
        opts = []
        for b in planner._allowed(t, s, None):
            if t.progressive[s]:
                lc = -(-int(np.sum(t.sizes[s, b:])) // ub)
                tv = planner.term(t, s, b, r)
            else:
                lc, tv = 0, 0.0
            if lc <= cap:
                opts.append((b, lc, tv))
        choices.append(opts)
    best = None
    for combo in itertools.product(*choices):
        if sum(o[1] for o in combo) > cap:
            continue
        err = 0.0
        for o in combo:
            err = err + o[2]
        if best is None or err < best[0]:
            best = (err, [o[0] for o in combo])
    return best


@pytest.mark.parametrize("interp", [predict.LINEAR, predict.CUBIC])
def test_planners_equal_exhaustive_search(interp):
    # anchors + 2 progressive passes -> 33^2 plans each
    x = fieldgen.random_field((5,), seed=1, dtype=np.float64, scale=50.0, smooth=False)
    x2 = fieldgen.random_field((3, 2), seed=2, dtype=np.float64, scale=50.0, smooth=False)
    for xx in (x, x2):
        eb = 1e-3
        buf = codec.compress(xx, eb, interp=interp)
        _, _, t = codec.open_stream(buf)
        assert t.n_passes == 3
        saved_of = lambda plan: sum(int(np.sum(t.sizes[s, :plan[s]])) for s in range(t.n_passes) if t.progressive[s])
        for E in (1e-3, 2e-3, 1e-2, 0.1, 1.0, 10.0, 1e3):
            plan, flags = planner.plan_error_bound(t, E)
            best = _exhaustive_eb(t, E)
            assert saved_of(plan) == best[0]
            assert list(plan) == best[1]   # same tie-break
            assert planner.bound_of(t, plan, t.maxabs + E) <= E
        for br in (0.5, 2.0, 8.0, 20.0, 64.0):
            plan, flags = planner.plan_bitrate(t, br)
            if flags & planner.FLAG_BUDGET_BELOW_MIN:
                continue
            best = _exhaustive_br(t, br)
            err = 0.0
            r = planner.rounding_step(t, t.maxabs)
            for s in range(t.n_passes):
                err = err + (planner.term(t, s, int(plan[s]), r) if t.progressive[s] else 0.0)
            assert abs(err - best[0]) <= 1e-12 * max(1.0, best[0])
            assert planner.loaded_bytes(t, plan) <= np.floor(br * t.n_points / 8.0)


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_retrieval_meets_error_targets(dtype):
    x = fieldgen.blobs_64(n=33, dtype=dtype)
    rng = fieldgen.value_range(x)
    eb = 1e-5 * rng
    buf = codec.compress(x, eb, interp=predict.CUBIC)
    prev = None
    for rel in (1e-1, 1e-2, 1e-3, 1e-4, 1e-5, 1e-6):
        E = rel * rng
        st = codec.retrieve(buf, "eb", E)
        err = float(np.max(np.abs(st.field.astype(np.float64) - x.astype(np.float64))))
        assert err <= st.bound <= max(E, eb)
        if prev is not None:
            assert st.bytes_read >= prev
        prev = st.bytes_read


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_retrieval_meets_bitrate_targets(dtype):
    x = fieldgen.climate_2d(1, shape=(90, 180), dtype=dtype)
    eb = 1e-3 * fieldgen.value_range(x)
    buf = codec.compress(x, eb, interp=predict.CUBIC)
    _, _, t = codec.open_stream(buf)
    prev = np.inf
    for br in (0.25, 1.0, 2.0, 4.0, 8.0):
        st = codec.retrieve(buf, "bitrate", br)
        loaded = planner.loaded_bytes(t, st.plan)
        if not st.flags & planner.FLAG_BUDGET_BELOW_MIN:
            assert loaded <= br * x.size / 8.0
        err = float(np.max(np.abs(st.field.astype(np.float64) - x.astype(np.float64))))
        assert err <= st.bound
        assert st.bound <= prev
        prev = st.bound


@pytest.mark.parametrize("mode,chain", [("eb", [1e-1, 1e-2, 1e-3, 1e-4]),
                                        ("bitrate", [0.5, 1.0, 3.0, 6.0])])
def test_refine_chain_equals_fresh_retrieve(mode, chain):
    x = fieldgen.grf((24, 40, 33), -5.0 / 6.0, seed=3, dtype=np.float32)
    r = fieldgen.value_range(x)
    eb = 1e-4 * r
    buf = codec.compress(x, eb)
    vals = [v * r for v in chain] if mode == "eb" else chain
    st = codec.retrieve(buf, mode, vals[0])
    total_read = st.bytes_read
    for v in vals[1:]:
        old_plan = st.plan.copy()
        st = codec.refine(st, mode, v)
        total_read += st.bytes_read
        assert np.all(st.plan <= old_plan)
        fresh = codec.retrieve_with_plan(buf, st.plan)
        assert st.field.tobytes() == fresh.field.tobytes()
        err = float(np.max(np.abs(st.field.astype(np.float64) - x.astype(np.float64))))
        assert err <= st.bound
        # only new planes were read: the chain never reads more than a fresh load
        assert total_read == fresh.bytes_read
    if mode == "eb":
        st2 = codec.refine(st, "eb", vals[-1] * 10)
        assert st2.flags & planner.FLAG_NOOP and st2.bytes_read == 0


def test_special_cases():
    # nothing progressive loaded: pure interpolation of anchors (+ outliers)
    x = fieldgen.random_field((33, 33), seed=9, dtype=np.float64)
    buf = codec.compress(x, 1e-3, interp=predict.LINEAR)
    _, _, t = codec.open_stream(buf)
    plan = np.full(t.n_passes, 32)
    plan[0] = 0
    st = codec.retrieve_with_plan(buf, plan)
    a = st.field[::32, ::32]
    assert np.allclose(st.field[0, 16], (a[0, 0] + a[0, 1]) * 0.5, rtol=0, atol=0)
    # constant field: every code 0, every plane absent
    c = np.full((17, 9, 40), 3.25, dtype=np.float32)
    buf, dbg = codec.compress(c, 1e-2, debug=True)
    ps = parse_stream(buf)
    assert np.all(ps.masks[1:] == 0)
    assert ps.payload.size == bin(int(ps.masks[0])).count("1")   # the one anchor's planes
    assert all(np.all(q == 0) for q in dbg.codes[1:])


def test_determinism_and_nonprog_levels():
    x = _field((20, 21, 22), np.float32, seed=8)
    eb = 1e-3
    assert codec.compress(x, eb) == codec.compress(x, eb)
    buf = codec.compress(x, eb, nonprog_levels=2)
    st = codec.retrieve(buf, "eb", 1e3)
    ps = parse_stream(buf)
    sched = schedule.make_schedule(x.shape)
    for p in sched.passes:
        if p.level > ps.header.K - 2 or p.index == 0:
            assert st.plan[p.index] == 0


def test_stream_validation():
    x = _field((10, 10), np.float64)
    buf = codec.compress(x, 1e-2)
    parse_stream(buf)
    with pytest.raises(StreamError):
        parse_stream(buf[:-8])
    with pytest.raises(StreamError):
        parse_stream(b"XXXX" + buf[4:])
    with pytest.raises(StreamError):
        parse_stream(buf[:100])


@pytest.mark.parametrize("shape,dtype", [((40, 33), np.float32), ((9, 17, 33), np.float64)])
def test_errq_bound_mode_changes_only_the_table_and_keeps_targets(shape, dtype):
    """errq_mode="bound": the stream equals the exact one except for its
    delta-y rows, which are the fixed table; plans built on it meet their
    targets and load at least as much as plans on the measured table."""
    x = _field(shape, dtype, seed=9)
    r = fieldgen.value_range(x)
    eb = 1e-5 * r
    a = parse_stream(codec.compress(x, eb))
    bbuf = codec.compress(x, eb, errq_mode="bound")
    b = parse_stream(bbuf)
    assert np.array_equal(a.masks, b.masks) and np.array_equal(a.payload, b.payload)
    assert np.array_equal(a.out_keys, b.out_keys) and a.out_vals.tobytes() == b.out_vals.tobytes()
    assert all(np.array_equal(row, coding.errq_bound_table()) for row in b.errq)
    exact = codec.compress(x, eb)
    for rel in (1e-1, 1e-2, 1e-3, 1e-4):
        E = rel * r
        st = codec.retrieve(bbuf, "eb", E)
        err = np.max(np.abs(st.field.astype(np.float64) - x.astype(np.float64)))
        assert err <= st.bound <= E
        assert st.bytes_read >= codec.retrieve(exact, "eb", E).bytes_read
