"""Pins of the oracle's schedule, stencils and quantizer (not gpu).

* Schedule (Sec. 4.1, Fig. "interp-design"): brute force over every point.
* Stencils (Eq. interp-linear, Eq. interp-cubic): the paper's coefficients, an
  independent Lagrange fit, the norm p of Thm. 1, and exact reproduction of
  integer polynomial fields.
* Quantizer (Sec. 4.2.2, Eq. error-prediction-interp): |x - x^| <= eb.
"""

import itertools
import json
import os

import numpy as np
import pytest

import fieldgen
from oracle import brute, codec, predict, schedule

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_examples.json")))

SHAPES = [(1,), (2,), (3,), (5,), (9,), (17,), (33,), (1, 1), (2, 3), (5, 9), (17, 5), (9, 17),
          (3, 3, 3), (5, 2, 9), (10, 11, 12), (33, 2, 65), (17, 17, 17), (1, 7, 1), (4, 1, 6)]


@pytest.mark.parametrize("dims", SHAPES)
def test_schedule_partitions_points(dims):
    sched = schedule.make_schedule(dims)
    K = sched.K
    assert K == brute.levels(dims)
    seen = np.full(dims, -1, dtype=np.int64)
    for p in sched.passes:
        if p.index == 0:
            grids = [np.arange(0, d, p.h) for d in dims]
        else:
            grids = schedule.fine_index_grids(sched, p)
        if p.n_targets == 0:
            continue
        sub = seen[np.ix_(*grids)]
        assert np.all(sub == -1), "point in two passes"
        seen[np.ix_(*grids)] = p.index
    assert np.all(seen >= 0), "point in no pass"
    for i in itertools.product(*[range(d) for d in dims]):
        s, lev, k = brute.pass_of_point(i, dims, K)
        assert seen[i] == s
        if s == 0:
            continue
        h = 1 << (lev - 1)
        for off in (-3, -1, 1, 3):
            j = list(i)
            j[k] += off * h
            if 0 <= j[k] < dims[k]:
                s2, _, _ = brute.pass_of_point(tuple(j), dims, K)
                assert s2 < s, "neighbour not reconstructed before its target"
        assert 0 <= i[k] - h  # the -1 neighbour always exists


@pytest.mark.parametrize("dims", SHAPES)
def test_chunk_order_is_a_permutation(dims):
    sched = schedule.make_schedule(dims, tuple([1] * len(dims)))
    for cl in (tuple([1] * len(dims)), schedule.DEFAULT_CHUNK_LOG2[len(dims)]):
        sched = schedule.make_schedule(dims, cl)
        for p in sched.passes:
            order = schedule.canonical_order(p)
            assert np.array_equal(np.sort(order), np.arange(p.n_targets))
            assert int(p.chunk_counts.sum()) == p.n_targets


def _apply(interp, vals, offsets, present):
    """Run the oracle stencil on one target whose neighbours hold ``vals``."""
    d = {o: v for o, v in zip(offsets, vals)}
    return float(predict.stencil_1d(interp, d.get(-1, 0.0), d.get(1, 0.0), d.get(-3, 0.0),
                                    d.get(3, 0.0), 1 in present, -3 in present, 3 in present,
                                    np.float64))


def _coefs(interp, present):
    offs = sorted(present)
    out = []
    for o in offs:
        vals = [1.0 if oo == o else 0.0 for oo in offs]
        out.append(_apply(interp, vals, offs, set(present)))
    return offs, out


def test_stencil_coefficients_match_paper():
    g = GOLDEN["interpolation_coefficients"]
    offs, c = _coefs(predict.LINEAR, {-1, 1})
    assert offs == g["linear"]["offsets"] and c == g["linear"]["coefficients"]
    offs, c = _coefs(predict.CUBIC, {-3, -1, 1, 3})
    assert offs == g["cubic"]["offsets"] and c == g["cubic"]["coefficients"]


@pytest.mark.parametrize("present", [{-3, -1, 1, 3}, {-1, 1, 3}, {-3, -1, 1}, {-1, 1}])
def test_stencils_are_lagrange_interpolants(present):
    # independent construction: the polynomial through the known offsets, at 0
    offs, c = _coefs(predict.CUBIC, present)
    fit_deg = len(offs) - 1
    for o, coef in zip(offs, c):
        y = [1.0 if oo == o else 0.0 for oo in offs]
        poly = np.polynomial.polynomial.Polynomial.fit(offs, y, fit_deg)
        assert abs(poly(0.0) - coef) < 1e-12
    g = GOLDEN["interpolation_norm"]
    assert sum(abs(v) for v in c) <= g["cubic"] + 1e-15
    _, cl = _coefs(predict.LINEAR, present)
    assert sum(abs(v) for v in cl) <= g["linear"] + 1e-15
    assert predict.amplification(predict.LINEAR) == g["linear"]
    assert predict.amplification(predict.CUBIC) == g["cubic"]


STENCIL_DEGREE = {"copy": 0, "linear": 1, "quad": 2, "cubic": 3}


def _stencil_kind(interp, t, dk, h):
    has_c = t + h < dk
    if not has_c:
        return "copy"
    if interp == predict.LINEAR:
        return "linear"
    has_a, has_e = t - 3 * h >= 0, t + 3 * h < dk
    if has_a and has_e:
        return "cubic"
    if has_a or has_e:
        return "quad"
    return "linear"


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("shape,degrees", [((17, 17), (3, 1)), ((17, 17), (1, 3)),
                                           ((9, 9, 17), (1, 2, 3)), ((33,), (3,)),
                                           ((16, 20), (2, 2)), ((17, 9, 9), (3, 0, 1))])
@pytest.mark.parametrize("interp", [predict.LINEAR, predict.CUBIC])
def test_polynomial_reproduction(shape, degrees, interp, dtype):
    x = fieldgen.poly_field(shape, degrees, seed=7, dtype=dtype)
    eb = 1.0 / 32.0
    buf, dbg = codec.compress(x, eb, interp=interp, debug=True)
    # prediction of exact integers is a multiple of 1/16 = 2 eb: nothing is lost
    assert np.array_equal(dbg.xhat, x)
    sched = schedule.make_schedule(shape)
    checked = 0
    for p in sched.passes[1:]:
        if p.n_targets == 0:
            continue
        q = dbg.codes[p.index]
        coords = [p.target_coords(j) * p.h for j in range(len(shape))]
        for idx in itertools.product(*[range(n) for n in p.tdims]):
            t = coords[p.dim][idx[p.dim]]
            kind = _stencil_kind(interp, t, shape[p.dim], p.h)
            if STENCIL_DEGREE[kind] >= degrees[p.dim]:
                assert q[idx] == 0, (p.index, idx, kind)
                checked += 1
    if interp == predict.CUBIC or min(degrees) <= 1:
        assert checked > 0


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("interp", [predict.LINEAR, predict.CUBIC])
def test_error_bound_everywhere(dtype, interp):
    for shape, rel in [((33, 17, 9), 1e-2), ((64, 64), 1e-4), ((1000,), 1e-6), ((12, 13, 14), 1e-3)]:
        x = fieldgen.random_field(shape, seed=5, dtype=dtype)
        eb = rel * fieldgen.value_range(x)
        buf, dbg = codec.compress(x, eb, interp=interp, debug=True)
        err = np.abs(dbg.xhat.astype(np.float64) - x.astype(np.float64))
        assert err.max() <= eb


def test_special_values_become_outliers():
    x = fieldgen.random_field((9, 10, 11), seed=3, dtype=np.float32)
    x[0, 0, 0] = np.nan
    x[4, 5, 6] = np.inf
    x[8, 9, 10] = -np.inf
    x[3, 3, 3] = np.float32(3e38)
    x[2, 2, 2] = np.float32(1e-42)   # subnormal
    x[1, 1, 1] = -0.0
    eb = 1e-3
    buf, dbg = codec.compress(x, eb, debug=True)
    same = (dbg.xhat.view(np.uint32) == x.view(np.uint32))
    assert same[0, 0, 0] and same[4, 5, 6] and same[8, 9, 10]
    fin = np.isfinite(x)
    assert np.all(np.abs(dbg.xhat[fin].astype(np.float64) - x[fin].astype(np.float64)) <= eb)
    n_out = sum(int(o.sum()) for o in dbg.outlier_masks)
    assert n_out >= 3
    st = codec.retrieve_with_plan(buf, np.zeros(len(dbg.codes), dtype=np.int64))
    assert np.array_equal(st.field.view(np.uint32), dbg.xhat.view(np.uint32))


def test_quantizer_scalar_matches_vector():
    rng = np.random.default_rng(11)
    for dt in (np.float32, np.float64):
        x = (rng.standard_normal(5000) * 10).astype(dt)
        pred = (x + rng.standard_normal(5000).astype(dt) * dt(0.3)).astype(dt)
        eb = 1e-3
        q, xh, out = predict.quantize(x, pred, eb)
        for i in range(0, 5000, 37):
            qs, xs, os_ = predict.quantize_scalar(x[i], pred[i], eb, dt)
            assert (qs, os_) == (int(q[i]), bool(out[i]))
            assert np.array([xs], dtype=dt).view(np.uint8).tobytes() == xh[i:i + 1].view(np.uint8).tobytes()
