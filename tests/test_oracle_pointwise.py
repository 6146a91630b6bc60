"""Pins of the pointwise oracle (CPU).

Every point of small ragged fields, evaluated one at a time through its
dependency cone, must equal the vectorized codec (compression reconstruction,
the multiset of codes and outliers of every pass, and retrievals with random
plans), and the scalar truncation by repeated division must equal the
mask-and-decode form.  These tie the pointwise evaluator, which the full-size
GPU checks rely on, to the rest of the pinned oracle.
"""

import itertools

import numpy as np
import pytest

import fieldgen
from oracle import codec, coding, predict
from oracle.pointwise import Cone, truncated_code

CASES = [
    ("3d_cubic_f32", (9, 13, 17), np.float32, predict.CUBIC, 1e-3),
    ("3d_linear_f64", (8, 11, 6), np.float64, predict.LINEAR, 1e-6),
    ("3d_pow2_plus1", (17, 17, 17), np.float32, predict.CUBIC, 1e-4),
    ("2d_cubic", (23, 40), np.float32, predict.CUBIC, 1e-3),
    ("1d_cubic_f64", (77,), np.float64, predict.CUBIC, 1e-9),
]


def _field(shape, dt, seed):
    x = fieldgen.grf(shape, -5.0 / 6.0, seed=seed, dtype=dt) if len(shape) > 1 else \
        fieldgen.random_field(shape, seed=seed, dtype=dt)
    return np.ascontiguousarray(x)


@pytest.mark.parametrize("case", CASES, ids=lambda c: c[0])
def test_every_point_matches_codec(case):
    name, shape, dt, interp, rel = case
    x = _field(shape, dt, seed=len(name))
    # a planted outlier (its code would exceed the quantizer's range)
    x.reshape(-1)[x.size // 3] = dt(3e30)
    eb = rel * float(np.ptp(x[np.abs(x) < 1e20]))
    buf, dbg = codec.compress(x, eb, interp=interp, debug=True)
    cone = Cone(x, eb, interp)
    pts = list(itertools.product(*[range(d) for d in shape]))
    got = np.array([cone.xhat(i) for i in pts], dtype=dt).reshape(shape)
    assert got.tobytes() == dbg.xhat.tobytes()
    # codes and outliers, pass by pass, as multisets
    by_pass = {}
    for i in pts:
        s = cone.pass_of(i)[0]
        q, _, out = cone.compressed(i)
        by_pass.setdefault(s, []).append((int(q), bool(out)))
    assert set(by_pass) <= set(range(len(dbg.codes)))
    n_out = 0
    for s in range(len(dbg.codes)):
        lst = by_pass.get(s, [])  # a pass can be empty on a small grid
        assert sorted(q for q, _ in lst) == sorted(int(v) for v in dbg.codes[s].reshape(-1))
        assert sum(o for _, o in lst) == int(dbg.outlier_masks[s].sum())
        n_out += sum(o for _, o in lst)
    assert n_out >= 1
    # retrievals with random plans, every point
    _, _, t = codec.open_stream(buf)
    rng = np.random.default_rng(len(name) + 1)
    for trial in range(3):
        plan = [int(rng.integers(0, 24)) for _ in range(t.n_passes)]
        ref = codec.retrieve_with_plan(buf, plan).field
        got = np.array([cone.retrieved(i, plan) for i in pts], dtype=dt).reshape(shape)
        assert got.tobytes() == ref.tobytes(), trial


def test_truncation_by_division_equals_mask_decode():
    rng = np.random.default_rng(4)
    qs = np.concatenate([rng.integers(-2 ** 30, 2 ** 30, size=300),
                         np.arange(-40, 41), [0x55555555, -0x2AAAAAAA, 2 ** 30, -2 ** 30]])
    e = coding.xor_encode(coding.to_negabinary(qs))
    for b in (0, 1, 2, 5, 13, 14, 20, 31, 32):
        ref = coding.truncated_codes(e, b)
        got = np.array([truncated_code(int(q), b) for q in qs], dtype=np.int64)
        assert np.array_equal(got, ref), b
    # b = 0 keeps the code; b = 32 clears it
    assert truncated_code(-7, 0) == -7 and truncated_code(-7, 32) == 0


def test_cone_is_small_on_a_large_grid():
    """The cone of a level-1 point of a 512^3 grid stays a few thousand points
    (the values do not matter for its size: a constant field is used)."""

    class Const:
        shape = (512, 512, 512)
        dtype = np.float32

        def __getitem__(self, i):
            return np.float32(1.0)

    cone = Cone(Const(), 1e-3)
    for i in [(511, 511, 511), (1, 1, 1), (255, 300, 101)]:
        cone.xhat(i)
    assert cone.cone_size() < 20000
