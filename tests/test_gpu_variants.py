"""The paper's variants on the GPU (gpu): per-level plane groups in the
planner, and the additive form of Alg. 2, each byte-exact against the
oracle's variant."""

import numpy as np
import pytest

import fieldgen
from oracle import codec

torch = pytest.importorskip("torch")
pkg = pytest.importorskip("paper_2502_04093_amd")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = pkg.Context(0)
    yield c
    c.close()


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")


def _bytes(t):
    return t.detach().cpu().numpy().tobytes()


CASES = [
    ("grf3d_f32", lambda: fieldgen.grf((40, 70, 200), -5.0 / 6.0, seed=41, dtype=np.float32), 1e-6),
    ("climate2d", lambda: fieldgen.climate_2d(1)[200:600, 1000:1700].copy(), 1e-5),
    ("line1d", lambda: fieldgen.random_field((20000,), seed=42, dtype=np.float32), 1e-6),
    ("grf3d_f64", lambda: fieldgen.grf((33, 48, 50), -5.0 / 6.0, seed=43, dtype=np.float64), 1e-10),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: c[0])
def test_additive_refine_matches_oracle(ctx, case):
    name, make, rel = case
    x = make()
    r = fieldgen.value_range(x)
    eb = rel * r
    print(f"case {name} {x.shape} {x.dtype}", flush=True)
    ref = codec.compress(x, eb)
    s = ctx.compress(_dev(x), eb)
    st = s.retrieve(eb=1e-1 * r)
    o = codec.retrieve(ref, "eb", 1e-1 * r)
    assert st.plan == list(o.plan)
    steps = [("eb", 1e-2 * r), ("bitrate", 6.0), ("eb", 1e-4 * r), ("eb", 30 * eb), ("eb", eb)]
    for mode, v in steps:
        info = st.refine_additive(**{mode: v})
        o = codec.refine_additive(o, mode, v)
        assert st.plan == list(o.plan), (mode, v)
        assert info.bound == o.bound
        assert info.bytes_read == o.bytes_read
        assert _bytes(st.tensor()) == o.field.tobytes(), (mode, v)
    err = float((st.tensor().double() - _dev(x).double()).abs().max())
    assert err <= st.info.bound
    st.free()
    s.free()


@pytest.mark.parametrize("case", CASES[:2], ids=lambda c: c[0])
def test_level_groups_match_oracle(ctx, case):
    name, make, rel = case
    x = make()
    r = fieldgen.value_range(x)
    eb = rel * r
    ref = codec.compress(x, eb)
    s = ctx.compress(_dev(x), eb)
    for mode, v in (("eb", 1e-2 * r), ("eb", 1e-4 * r), ("bitrate", 2.0), ("bitrate", 8.0)):
        st = s.retrieve(level_groups=True, **{mode: v})
        o = codec.retrieve(ref, mode, v, level_groups=True)
        assert st.plan == list(o.plan)
        assert st.info.bound == o.bound
        assert _bytes(st.tensor()) == o.field.tobytes()
        st.free()
    # refinement with level groups (recompute form and additive form)
    st = s.retrieve(eb=1e-2 * r, level_groups=True)
    o = codec.retrieve(ref, "eb", 1e-2 * r, level_groups=True)
    st.refine(eb=1e-4 * r, level_groups=True)
    o = codec.refine(o, "eb", 1e-4 * r, level_groups=True)
    assert st.plan == list(o.plan)
    assert _bytes(st.tensor()) == o.field.tobytes()
    st.refine_additive(eb=1e-5 * r, level_groups=True)
    o = codec.refine_additive(o, "eb", 1e-5 * r, level_groups=True)
    assert st.plan == list(o.plan)
    assert _bytes(st.tensor()) == o.field.tobytes()
    st.free()
    s.free()
