"""Entropy stage on the GPU (gpu): coded streams byte-exact against the
oracle's, coded streams the oracle wrote decoded on the device, and the
planner's coded plane sizes driving the same plans as the oracle's."""

import numpy as np
import pytest

import fieldgen
from oracle import codec
from oracle.stream import entropy_code_stream

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


# (name, field maker, relative eb): the fused 3-D path, the per-pass 2-D and
# 1-D paths, float64, a rough field whose low planes stay raw, and a masked
# climate crop whose planes code well
CASES = [
    ("grf3d", lambda: fieldgen.grf((40, 70, 200), -5.0 / 6.0, seed=31, dtype=np.float32), 1e-4),
    ("climate2d", lambda: fieldgen.climate_2d(1)[300:700, 900:1700].copy(), 1e-3),
    ("line1d", lambda: fieldgen.random_field((5000,), seed=32, dtype=np.float32), 1e-5),
    ("lognormal_f64", lambda: fieldgen.lognormal((33, 48, 50), seed=3), 1e-5),
    ("rough", lambda: fieldgen.grf((24, 40, 64), -5.0 / 6.0, seed=33, dtype=np.float32), 1e-7),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: c[0])
def test_device_coding_matches_oracle(ctx, case):
    name, make, rel = case
    x = make()
    eb = rel * fieldgen.value_range(x)
    print(f"case {name} {x.shape} {x.dtype} eb={eb}", flush=True)
    ref = codec.compress(x, eb)
    coded_ref = entropy_code_stream(ref)
    s = ctx.compress(_dev(x), eb)
    assert s.to_bytes() == ref
    full = s.retrieve(eb=eb)
    before = _bytes(full.tensor())
    full.free()
    s.entropy_code()
    assert s.coding == 1
    assert s.nbytes == len(coded_ref)
    assert s.to_bytes() == coded_ref
    s.entropy_code()  # already coded: unchanged
    assert s.to_bytes() == coded_ref
    # the resident planes are unchanged; plans now count coded bytes
    st = s.retrieve(eb=eb)
    assert _bytes(st.tensor()) == before
    st.free()
    for br in (1.0, 2.0, 4.0):
        st = s.retrieve(bitrate=br)
        o = codec.retrieve(coded_ref, "bitrate", br)
        assert st.plan == list(o.plan)
        assert _bytes(st.tensor()) == o.field.tobytes()
        assert st.info.bytes_read == o.bytes_read
        st.free()
    s.free()


@pytest.mark.parametrize("case", CASES[:2], ids=lambda c: c[0])
def test_oracle_coded_stream_decoded_on_device(ctx, case):
    name, make, rel = case
    x = make()
    eb = rel * fieldgen.value_range(x)
    coded = entropy_code_stream(codec.compress(x, eb))
    s = ctx.stream_from_bytes(coded)
    assert s.coding == 1
    assert s.to_bytes() == coded
    rng = np.random.default_rng(5)
    for trial in range(3):
        plan = [int(b) if s.pass_info(i)["progressive"] else 0
                for i, b in enumerate(rng.integers(0, 20, size=s.n_passes))]
        st = s.retrieve_plan(plan)
        o = codec.retrieve_with_plan(coded, plan)
        assert _bytes(st.tensor()) == o.field.tobytes()
        st.free()
    r = fieldgen.value_range(x)
    st = s.retrieve(eb=1e-1 * r)
    st.refine(eb=1e2 * eb)
    fresh = codec.retrieve(coded, "eb", 1e2 * eb)
    assert st.plan == list(fresh.plan)
    assert _bytes(st.tensor()) == fresh.field.tobytes()
    st.free()
    s.free()


def test_climate_full_size_coded(ctx):
    """A full 1800 x 3600 climate field (30 % masked): coded stream equal to the
    oracle's; bitrate retrievals at 1, 2, 4 bits per value count coded bytes."""
    x = fieldgen.climate_2d(1)
    eb = 1e-3 * fieldgen.value_range(x)
    s = ctx.compress(_dev(x), eb)
    raw_bytes = s.nbytes
    s.entropy_code()
    got = s.to_bytes()
    coded_ref = entropy_code_stream(codec.compress(x, eb))
    assert got == coded_ref
    assert len(got) < raw_bytes
    for br in (1.0, 2.0, 4.0):
        st = s.retrieve(bitrate=br)
        o = codec.retrieve(coded_ref, "bitrate", br)
        assert st.plan == list(o.plan)
        assert _bytes(st.tensor()) == o.field.tobytes()
        assert st.info.bytes_loaded <= br * x.size / 8 or st.info.flags & pkg.IPC_FLAG_BUDGET_BELOW_MIN
        st.free()
    s.free()


def test_benchmark_field_coded_round_trip(ctx):
    """512^3 float32 at 1e-4 * range: coded on the device, serialized, loaded
    back and decoded on the device; every plane and the full reconstruction
    survive, and the coded form is smaller."""
    x = fieldgen.grf_torch((512, 512, 512), -5.0 / 6.0, 0)
    r = float(x.max().double() - x.min().double())
    s = ctx.compress(x, 1e-4 * r)
    raw = s.to_bytes()
    s.entropy_code()
    coded = s.to_bytes()
    assert len(coded) < len(raw)
    assert coded[11] == 1 and raw[11] == 0 and coded[12:80] == raw[12:80]
    s2 = ctx.stream_from_bytes(coded)
    a = s.retrieve(eb=1e-4 * r)
    b = s2.retrieve(eb=1e-4 * r)
    assert a.plan == b.plan
    assert torch.equal(a.tensor(), b.tensor())
    a.free()
    b.free()
    # decoded planes equal the raw ones: the loaded stream serializes raw the
    # same way after the round trip of its coded form
    s3 = ctx.stream_from_bytes(raw)
    for br in (1.0, 3.0):
        a = s2.retrieve(bitrate=br)
        plan = a.plan
        c = s3.retrieve_plan(plan)
        assert torch.equal(a.tensor(), c.tensor())
        a.free()
        c.free()
    s3.free()
    s2.free()
    s.free()
