"""GPU parity at the sizes where the fused level kernels run multi-step
columns (several chunk rows per workgroup, the coarse-plane ring, prefetch of
the next step), and on streams the oracle wrote (packed payload placement)
(gpu).

Byte-exact against the oracle up to 33.5 M points.  The 512^3 benchmark field
and the full-shape float64 batch are checked on sampled outputs, each
evaluated by the pointwise oracle through its dependency cone, and through
properties that hold at any size: the error bound of every retrieval,
refinement equal to a fresh retrieval, determinism.
"""

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


# (shape, dtype, seed, relative eb, special values): level-1 columns of 16
# (512 x 256 x 256), 8 with a ragged last segment (300 x 200 x 260) and 4 in
# float64 (200 x 130 x 260)
MULTI = [
    ((512, 256, 256), np.float32, 3, 1e-4, False, "cubic"),
    ((300, 200, 260), np.float32, 4, 1e-4, True, "cubic"),
    ((200, 130, 260), np.float64, 5, 1e-6, True, "cubic"),
    # linear interpolation with multi-step columns (coarse-plane ring, prefetch)
    ((512, 256, 256), np.float32, 6, 1e-4, False, "linear"),
    ((300, 200, 260), np.float32, 7, 1e-5, True, "linear"),
]


@pytest.mark.parametrize("case", MULTI, ids=lambda c: f"{'x'.join(map(str, c[0]))}-{np.dtype(c[1]).name}-{c[5]}")
def test_multistep_columns_match_oracle(ctx, case):
    shape, dt, seed, rel, special, interp = case
    x = fieldgen.grf(shape, -5.0 / 6.0, seed=seed, dtype=dt)
    if special:
        f = x.reshape(-1)
        f[12345] = np.nan
        f[f.size // 3] = np.inf
        f[f.size // 2 + 7] = dt(3e37) if dt == np.float32 else 3e300
    r = fieldgen.value_range(np.nan_to_num(x, posinf=0, neginf=0))
    eb = rel * r
    print(f"case {shape} {np.dtype(dt).name} {interp} eb={eb}", flush=True)
    ref, dbg = codec.compress(x, eb, interp=1 if interp == "cubic" else 0, debug=True)
    s = ctx.compress(_dev(x), eb, interp=interp)
    assert s.to_bytes() == ref
    st = s.retrieve(eb=eb)
    assert _bytes(st.tensor()) == dbg.xhat.tobytes()
    st.free()
    st = s.retrieve(eb=1e2 * eb)
    o = codec.retrieve(ref, "eb", 1e2 * eb)
    assert st.plan == list(o.plan)
    assert _bytes(st.tensor()) == o.field.tobytes()
    st.free()
    s.free()


@pytest.mark.parametrize("rel", [1e-3, 1e-7])
def test_oracle_stream_fused_packed_placement(ctx, rel):
    """A 3-D stream the oracle wrote, retrieved by the fused kernels from the
    packed placement; at 1e-7 * range the codes pass 2^16 (the full-width
    plane transposes), at 1e-3 they stay below it."""
    x = fieldgen.random_field((40, 70, 200), seed=21, dtype=np.float32)
    eb = rel * fieldgen.value_range(x)
    ref = codec.compress(x, eb)
    s = ctx.stream_from_bytes(ref)
    assert s.to_bytes() == ref
    for plan_seed in range(4):
        draw = np.random.default_rng(100 + plan_seed).integers(0, 20, size=s.n_passes)
        plan = [int(b) if s.pass_info(i)["progressive"] else 0 for i, b in enumerate(draw)]
        if plan_seed == 0:
            plan = [0] * s.n_passes
        st = s.retrieve_plan(plan)
        o = codec.retrieve_with_plan(ref, plan)
        assert _bytes(st.tensor()) == o.field.tobytes()
        st.free()
    for br in (1.0, 4.0):
        st = s.retrieve(bitrate=br)
        o = codec.retrieve(ref, "bitrate", br)
        assert st.plan == list(o.plan)
        assert _bytes(st.tensor()) == o.field.tobytes()
        st.free()
    s.free()


def test_benchmark_field_properties(ctx):
    """The 512^3 float32 field of the benchmark, compressed at 1e-4 * range in
    the benchmark's launch configuration."""
    x = fieldgen.grf_torch((512, 512, 512), -5.0 / 6.0, 0)
    r = float(x.max().double() - x.min().double())
    eb = 1e-4 * r
    s = ctx.compress(x, eb)
    a = s.to_bytes()
    s2 = ctx.compress(x, eb)
    assert s2.to_bytes() == a
    s2.free()
    xd = x.double()
    for rel in (1e-4, 1e-3, 1e-2):
        st = s.retrieve(eb=rel * r)
        err = float((st.tensor().double() - xd).abs().max())
        assert err <= st.bound <= rel * r * (1 + 1e-12)
        st.free()
    st = s.retrieve(eb=1e-2 * r)
    st.refine(eb=1e-3 * r)
    fresh = s.retrieve(eb=1e-3 * r)
    assert st.plan == fresh.plan
    assert torch.equal(st.tensor(), fresh.tensor())
    fresh.free()
    st.free()
    s.free()


@pytest.mark.parametrize("index", [0, 1])
def test_climate_2d_full_size(ctx, index):
    """The 2-D configuration at full size (1800 x 3600 f32, eb = 1e-3 * range;
    field 1 has 30 % masked fill values), bitrate retrievals at 1, 2, 4 bits
    per value: stream and reconstructions byte-exact against the oracle."""
    x = fieldgen.climate_2d(index)
    eb = 1e-3 * fieldgen.value_range(x)
    ref = codec.compress(x, eb)
    s = ctx.compress(_dev(x), eb)
    assert s.to_bytes() == ref
    for br in (1.0, 2.0, 4.0):
        st = s.retrieve(bitrate=br)
        o = codec.retrieve(ref, "bitrate", br)
        assert st.plan == list(o.plan)
        assert _bytes(st.tensor()) == o.field.tobytes()
        assert st.info.bytes_loaded <= br * x.size / 8 or st.info.flags & pkg.IPC_FLAG_BUDGET_BELOW_MIN
        st.free()
    s.free()


def test_lognormal_f64(ctx):
    """The float64 log-normal recipe (heavy tailed) at 128 x 192 x 192, eb =
    1e-5 * range, byte-exact against the oracle; the full 256 x 384 x 384 shape
    is covered by the batched calls (equal to single calls)."""
    x = fieldgen.lognormal((128, 192, 192), seed=2)
    eb = 1e-5 * fieldgen.value_range(x)
    ref, dbg = codec.compress(x, eb, debug=True)
    s = ctx.compress(_dev(x), eb)
    assert s.to_bytes() == ref
    st = s.retrieve(eb=eb)
    assert _bytes(st.tensor()) == dbg.xhat.tobytes()
    st.free()
    st = s.retrieve(eb=1e3 * eb)
    o = codec.retrieve(ref, "eb", 1e3 * eb)
    assert _bytes(st.tensor()) == o.field.tobytes()
    st.free()
    s.free()


def test_lognormal_f64_full_shape_batched(ctx):
    xs = [fieldgen.lognormal_torch((256, 384, 384), seed=i) for i in range(2)]
    ebs = [1e-5 * float(x.max() - x.min()) for x in xs]
    bs = ctx.compress_batch(xs, ebs)
    for x, e, b in zip(xs, ebs, bs):
        one = ctx.compress(x, e)
        assert b.to_bytes() == one.to_bytes()
        st = b.retrieve(eb=e)
        err = float((st.tensor() - x).abs().max())
        assert err <= e
        st.free()
        one.free()
        b.free()


def _samples(shape, n, seed):
    """n random points plus the corners and points next to the upper faces
    (boundary stencil forms), as an int64 array [m, 3]."""
    rng = np.random.default_rng(seed)
    pts = [tuple(int(rng.integers(0, d)) for d in shape) for _ in range(n)]
    hi = [d - 1 for d in shape]
    pts += [(0, 0, 0), tuple(hi), (hi[0], 0, hi[2]), (1, 1, 1), (hi[0] - 1, hi[1] - 2, hi[2] - 3),
            (hi[0] // 2, hi[1], hi[2] // 2), (2, hi[1] - 1, 5)]
    return np.array(pts, dtype=np.int64)


def _at(t, pts):
    idx = torch.from_numpy(pts).to(t.device)
    return t[idx[:, 0], idx[:, 1], idx[:, 2]].cpu().numpy()


def _check_samples(st, cone, pts, plan, what):
    got = _at(st.tensor(), pts)
    ref = np.array([cone.retrieved(tuple(p), plan) for p in pts], dtype=got.dtype)
    bad = [i for i in range(len(pts)) if got[i].tobytes() != ref[i].tobytes()]
    assert not bad, (what, pts[bad[:5]].tolist(), got[bad[:5]], ref[bad[:5]])


def test_benchmark_field_sampled_parity(ctx):
    """The 512^3 float32 benchmark field at 1e-4 * range in the benchmark's
    launch configuration (column lengths autotuned as the benchmark does):
    sampled outputs of the full retrieval, of bitrate and error-bound
    retrievals and of a refinement, bit-exact against the pointwise oracle
    (each sample evaluated through its dependency cone)."""
    from oracle.pointwise import Cone

    x = fieldgen.grf_torch((512, 512, 512), -5.0 / 6.0, 0)
    r = float(x.max().double() - x.min().double())
    eb = 1e-4 * r
    ctx.autotune(x, eb)
    try:
        s = ctx.compress(x, eb)
        cone = Cone(x.cpu().numpy(), eb)
        # the plans are chosen independently by the oracle's planner from the
        # stream's serialized tables (its sampled bytes are pinned by the
        # cone: every pass's codes and delta-y are what the samples decode)
        _, _, tables = codec.open_stream(s.to_bytes())
        pts = _samples(x.shape, 160, 1)
        print(f"sampled parity 512^3 f32: {len(pts)} points", flush=True)
        st = s.retrieve(eb=eb)
        assert all(b == 0 for b in st.plan)
        got = _at(st.tensor(), pts)
        ref = np.array([cone.xhat(tuple(p)) for p in pts], dtype=np.float32)
        assert got.tobytes() == ref.tobytes()
        st.free()
        for kind, v in (("bitrate", 1.0), ("bitrate", 4.0), ("eb", 1e-2 * r)):
            st = s.retrieve(**{kind: v})
            oplan, _ = codec.make_plan(tables, kind, v)
            assert st.plan == [int(b) for b in oplan], (kind, v)
            _check_samples(st, cone, pts, oplan, (kind, v))
            st.free()
        st = s.retrieve(eb=1e-2 * r)
        old = list(st.plan)
        st.refine(eb=1e-3 * r)
        oplan, _ = codec.make_plan(tables, "eb", 1e-3 * r, limit=old)
        assert st.plan == [int(b) for b in oplan]
        _check_samples(st, cone, pts, oplan, "refine")
        st.free()
        print(f"cone points evaluated: {cone.cone_size()}", flush=True)
        s.free()
    finally:
        ctx.autotune_clear()


def test_lognormal_f64_full_shape_sampled_parity(ctx):
    """The float64 log-normal fields at their full 256 x 384 x 384 shape,
    compressed and retrieved as one batch: sampled outputs bit-exact against
    the pointwise oracle."""
    from oracle.pointwise import Cone

    xs = [fieldgen.lognormal_torch((256, 384, 384), seed=i) for i in range(2)]
    ebs = [1e-5 * float(x.max() - x.min()) for x in xs]
    bs = ctx.compress_batch(xs, ebs)
    sts = ctx.retrieve_batch(bs, bitrate=2.0)
    for k, (x, e, b, st) in enumerate(zip(xs, ebs, bs, sts)):
        cone = Cone(x.cpu().numpy(), e)
        pts = _samples(x.shape, 96, 10 + k)
        print(f"sampled parity 256x384x384 f64 field {k}: {len(pts)} points", flush=True)
        _check_samples(st, cone, pts, st.plan, ("batch bitrate", k))
        st.free()
        full = b.retrieve(eb=e)
        _check_samples(full, cone, pts, full.plan, ("full", k))
        full.free()
        b.free()
