"""GPU parity: the HIP path through the C ABI against the oracle (gpu).

Every comparison is exact: serialized stream bytes, reconstructed values (as
bytes) and plans.  Inputs are seeded synthetic fields shared by both sides
(``fieldgen``); the oracle never sees anything the GPU produced except where a
test explicitly feeds an oracle-written stream to the GPU retrieval.
"""

import numpy as np
import pytest

import fieldgen
from oracle import codec, predict

torch = pytest.importorskip("torch")
pkg = pytest.importorskip("paper_2502_04093_amd")

pytestmark = pytest.mark.gpu

INTERP = {predict.LINEAR: "linear", predict.CUBIC: "cubic"}


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


def _case(shape, dtype, seed, special=False):
    x = fieldgen.random_field(shape, seed=seed, dtype=dtype)
    if special and x.size > 40:
        f = x.reshape(-1)
        f[3] = np.nan
        f[17] = np.inf
        f[-5] = -np.inf
        f[x.size // 2] = dtype(1e30) if dtype == np.float32 else 1e300
    return x


CASES = [
    ((1,), np.float32, predict.CUBIC, 1e-3, None, 0, False),
    ((2,), np.float64, predict.LINEAR, 1e-3, None, 0, False),
    ((5000,), np.float32, predict.CUBIC, 1e-4, None, 0, True),
    ((4097,), np.float64, predict.CUBIC, 1e-6, None, 0, False),
    ((33, 65), np.float32, predict.LINEAR, 1e-3, None, 0, False),
    ((100, 130), np.float32, predict.CUBIC, 1e-4, None, 0, True),
    ((31, 200), np.float64, predict.CUBIC, 1e-5, None, 1, False),
    ((9, 17, 33), np.float32, predict.CUBIC, 1e-3, None, 0, False),
    ((17, 33, 65), np.float64, predict.LINEAR, 1e-4, None, 0, True),
    ((20, 21, 70), np.float32, predict.CUBIC, 1e-5, (1, 2, 3), 0, True),
    ((40, 50, 130), np.float32, predict.CUBIC, 1e-4, None, 2, False),
    ((3, 1, 700), np.float32, predict.CUBIC, 1e-4, None, 0, False),
    ((2, 2, 2), np.float32, predict.CUBIC, 1e-3, None, 0, False),
    ((1, 1, 5), np.float64, predict.CUBIC, 1e-3, None, 0, False),
    ((5, 70, 130), np.float32, predict.CUBIC, 1e-4, None, 0, True),
    ((33, 17, 65), np.float64, predict.CUBIC, 1e-6, None, 0, True),
    ((64, 96, 200), np.float32, predict.LINEAR, 1e-5, None, 0, False),
    ((65, 33, 129), np.float32, predict.CUBIC, 1e-3, None, 1, True),
    # 2-D fields on the fused level kernels (one plane, pass A absent):
    # ragged multi-tile grids, degenerate rows and columns, an exact tile, and
    # the former 32 x 64 chunk on the per-pass kernels
    ((77, 300), np.float32, predict.LINEAR, 1e-4, None, 0, True),
    ((257, 1025), np.float32, predict.CUBIC, 1e-5, None, 1, False),
    ((130, 515), np.float64, predict.CUBIC, 1e-6, None, 0, True),
    ((1, 700), np.float64, predict.CUBIC, 1e-4, None, 0, False),
    ((700, 1), np.float32, predict.LINEAR, 1e-4, None, 0, False),
    ((16, 64), np.float32, predict.CUBIC, 1e-3, None, 0, False),
    ((100, 130), np.float32, predict.CUBIC, 1e-4, (5, 6), 0, True),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[0]}-{np.dtype(c[1]).name}-{INTERP[c[2]]}")
def test_compress_stream_bytes_and_full_retrieve(ctx, case):
    shape, dt, interp, rel, cl, npl, special = case
    x = _case(shape, dt, seed=sum(shape), special=special)
    eb = rel * max(fieldgen.value_range(np.nan_to_num(x, posinf=0, neginf=0)), 1e-3)
    print(f"case {shape} {np.dtype(dt).name} {INTERP[interp]} eb={eb}", flush=True)
    ref, dbg = codec.compress(x, eb, interp=interp, chunk_log2=cl, nonprog_levels=npl, debug=True)
    s = ctx.compress(_dev(x), eb, interp=INTERP[interp], nonprog_levels=npl, chunk_log2=cl)
    got = s.to_bytes()
    assert len(got) == len(ref)
    assert got == ref
    st = s.retrieve(eb=eb)
    assert st.plan == [0] * s.n_passes
    assert _bytes(st.tensor()) == dbg.xhat.tobytes()
    st.free()
    s.free()


@pytest.mark.parametrize("dtype,shape", [(np.float32, (40, 48, 72)), (np.float64, (40, 48, 72)),
                                         (np.float32, (150, 333))])
def test_partial_retrieve_and_refine_match_oracle(ctx, dtype, shape):
    x = fieldgen.grf(shape, -5.0 / 6.0, seed=2, dtype=dtype)
    r = fieldgen.value_range(x)
    eb = 1e-5 * r
    ref = codec.compress(x, eb)
    s = ctx.compress(_dev(x), eb)
    assert s.to_bytes() == ref
    for rel in (1e-1, 1e-2, 1e-3, 1e-4):
        st = s.retrieve(eb=rel * r)
        o = codec.retrieve(ref, "eb", rel * r)
        assert st.plan == list(o.plan)
        assert st.bound == o.bound
        assert _bytes(st.tensor()) == o.field.tobytes()
        st.free()
    for br in (0.5, 1.0, 2.0, 4.0):
        st = s.retrieve(bitrate=br)
        o = codec.retrieve(ref, "bitrate", br)
        assert st.plan == list(o.plan)
        assert _bytes(st.tensor()) == o.field.tobytes()
        st.free()
    # refine chain vs fresh retrievals
    st = s.retrieve(eb=1e-1 * r)
    o = codec.retrieve(ref, "eb", 1e-1 * r)
    for rel in (1e-2, 1e-3, 1e-5):
        info = st.refine(eb=rel * r)
        o = codec.refine(o, "eb", rel * r)
        assert st.plan == list(o.plan)
        assert info.bytes_read == o.bytes_read
        fresh = codec.retrieve_with_plan(ref, o.plan)
        assert _bytes(st.tensor()) == fresh.field.tobytes() == o.field.tobytes()
    info = st.refine(eb=1.0 * r)
    assert info.flags & pkg.IPC_FLAG_NOOP
    st.free()
    s.free()


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_dense_outliers(ctx, dtype):
    """About 1 % unpredictable values (NaN, inf, huge) spread over a field whose
    level grids span several chunk columns, so outliers fall inside the halos
    that neighbouring workgroups recompute."""
    shape = (21, 70, 200)
    x = fieldgen.random_field(shape, seed=11, dtype=dtype)
    rng = np.random.default_rng(5)
    f = x.reshape(-1)
    idx = rng.choice(f.size, size=f.size // 100, replace=False)
    kinds = rng.integers(0, 4, size=idx.size)
    big = dtype(3e37) if dtype == np.float32 else 3e300
    f[idx] = np.where(kinds == 0, np.nan, np.where(kinds == 1, np.inf, np.where(kinds == 2, -big, big)))
    eb = 1e-3
    ref, dbg = codec.compress(x, eb, debug=True)
    s = ctx.compress(_dev(x), eb)
    assert s.to_bytes() == ref
    st = s.retrieve(eb=eb)
    assert _bytes(st.tensor()) == dbg.xhat.tobytes()
    st.free()
    for plan_seed in range(3):
        draw = np.random.default_rng(plan_seed).integers(0, 12, size=s.n_passes)
        plan = [int(b) if s.pass_info(i)["progressive"] else 0 for i, b in enumerate(draw)]
        st = s.retrieve_plan(plan)
        o = codec.retrieve_with_plan(ref, plan)
        assert _bytes(st.tensor()) == o.field.tobytes()
        st.free()
    s.free()


def test_oracle_stream_retrieved_on_gpu(ctx):
    """A stream the oracle wrote, loaded through the packed placement."""
    x = fieldgen.climate_2d(1, shape=(180, 360), dtype=np.float32)
    eb = 1e-3 * fieldgen.value_range(x)
    ref = codec.compress(x, eb)
    s = ctx.stream_from_bytes(ref)
    assert s.to_bytes() == ref
    for br in (1.0, 2.0, 4.0):
        st = s.retrieve(bitrate=br)
        o = codec.retrieve(ref, "bitrate", br)
        assert st.plan == list(o.plan)
        assert _bytes(st.tensor()) == o.field.tobytes()
        assert st.info.bytes_loaded <= br * x.size / 8
        st.free()
    s.free()


def test_blobs_64_config(ctx):
    """The 64^3 smooth-field workload: compress, retrieve at 1e-2/1e-3/1e-4 * range."""
    x = fieldgen.blobs_64()
    r = fieldgen.value_range(x)
    eb = 1e-4 * r
    ref = codec.compress(x, eb)
    s = ctx.compress(_dev(x), eb)
    assert s.to_bytes() == ref
    for rel in (1e-2, 1e-3, 1e-4):
        st = s.retrieve(eb=rel * r)
        o = codec.retrieve(ref, "eb", rel * r)
        f = st.tensor()
        assert _bytes(f) == o.field.tobytes()
        err = float((f.double() - _dev(x).double()).abs().max())
        assert err <= st.bound <= rel * r
        st.free()
    s.free()


def test_errors_are_reported(ctx):
    x = _dev(np.zeros((4, 4), dtype=np.float32))
    with pytest.raises(pkg.IpcError):
        ctx.compress(x, 0.0)
    with pytest.raises(pkg.IpcError):
        ctx.compress(x, float("nan"))
    with pytest.raises(pkg.IpcError) as ei:
        ctx.stream_from_bytes(b"IPCM" + b"\0" * 200)
    assert ei.value.status == -3
    s = ctx.compress(x, 1e-3)
    with pytest.raises(pkg.IpcError):
        s.retrieve(eb=-1.0)
    with pytest.raises(pkg.IpcError):
        s.retrieve_plan([0] * (s.n_passes + 1))
    s.free()
    # an empty field is refused before anything runs on the device
    with pytest.raises(pkg.IpcError) as ei:
        ctx.compress(_dev(np.zeros((0, 4), dtype=np.float32)), 1e-3)
    assert ei.value.status == -1


def test_deterministic(ctx):
    x = _case((30, 40, 50), np.float32, seed=4, special=True)
    d = _dev(x)
    a = ctx.compress(d, 1e-3)
    b = ctx.compress(d, 1e-3)
    assert a.to_bytes() == b.to_bytes()
    a.free()
    b.free()


def _edge_fields():
    """Fields of edge values (SURVEY T5 style): subnormal magnitudes, signed
    zeros, tiny bounds whose quantizer constants leave the normal range."""
    rng = np.random.default_rng(77)
    base = fieldgen.random_field((20, 33, 70), seed=31, dtype=np.float32)
    out = []
    # subnormal magnitudes throughout (float32 normals start at 1.18e-38):
    # 2 eb is subnormal and 1 / (2 eb) overflows, so every point is an outlier
    x = (base * np.float32(1e-40)).astype(np.float32)
    out.append(("f32 subnormal field", x, 1e-4 * fieldgen.value_range(x)))
    # a normal field with subnormals and signed zeros sprinkled in
    x = base.copy()
    f = x.reshape(-1)
    idx = rng.choice(f.size, size=600, replace=False)
    f[idx[:200]] = np.float32(1e-42)
    f[idx[200:300]] = np.float32(-3e-41)
    f[idx[300:450]] = np.float32(-0.0)
    f[idx[450:]] = np.float32(0.0)
    out.append(("f32 with subnormals and signed zeros", x, 1e-3 * fieldgen.value_range(x)))
    # only signed zeros
    z = np.zeros((9, 17, 70), dtype=np.float32)
    z.reshape(-1)[::3] = np.float32(-0.0)
    out.append(("f32 signed zeros", z, 1e-3))
    # small normals with a subnormal error bound: 2 eb subnormal, 1 / (2 eb) finite
    x = (base * np.float32(1e-36)).astype(np.float32)
    out.append(("f32 subnormal bound", x, 5e-39))
    # float64 subnormal magnitudes (normals start at 2.2e-308)
    x = fieldgen.random_field((17, 33, 65), seed=32, dtype=np.float64) * 1e-310
    out.append(("f64 subnormal field", x, 1e-4 * fieldgen.value_range(x)))
    x = fieldgen.random_field((17, 33, 65), seed=34, dtype=np.float64) * 1e-306
    out.append(("f64 subnormal bound", x, 5e-309))
    x = fieldgen.random_field((130, 257), seed=33, dtype=np.float64)
    f = x.reshape(-1)
    f[::97] = -0.0
    f[5::101] = 4e-320
    out.append(("f64 2-D with subnormals and signed zeros", x, 1e-6 * fieldgen.value_range(x)))
    return out


@pytest.mark.parametrize("k", range(7))
def test_edge_values_match_oracle(ctx, k):
    what, x, eb = _edge_fields()[k]
    print(f"edge values: {what}, eb={eb}", flush=True)
    ref, dbg = codec.compress(x, eb, debug=True)
    s = ctx.compress(_dev(x), eb)
    assert s.to_bytes() == ref
    st = s.retrieve(eb=eb)
    assert _bytes(st.tensor()) == dbg.xhat.tobytes()
    st.free()
    for tg in ({"eb": 100 * eb}, {"bitrate": 1.0}):
        kind, v = next(iter(tg.items()))
        st = s.retrieve(**tg)
        o = codec.retrieve(ref, kind, v)
        assert st.plan == list(o.plan)
        assert st.bound == o.bound
        assert _bytes(st.tensor()) == o.field.tobytes()
        st.free()
    s.free()
