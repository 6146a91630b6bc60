"""Batched compression and retrieval (gpu): several fields per call, one
launch per level over all of them.  Each result must equal, byte for byte,
the same field compressed or retrieved alone, which the single-field tests
tie to the oracle; the smaller fields are also compared with the oracle
directly."""

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


def _fields(shapes, dtype, seed0):
    out = []
    for i, sh in enumerate(shapes):
        x = fieldgen.grf(sh, -5.0 / 6.0, seed=seed0 + i, dtype=dtype)
        out.append(x)
    return out


@pytest.mark.parametrize("dtype,rel", [(np.float32, 1e-4), (np.float64, 1e-6)])
def test_batch_equals_single_calls(ctx, dtype, rel):
    # uneven shapes: different level counts, ragged tiles, one field large
    # enough for multi-step columns
    shapes = [(33, 40, 70), (9, 17, 130), (64, 96, 200), (2, 3, 5), (130, 70, 66)]
    xs = _fields(shapes, dtype, 40)
    ebs = [rel * fieldgen.value_range(x) for x in xs]
    devs = [_dev(x) for x in xs]
    batch = ctx.compress_batch(devs, ebs)
    singles = [ctx.compress(d, e) for d, e in zip(devs, ebs)]
    for i, (b, s) in enumerate(zip(batch, singles)):
        bb = b.to_bytes()
        assert bb == s.to_bytes(), f"field {i} {shapes[i]}"
        if xs[i].size < 300_000:
            assert bb == codec.compress(xs[i], ebs[i]), f"field {i} vs oracle"
    # mixed targets: full precision, looser bounds, a bitrate
    targets = [("eb", ebs[0]), ("eb", 100 * ebs[1]), ("eb", 10 * ebs[2]), ("eb", ebs[3]),
               ("bitrate", 2.0)]
    sts = []
    for kind in ("eb", "bitrate"):
        idx = [i for i, t in enumerate(targets) if t[0] == kind]
        vals = [targets[i][1] for i in idx]
        got = ctx.retrieve_batch([batch[i] for i in idx], **{kind: vals})
        for i, st in zip(idx, got):
            one = singles[i].retrieve(**{kind: targets[i][1]})
            assert st.plan == one.plan
            assert st.bound == one.bound
            assert _bytes(st.tensor()) == _bytes(one.tensor()), f"field {i}"
            one.free()
            sts.append(st)
    # a batch state refines like any other
    st = sts[1]
    st.refine(eb=ebs[1])
    fresh = singles[1].retrieve(eb=ebs[1])
    assert _bytes(st.tensor()) == _bytes(fresh.tensor())
    fresh.free()
    for st in sts:
        st.free()
    for s in batch + singles:
        s.free()


def test_batch_2d_fields_and_mixed_rank_retrieval(ctx):
    """2-D fields batched on the fused level kernels (one plane, no pass A),
    uneven in size and level count; their streams retrieved in one batch with
    3-D streams; every result equal to the oracle's."""
    shapes2 = [(90, 300), (17, 1000), (257, 129)]
    xs = _fields(shapes2, np.float32, 70)
    ebs = [1e-4 * fieldgen.value_range(x) for x in xs]
    batch = ctx.compress_batch([_dev(x) for x in xs], ebs)
    refs = [codec.compress(x, e) for x, e in zip(xs, ebs)]
    assert [s.to_bytes() for s in batch] == refs
    x3 = fieldgen.grf((33, 40, 70), -5.0 / 6.0, seed=77, dtype=np.float32)
    e3 = 1e-4 * fieldgen.value_range(x3)
    s3 = ctx.compress(_dev(x3), e3)
    ref3 = codec.compress(x3, e3)
    ss = batch + [s3]
    refs = refs + [ref3]
    for kind, vals in (("eb", [10 * e for e in ebs] + [100 * e3]), ("bitrate", [1.0, 2.0, 4.0, 3.0])):
        sts = ctx.retrieve_batch(ss, **{kind: vals})
        for i, (st, ref, v) in enumerate(zip(sts, refs, vals)):
            o = codec.retrieve(ref, kind, v)
            assert st.plan == list(o.plan), (kind, i)
            assert _bytes(st.tensor()) == o.field.tobytes(), (kind, i)
            st.free()
    for s in ss:
        s.free()


def test_batch_outlier_overflow_and_fallback(ctx):
    """A field whose outliers exceed the batch's record share is compressed
    again alone; a batch of 2-D fields shares the pass launches."""
    rng = np.random.default_rng(3)
    a = fieldgen.random_field((40, 64, 128), seed=7, dtype=np.float32)
    f = a.reshape(-1)
    f[rng.choice(f.size, size=f.size // 10, replace=False)] = np.nan
    b = fieldgen.random_field((20, 30, 70), seed=8, dtype=np.float32)
    xs = [a, b]
    ebs = [1e-3, 1e-3]
    batch = ctx.compress_batch([_dev(x) for x in xs], ebs)
    for x, e, s in zip(xs, ebs, batch):
        assert s.to_bytes() == codec.compress(x, e)
        s.free()
    xs2 = [fieldgen.random_field((50, 70), seed=9 + i, dtype=np.float32) for i in range(3)]
    batch = ctx.compress_batch([_dev(x) for x in xs2], [1e-3] * 3)
    sts = ctx.retrieve_batch(batch, eb=[1e-2] * 3)
    for x, s, st in zip(xs2, batch, sts):
        ref = codec.compress(x, 1e-3)
        assert s.to_bytes() == ref
        assert _bytes(st.tensor()) == codec.retrieve(ref, "eb", 1e-2).field.tobytes()
        st.free()
        s.free()


def test_batch_outlier_index_paths(ctx):
    """Outlier indexes of a batch: a field with more than 2048 outliers (the
    general sort), one with a few (one-workgroup sort), one with none; the
    streams and retrievals through the indexes equal the oracle's."""
    rng = np.random.default_rng(5)
    a = fieldgen.random_field((40, 64, 128), seed=21, dtype=np.float32)
    a.reshape(-1)[rng.choice(a.size, size=600, replace=False)] = np.nan
    b = fieldgen.random_field((40, 64, 128), seed=22, dtype=np.float32)
    b.reshape(-1)[rng.choice(b.size, size=97, replace=False)] = np.inf
    c = np.zeros((40, 64, 128), dtype=np.float32)
    xs = [a, b, c]
    print("batch outlier index paths", flush=True)
    batch = ctx.compress_batch([_dev(x) for x in xs], [1e-3] * 3)
    counts = []
    for x, s in zip(xs, batch):
        ref = codec.compress(x, 1e-3)
        assert s.to_bytes() == ref
        counts.append(codec.open_stream(ref)[0].header.n_outliers)
        st = s.retrieve(eb=1e-3)
        assert _bytes(st.tensor()) == codec.retrieve(ref, "eb", 1e-3).field.tobytes()
        st.free()
        s.free()
    assert counts[0] > 2048 and 0 < counts[1] <= 2048 and counts[2] == 0, counts


def test_batch_argument_errors(ctx):
    x = _dev(np.zeros((4, 4, 4), dtype=np.float32))
    with pytest.raises(ValueError):
        ctx.compress_batch([x, x], [1e-3])
    with pytest.raises(pkg.IpcError):
        ctx.compress_batch([x, x], [1e-3, -1.0])


def test_autotune_keeps_results(ctx):
    """Tuned column lengths change launch shapes only: streams and
    reconstructions stay byte-identical, single and batched."""
    x = fieldgen.grf((130, 100, 260), -5.0 / 6.0, seed=12, dtype=np.float32)
    y = fieldgen.grf((130, 100, 260), -5.0 / 6.0, seed=13, dtype=np.float32)
    eb = 1e-4 * fieldgen.value_range(x)
    d, dy = _dev(x), _dev(y)
    ctx.autotune_clear()
    s0 = ctx.compress(d, eb)
    a = s0.to_bytes()
    st0 = s0.retrieve(eb=10 * eb)
    f0 = _bytes(st0.tensor())
    zc, zr = ctx.autotune(d, eb)
    levels = [l for l in range(1, 32) if zc[l]]
    assert levels == list(range(1, len(levels) + 1)) and len(levels) >= 7
    assert all(zc[l] in (1, 2, 4, 8, 16) and zr[l] in (1, 2, 4, 8, 16) for l in levels)
    assert zc[0] == 0 and zr[0] == 0
    s1 = ctx.compress(d, eb)
    assert s1.to_bytes() == a
    st1 = s1.retrieve(eb=10 * eb)
    assert _bytes(st1.tensor()) == f0
    bs = ctx.compress_batch([d, dy], [eb, eb])
    assert bs[0].to_bytes() == a
    ref_y = codec.compress(y, eb)
    assert bs[1].to_bytes() == ref_y
    sts = ctx.retrieve_batch(bs, eb=[10 * eb, 10 * eb])
    assert _bytes(sts[0].tensor()) == f0
    assert _bytes(sts[1].tensor()) == codec.retrieve(ref_y, "eb", 10 * eb).field.tobytes()
    for t in sts + [st0, st1]:
        t.free()
    for s in bs + [s0, s1]:
        s.free()
    ctx.autotune_clear()
    with pytest.raises(pkg.IpcError):
        ctx.autotune(_dev(np.zeros((40, 50), dtype=np.float32)), 1e-3)


@pytest.mark.parametrize("dtype,rel,cl2", [(np.float32, 1e-4, None), (np.float64, 1e-7, None),
                                          (np.float32, 1e-4, (5, 6))])
def test_pass_batch_equals_single_calls(ctx, dtype, rel, cl2):
    """2-D fields of uneven shapes (different pass counts, ragged chunks:
    the fused level launches with the default chunks, the
    one-pass-per-launch batch with 32 x 64 chunks) and 1-D fields (one pass
    per launch): streams, retrievals and refinements equal the same field
    alone and the oracle."""
    for shapes in ([(300, 500), (47, 1000), (9, 17), (1800, 700)], [(20000,), (333,), (5,)]):
        cl = cl2 if len(shapes[0]) == 2 else None
        xs = [fieldgen.random_field(sh, seed=60 + i, dtype=dtype) for i, sh in enumerate(shapes)]
        ebs = [rel * fieldgen.value_range(x) for x in xs]
        devs = [_dev(x) for x in xs]
        batch = ctx.compress_batch(devs, ebs, chunk_log2=cl)
        singles = [ctx.compress(d, e, chunk_log2=cl) for d, e in zip(devs, ebs)]
        for i, (b, one) in enumerate(zip(batch, singles)):
            bb = b.to_bytes()
            assert bb == one.to_bytes(), f"field {i} {shapes[i]}"
            if xs[i].size < 200_000:
                assert bb == codec.compress(xs[i], ebs[i], chunk_log2=cl), f"field {i} vs oracle"
        for kind, vals in (("eb", [30 * e for e in ebs]), ("bitrate", [1.0, 3.0, 6.0, 9.0][:len(xs)])):
            got = ctx.retrieve_batch(batch, **{kind: vals})
            for i, st in enumerate(got):
                one = singles[i].retrieve(**{kind: vals[i]})
                assert st.plan == one.plan
                assert _bytes(st.tensor()) == _bytes(one.tensor()), f"field {i} {kind}"
                one.free()
                st.free()
        # served together: new retrievals and refinements joining at their
        # first changed pass
        base = [b.retrieve(eb=1e3 * e) for b, e in zip(batch, ebs)]
        reqs = [(None, base[0], {"eb": ebs[0]}), (batch[1], None, {"bitrate": 4.0}),
                (None, base[2], {"eb": 10 * ebs[2]})]
        out = ctx.serve_batch(reqs)
        assert [o[2] for o in out] == [0, 0, 0]
        for (st, info, status), s in zip(out, [singles[0], singles[1], singles[2]]):
            alone = s.retrieve_plan(st.plan)
            assert _bytes(st.tensor()) == _bytes(alone.tensor())
            alone.free()
        out[1][0].free()
        for st in base:
            st.free()
        for b, one in zip(batch, singles):
            b.free()
            one.free()


def test_climate_batch_full_size(ctx):
    """Four full 1800 x 3600 climate fields (two 30 % masked) compressed and
    retrieved at 1, 2 and 4 bits per value in batches: equal to single calls."""
    xs = [fieldgen.climate_2d(i) for i in range(4)]
    ebs = [1e-3 * fieldgen.value_range(x) for x in xs]
    devs = [_dev(x) for x in xs]
    batch = ctx.compress_batch(devs, ebs)
    for d, e, b in zip(devs, ebs, batch):
        one = ctx.compress(d, e)
        assert b.to_bytes() == one.to_bytes()
        one.free()
    for br in (1.0, 2.0, 4.0):
        got = ctx.retrieve_batch(batch, bitrate=[br] * 4)
        for b, st in zip(batch, got):
            one = b.retrieve(bitrate=br)
            assert st.plan == one.plan
            assert _bytes(st.tensor()) == _bytes(one.tensor())
            one.free()
            st.free()
    for b in batch:
        b.free()
