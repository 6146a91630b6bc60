"""Batched retrievals as queue launches replayed from captured HIP graphs
(gpu).  Every result must equal, byte for byte, the oracle's retrieval for
the same target (plan, bound and reconstruction) and the same retrieval made
by the direct launches; a graph is captured once per launch shape and
replayed for later batches of that shape, with other work and
synchronizations between the replays, and every replay is checked."""

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


def _direct(ctx, stream, kind, value):
    ctx.set_batch_graphs(False)
    st = stream.retrieve(**{kind: value})
    out = (st.plan, st.bound, _bytes(st.tensor()))
    st.free()
    return out


def _check_batch(ctx, streams, kind, values, label, refs):
    """refs[i]: the oracle's stream for streams[i]"""
    ctx.set_batch_graphs(True)
    sts = ctx.retrieve_batch(streams, **{kind: values})
    ctx.set_batch_graphs(False)
    for i, (s, v, st, ref) in enumerate(zip(streams, values, sts, refs)):
        o = codec.retrieve(ref, kind, v)
        got = _bytes(st.tensor())
        assert st.plan == list(o.plan), (label, i)
        assert st.bound == o.bound, (label, i)
        assert got == o.field.tobytes(), (label, i)
        plan, bound, field = _direct(ctx, s, kind, v)
        assert (st.plan, st.bound, got) == (plan, bound, field), (label, i)
        st.free()


@pytest.mark.parametrize("dtype,interp,rel", [(np.float32, "cubic", 1e-4), (np.float64, "linear", 1e-6)])
def test_graph_batches_equal_direct_launches(ctx, dtype, interp, rel):
    # uneven shapes: level counts 3 .. 8, ragged tiles, multi-step columns,
    # small levels (grid class 16), middle ones (128) and the full class, a
    # 2-D field among them
    shapes = [(33, 40, 70), (9, 17, 130), (64, 96, 200), (2, 3, 5), (130, 70, 66), (90, 300)]
    xs = [fieldgen.grf(sh, -5.0 / 6.0, seed=60 + i, dtype=dtype) for i, sh in enumerate(shapes)]
    ebs = [rel * fieldgen.value_range(x) for x in xs]
    ss = [ctx.compress(_dev(x), e, interp=interp) for x, e in zip(xs, ebs)]
    it = 1 if interp == "cubic" else 0
    refs = [codec.compress(x, e, interp=it) for x, e in zip(xs, ebs)]
    assert [s.to_bytes() for s in ss] == refs
    c0, r0 = ctx.graph_stats()
    # first batch: captured
    _check_batch(ctx, ss, "eb", ebs, "full", refs)
    c1, r1 = ctx.graph_stats()
    assert (c1, r1) == (c0 + 1, r0 + 1)
    # same fields, other targets: the same launch shape, replayed; eager
    # work and synchronizations between the replays
    for trial, (kind, vals) in enumerate([("eb", [10 * e for e in ebs]),
                                          ("bitrate", [1.0, 2.0, 4.0, 8.0, 0.5, 3.0]),
                                          ("eb", [1e3 * e for e in ebs])]):
        y = torch.randn(1 << 20, device="cuda:0")
        _ = float((y * y).sum())
        torch.cuda.synchronize()
        _check_batch(ctx, ss, kind, vals, ("replay", trial), refs)
    c2, r2 = ctx.graph_stats()
    assert c2 == c1 and r2 == r1 + 3
    # another mix (a field fewer, one repeated): its own shape
    mix = [ss[2], ss[0], ss[0], ss[4], ss[5]]
    _check_batch(ctx, mix, "eb", [ebs[2], ebs[0], 5 * ebs[0], ebs[4], 30 * ebs[5]], "mix",
                 [refs[2], refs[0], refs[0], refs[4], refs[5]])
    # one field alone
    _check_batch(ctx, [ss[3]], "eb", [ebs[3]], "alone", [refs[3]])
    for s in ss:
        s.free()


def test_graph_serve_batch_refinements(ctx):
    """Refinements in a served batch start from a coarse grid gathered out of
    the resident reconstruction (the head jobs' gather mode)."""
    shapes = [(65, 65, 65), (40, 100, 90), (17, 33, 200)]
    xs = [fieldgen.grf(sh, -5.0 / 6.0, seed=80 + i, dtype=np.float32) for i, sh in enumerate(shapes)]
    rs = [fieldgen.value_range(x) for x in xs]
    ss = [ctx.compress(_dev(x), 1e-5 * r) for x, r in zip(xs, rs)]
    refs = [codec.compress(x, 1e-5 * r) for x, r in zip(xs, rs)]
    assert [s.to_bytes() for s in ss] == refs
    ctx.set_batch_graphs(True)
    try:
        for rnd in range(3):
            sts = [s.retrieve(eb=1e-2 * r) for s, r in zip(ss, rs)]
            olds = [codec.retrieve(ref, "eb", 1e-2 * r) for ref, r in zip(refs, rs)]
            reqs = [(None, st, {"eb": (1e-3 if rnd % 2 == 0 else 1e-4) * r}) for st, r in zip(sts, rs)]
            reqs.append((ss[0], None, {"bitrate": 2.0}))
            out = ctx.serve_batch(reqs)
            ctx.set_batch_graphs(False)
            for k, (st, info, status) in enumerate(out):
                assert status == 0, (rnd, k)
                tg = reqs[k][2]
                kind, v = next(iter(tg.items()))
                # the oracle: a refinement of its own retrieval, or a fresh retrieval
                o = codec.refine(olds[k], kind, v) if k < len(ss) else codec.retrieve(refs[0], kind, v)
                assert st.plan == list(o.plan), (rnd, k)
                assert _bytes(st.tensor()) == o.field.tobytes(), (rnd, k)
                src = ss[k] if k < len(ss) else ss[0]
                fresh = src.retrieve(**tg)
                assert st.plan == fresh.plan, (rnd, k)
                assert _bytes(st.tensor()) == _bytes(fresh.tensor()), (rnd, k)
                fresh.free()
                st.free()
            ctx.set_batch_graphs(True)
    finally:
        ctx.set_batch_graphs(False)
    captured, replays = ctx.graph_stats()
    assert replays >= 3
    for s in ss:
        s.free()


def _compress_graphs(ctx, xs, ebs, interp):
    ctx.set_batch_graphs(True)
    try:
        return ctx.compress_batch([_dev(x) for x in xs], ebs, interp=interp)
    finally:
        ctx.set_batch_graphs(False)


@pytest.mark.parametrize("dtype,interp", [(np.float32, "cubic"), (np.float64, "linear")])
def test_batched_compression_from_graph_replays_equals_oracle(ctx, dtype, interp):
    """Batched compression as persistent queue launches replayed from a
    captured graph: every stream equals the oracle's byte for byte, over a
    capture and two replays with new fields, with eager device work and
    synchronizations between them; uneven fields share the launches."""
    from oracle import predict
    it = predict.CUBIC if interp == "cubic" else predict.LINEAR
    c0, _ = ctx.graph_stats()
    # a batch of 3-D fields and one of 2-D fields (one plane on the fused
    # kernels), each its own launch shape
    batches = [[(40, 70, 130), (17, 33, 65), (64, 64, 64)], [(100, 260), (33, 700)]]
    for rep in range(3):
        for bi, shapes in enumerate(batches):
            print(f"compress graphs: {dtype.__name__} {interp} batch {bi} replay {rep}", flush=True)
            xs = [fieldgen.grf(sh, -5.0 / 6.0, seed=100 + 10 * rep + i, dtype=dtype)
                  for i, sh in enumerate(shapes)]
            if rep == 1:
                xs[0].reshape(-1)[11] = np.nan  # an outlier record through the queue path
            ebs = [1e-4 * fieldgen.value_range(np.nan_to_num(x)) for x in xs]
            ss = _compress_graphs(ctx, xs, ebs, interp)
            junk = torch.randn(1 << 20, device="cuda:0") * 2.0  # other work between replays
            torch.cuda.synchronize()
            del junk
            for x, e, s in zip(xs, ebs, ss):
                assert s.to_bytes() == codec.compress(x, e, interp=it)
                s.free()
    c1, r1 = ctx.graph_stats()
    assert c1 - c0 == 2  # two launch shapes: each captured once, then replayed


def test_batch_autotuner_and_automatic_mode(ctx):
    """ipc_autotune_batch picks a batch schedule for a shape; batches in the
    automatic mode (the tuned shape, and an untuned mix decided by field
    size) equal the oracle byte for byte."""
    x = fieldgen.grf((64, 96, 200), -5.0 / 6.0, seed=90, dtype=np.float32)
    eb0 = 1e-4 * fieldgen.value_range(x)
    ch = ctx.autotune_batch(_dev(x), eb0, copies=3)
    assert ch["compress"][0] == (ch["compress"][1] != 0) and ch["compress"][1] in (0, 2, 3, 4)
    assert ch["retrieve"][0] == (ch["retrieve"][1] != 0) and ch["retrieve"][1] in (0, 3, 4, 5)
    ctx.set_batch_graphs("auto")
    try:
        for shapes in ([(64, 96, 200)] * 3, [(33, 40, 70), (9, 17, 130), (40, 200, 16)]):
            print(f"automatic batches: {shapes}", flush=True)
            xs = [fieldgen.grf(sh, -5.0 / 6.0, seed=91 + i, dtype=np.float32) for i, sh in enumerate(shapes)]
            ebs = [1e-4 * fieldgen.value_range(v) for v in xs]
            ss = ctx.compress_batch([_dev(v) for v in xs], ebs)
            refs = [codec.compress(v, e) for v, e in zip(xs, ebs)]
            assert [s.to_bytes() for s in ss] == refs
            sts = ctx.retrieve_batch(ss, eb=[10 * e for e in ebs])
            for i, (st, ref, e) in enumerate(zip(sts, refs, ebs)):
                o = codec.retrieve(ref, "eb", 10 * e)
                assert st.plan == list(o.plan), (shapes, i)
                assert _bytes(st.tensor()) == o.field.tobytes(), (shapes, i)
                st.free()
            for s in ss:
                s.free()
    finally:
        ctx.set_batch_graphs(False)
        ctx.autotune_clear()
