"""The allocation-free retrieval entry point (ipc_retrieve_noalloc) through
the C ABI, against ipc_retrieve on the same streams (gpu).

Each call's output tensor is filled with NaN first, so every value compared
was written by the call.  Two calls in a row reuse the device's scratch, the
second on a smaller field; results are compared byte for byte with
ipc_retrieve and, for the small fields, with the oracle.
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


def _noalloc(s, **target):
    out = torch.full(s.shape, float("nan"), dtype=s.dtype, device="cuda:0")
    info = s.retrieve_noalloc(out, **target)
    return out, info


def _check_pair(ctx, x, rel_eb, target_rel=None, bitrate=None, oracle=False):
    r = fieldgen.value_range(x)
    s = ctx.compress(_dev(x), rel_eb * r)
    target = {"bitrate": bitrate} if bitrate is not None else {"eb": target_rel * r}
    out, info = _noalloc(s, **target)
    st = s.retrieve(**target)
    assert _bytes(out) == _bytes(st.tensor())
    assert info.plan_list() == st.plan
    assert info.bound == st.bound
    assert info.bytes_loaded == st.info.bytes_loaded
    if oracle:
        ref = codec.compress(x, rel_eb * r)
        o = codec.retrieve(ref, "bitrate" if bitrate is not None else "eb",
                           bitrate if bitrate is not None else target_rel * r)
        assert _bytes(out) == o.field.tobytes()
    st.free()
    s.free()


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_noalloc_equals_retrieve_twice_second_smaller(ctx, dtype):
    big = fieldgen.grf((96, 130, 200), -5.0 / 6.0, seed=3, dtype=dtype)
    small = fieldgen.grf((40, 50, 70), -5.0 / 6.0, seed=4, dtype=dtype)
    print(f"noalloc: {dtype.__name__} {big.shape} then {small.shape}", flush=True)
    _check_pair(ctx, big, 1e-5, target_rel=1e-3)
    _check_pair(ctx, small, 1e-5, bitrate=2.0, oracle=True)


def test_noalloc_full_precision_and_other_shapes(ctx):
    x3 = fieldgen.random_field((33, 47, 129), seed=5, dtype=np.float32)
    x2 = fieldgen.random_field((100, 130), seed=6, dtype=np.float32)
    x1 = fieldgen.random_field((5000,), seed=7, dtype=np.float64)
    for x in (x3, x2, x1):
        print(f"noalloc: {x.dtype} {x.shape}", flush=True)
        _check_pair(ctx, x, 1e-4, target_rel=1e-4, oracle=True)
        _check_pair(ctx, x, 1e-4, target_rel=1e-2, oracle=True)


def test_noalloc_refuses_oversized_and_bad_arguments(ctx):
    print("noalloc: refusal on 400^3 f32", flush=True)
    x = fieldgen.grf_torch((400, 400, 400), -5.0 / 6.0, 8)
    r = float(x.max().double() - x.min().double())
    s = ctx.compress(x, 1e-4 * r)
    out = torch.zeros(s.shape, dtype=s.dtype, device="cuda:0")
    with pytest.raises(pkg.IpcError) as e:
        s.retrieve_noalloc(out, eb=1e-2 * r)
    assert e.value.status == -1 and "scratch" in str(e.value)
    assert bool((out == 0).all())  # refused before any device work
    small = torch.zeros((10,), dtype=s.dtype, device="cuda:0")
    L = pkg.lib()
    st = L.ipc_retrieve_noalloc(ctx.handle, s._p, pkg._target(1e-2 * r, None),
                                pkg.c_void_p(small.data_ptr()), 40, None)
    assert st == -1
    s.free()
    # the scratch still serves a field that fits after the refusal
    y = fieldgen.grf((64, 64, 64), -5.0 / 6.0, seed=9, dtype=np.float32)
    _check_pair(ctx, y, 1e-4, target_rel=1e-3, oracle=True)
