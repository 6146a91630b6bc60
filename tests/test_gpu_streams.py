"""Ordering of library calls after work the caller queued on the null stream
(gpu).

A context made without a stream issues its kernels on a blocking stream of
its own, which waits for what is pending on the null stream (torch's default
stream).  Each test queues a long spin kernel on the null stream and,
behind it, the kernel that writes the call's input (or last uses its output
buffer), then calls the library at once: without the wait the call would read
the input before it is written.  Results are compared with the oracle.
"""

import numpy as np
import pytest

import fieldgen
from oracle import codec

torch = pytest.importorskip("torch")
pkg = pytest.importorskip("paper_2502_04093_amd")

pytestmark = pytest.mark.gpu

# clock cycles of the spin kernel: tens of milliseconds whatever the clock it counts
SPIN = 20_000_000


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = pkg.Context(0)
    yield c
    c.close()


def test_compress_reads_input_written_by_pending_kernel(ctx):
    x = fieldgen.grf((40, 64, 130), -5.0 / 6.0, seed=3, dtype=np.float32)
    eb = 1e-4 * fieldgen.value_range(x)
    ref = codec.compress(x, eb)
    src = torch.from_numpy(x).to("cuda:0")
    dst = torch.zeros_like(src)
    torch.cuda.synchronize()
    assert torch.cuda.current_stream(0).cuda_stream == 0
    print("compress behind a pending copy", flush=True)
    torch.cuda._sleep(SPIN)
    dst.copy_(src)          # pending behind the spin when compress starts
    s = ctx.compress(dst, eb)
    assert s.to_bytes() == ref


def test_copy_out_waits_for_pending_writes_to_its_buffer(ctx):
    x = fieldgen.grf((24, 40, 66), -5.0 / 6.0, seed=4, dtype=np.float32)
    r = fieldgen.value_range(x)
    eb = 1e-4 * r
    ref = codec.compress(x, eb)
    o = codec.retrieve(ref, "eb", 1e-2 * r)
    s = ctx.compress(torch.from_numpy(x).to("cuda:0"), eb)
    st = s.retrieve(eb=1e-2 * r)
    out = torch.empty(x.shape, dtype=torch.float32, device="cuda:0")
    torch.cuda.synchronize()
    print("state copy behind a pending fill of its buffer", flush=True)
    torch.cuda._sleep(SPIN)
    out.fill_(7.0)          # pending: the copy must land after it
    st.copy_into(out)
    assert out.cpu().numpy().tobytes() == o.field.tobytes()
