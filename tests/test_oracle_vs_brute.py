"""The vectorized oracle against the scalar per-point reference (not gpu).

Codes, outliers, reconstructions, chunk order and stored planes of every pass
must agree exactly on all small shapes of one to three dimensions.
"""

import numpy as np
import pytest

import fieldgen
from oracle import brute, codec, coding, predict, schedule
from oracle.stream import parse_stream

SHAPES = [(1,), (2,), (5,), (17,), (33,), (70,), (2, 3), (5, 9), (9, 17), (17, 5),
          (3, 3, 3), (5, 2, 9), (10, 11, 12), (9, 9, 9), (2, 17, 9)]


@pytest.mark.parametrize("dims", SHAPES)
@pytest.mark.parametrize("interp", [predict.LINEAR, predict.CUBIC])
@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_oracle_matches_brute(dims, interp, dtype):
    x = fieldgen.random_field(dims, seed=sum(dims), dtype=dtype)
    x.reshape(-1)[::13] += dtype(0.37)
    if x.size > 20:
        x.reshape(-1)[7] = np.nan
    eb = max(2e-3 * fieldgen.value_range(np.nan_to_num(x)), 1e-3)
    cl = tuple([1, 2, 3][: len(dims)])        # small chunks: many chunks, ragged edges
    buf, dbg = codec.compress(x, eb, interp=interp, chunk_log2=cl, debug=True)
    ref = brute.compress_brute(x, eb, interp, cl)
    assert np.array_equal(dbg.xhat.view(np.uint8), ref["xhat"].view(np.uint8))
    sched = schedule.make_schedule(dims, cl)
    ps = parse_stream(buf)
    w = 0
    cbase = 0
    for p in sched.passes:
        chunk_id, local = schedule.stream_positions(p)
        q = dbg.codes[p.index]
        for key, val in ref["codes"][p.index].items():
            sel = (chunk_id == key[0]) & (local == key[1])
            assert int(q[sel][0]) == val
        # stored planes of each chunk, built bit by bit from the brute codes
        for ci in range(p.n_chunks):
            n = int(p.chunk_counts[ci])
            codes = [ref["codes"][p.index][(ci, j)] for j in range(n)]
            e = [int(v) for v in coding.xor_encode(coding.to_negabinary(np.array(codes, dtype=np.int64)))] if n else []
            planes = brute.planes_brute(e) if n else [[] for _ in range(32)]
            mask = sum(1 << k for k in range(32) if any(planes[k]))
            assert int(ps.masks[cbase + ci]) == mask
            for k in range(31, -1, -1):
                if (mask >> k) & 1:
                    W = len(planes[k])
                    assert ps.payload[w:w + W].tolist() == planes[k]
                    w += W
        cbase += p.n_chunks
        # outliers
        got = [(tuple(int(v) for v in row[1:]), ps.out_vals[i]) for i, row in enumerate(ps.out_keys) if row[0] == p.index]
        exp = ref["outliers"][p.index]
        assert [g[0] for g in got] == [e[0] for e in exp]
        for g, e in zip(got, exp):
            assert np.array([g[1]], dtype=dtype).view(np.uint8).tobytes() == np.array([e[1]], dtype=dtype).view(np.uint8).tobytes()
    assert w == ps.payload.size
