#!/usr/bin/env python3
"""Throughput of the IPComp hot path on one MI355X.

One step = one compress of the whole field plus one retrieval of it at the
compression bound (every plane loaded), both through the C ABI, with the field
resident in HBM.  The default workload is the 512^3 float32 Gaussian random
field with a k^-5/3 power spectrum (turbulence-like, unit variance), cubic
interpolation, absolute error bound 1e-4 * (max - min).

Printed (one JSON line): value = input GB (10^9 bytes of float32) per second
through compress + retrieve (n * 4 / ms_per_step), the two halves separately,
p50/p99 host latency of a retrieval call, the roofline of the dominant kernel
(measured with HIP events on the library's stream) and the oracle timed on a
bounded sample of the same field on the host CPU.
"""

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0


def parse_args():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--shape", type=int, nargs="+", default=[512, 512, 512])
    ap.add_argument("--interp", choices=["linear", "cubic"], default="cubic")
    ap.add_argument("--rel-eb", type=float, default=1e-4)
    ap.add_argument("--dtype", choices=["f32", "f64"], default="f32")
    ap.add_argument("--latency-calls", type=int, default=50)
    ap.add_argument("--cpu-sample", type=int, default=384,
                    help="edge of the cubic sub-block the oracle compresses and retrieves")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--workload", choices=["field512", "blobs64", "climate-batch", "lognormal-batch", "serve",
                                           "entropy", "variants"],
                    default="field512",
                    help="field512: the headline line (one field); blobs64: the 64^3 smooth "
                         "field (Gaussian blobs, sines, noise), compress and retrievals at 1e-2, "
                         "1e-3 and 1e-4 * range, beside the oracle on the same field; "
                         "climate-batch: 20 (--fields) "
                         "1800x3600 float32 climate fields, batched compress and batched "
                         "retrievals at 1, 2 and 4 bits per value, beside one field per call; "
                         "lognormal-batch: --fields float64 "
                         "256x384x384 log-normal fields through the batched calls, beside "
                         "the same fields one call at a time; serve: a Poisson request "
                         "mix over --fields resident fields through the serving loop, beside "
                         "the same trace served one request at a time; entropy: the entropy "
                         "stage on the 512^3 field (compression ratio, coder times) and on "
                         "--fields 1800x3600 climate fields (bitrate retrievals planned on "
                         "raw and on coded plane sizes); variants: the paper's per-level "
                         "plane groups against per-pass groups, and its additive refinement "
                         "against the recompute form, on the 512^3 field")
    ap.add_argument("--requests", type=int, default=600)
    ap.add_argument("--rate", type=float, default=2000.0, help="serve: arrivals per second")
    ap.add_argument("--budget-gib", type=float, default=32.0, help="serve: device-memory budget")
    ap.add_argument("--fields", type=int, default=8)
    ap.add_argument("--direct-batches", action="store_true",
                    help="serve: batched retrievals as direct launches instead of graph replays")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default column lengths (no ipc_autotune before timing)")
    ap.add_argument("--column-rows", default=None,
                    help="install these column lengths instead of tuning: "
                         "'c=16,8,1,...;r=8,2,1,...' (by level from 1)")
    ap.add_argument("--copy-reference", action="store_true",
                    help="first run one plain device copy of the field (a known-size "
                         "reference for hardware byte counters)")
    return ap.parse_args()


def main():
    args = parse_args()
    if args.gpus != 1:
        print(f"bench.py: measures one GPU (asked for --gpus {args.gpus}); "
              "independent fields would shard across GPUs with no exchange",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import fieldgen
    import paper_2502_04093_amd as pkg

    if args.workload == "lognormal-batch":
        return batch_main(args)
    if args.workload == "blobs64":
        return blobs_main(args)
    if args.workload == "climate-batch":
        return climate_batch_main(args)
    if args.workload == "serve":
        return serve_main(args)
    if args.workload == "entropy":
        return entropy_main(args)
    if args.workload == "variants":
        return variants_main(args)
    dev = "cuda:0"
    shape = tuple(args.shape)
    n = int(np.prod(shape))
    print(f"[bench] generating {shape} field on {dev}", file=sys.stderr, flush=True)
    x = fieldgen.grf_torch(shape, -5.0 / 6.0, args.seed, device=dev)
    if args.dtype == "f64":
        x = x.double()
    itemsize = x.element_size()
    rng = float(x.max().double() - x.min().double())
    eb = args.rel_eb * rng
    if args.copy_reference:
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
        print(f"[bench] copy reference: {x.numel() * itemsize} bytes read, same written",
              file=sys.stderr, flush=True)
        del y
    ctx = pkg.Context(0)
    tuned = None
    if args.column_rows:
        parts = dict(p.split("=") for p in args.column_rows.split(";"))
        zc = [0] + [int(v) for v in parts["c"].split(",")]
        zr = [0] + [int(v) for v in parts["r"].split(",")]
        ctx.autotune_set(shape, x.dtype, zc, zr, interp=args.interp)
        tuned = {"compress": zc[1:], "retrieve": zr[1:]}
    elif not args.no_autotune:
        try:
            zc, zr = ctx.autotune(x, eb, interp=args.interp)
            tuned = {"compress": [v for v in zc if v], "retrieve": [v for v in zr if v]}
        except pkg.IpcError:  # no fused launches to tune for this shape
            tuned = None
    if tuned:
        print(f"[bench] column lengths by level 1..: {tuned}", file=sys.stderr, flush=True)

    def step():
        t0 = time.perf_counter()
        s = ctx.compress(x, eb, interp=args.interp)
        t1 = time.perf_counter()
        st = s.retrieve(eb=eb)
        t2 = time.perf_counter()
        return s, st, t1 - t0, t2 - t1

    # warm-up (code objects load on the first call); the last warm-up step
    # times every launch to find the dominant kernel
    for _ in range(max(1, args.warmup) - 1):
        s, st, _, _ = step()
        st.free()
        s.free()
    ctx.set_profiling(True, -1)
    s = ctx.compress(x, eb, interp=args.interp)
    c_ms = ctx.pass_times()
    st = s.retrieve(eb=eb)
    r_ms = ctx.pass_times()
    P = s.n_passes
    pinfo = [s.pass_info(i) for i in range(P)]
    stream_bytes = s.nbytes
    st.free()
    s.free()
    ctx.set_profiling(False)
    launches = sorted({p["launch_pass"] for p in pinfo})
    dom_op, dom_pass = max([("compress", i) for i in launches] + [("retrieve", i) for i in launches],
                           key=lambda k: (c_ms if k[0] == "compress" else r_ms)[k[1]])

    # timed region; only the dominant pass is bracketed by events
    ctx.set_profiling(True, dom_pass)
    torch.cuda.synchronize()
    tc = tr = 0.0
    dom_c = []
    dom_r = []
    step_c, step_r = [], []
    T0 = time.perf_counter()
    for _ in range(args.steps):
        t0 = time.perf_counter()
        s = ctx.compress(x, eb, interp=args.interp)
        dom_c.append(ctx.pass_times()[dom_pass])
        t1 = time.perf_counter()
        st = s.retrieve(eb=eb)
        dom_r.append(ctx.pass_times()[dom_pass])
        t2 = time.perf_counter()
        tc += t1 - t0
        tr += t2 - t1
        step_c.append((t1 - t0) * 1e3)
        step_r.append((t2 - t1) * 1e3)
        st.free()
        s.free()
    torch.cuda.synchronize()
    T1 = time.perf_counter()
    ctx.set_profiling(False)
    ms_per_step = (T1 - T0) * 1e3 / args.steps
    gb = n * itemsize / 1e9

    # retrieval latency
    s = ctx.compress(x, eb, interp=args.interp)
    lat = []
    plan_ms = []
    L = args.latency_calls
    for _ in range(L):
        t0 = time.perf_counter()
        st = s.retrieve(eb=eb)
        lat.append((time.perf_counter() - t0) * 1e3)
        plan_ms.append(st.info.t_plan_ms)
        st.free()
    # a partial target (1e-3 * range): the planner's program runs
    part = {}
    for rel_t in ((1e-3,) if L > 0 else ()):
        e_t = rel_t * rng
        lp, pp = [], []
        for _ in range(L):
            t0 = time.perf_counter()
            st = s.retrieve(eb=e_t)
            lp.append((time.perf_counter() - t0) * 1e3)
            pp.append(st.info.t_plan_ms)
            bl = st.info.bytes_loaded
            st.free()
        lp.sort()
        part[f"eb={rel_t:g}*range"] = {
            "p50": round(lp[len(lp) // 2], 4),
            "p99": round(lp[min(len(lp) - 1, int(math.ceil(0.99 * len(lp))) - 1)], 4),
            "planner_median": round(sorted(pp)[len(pp) // 2], 4), "bytes_loaded": int(bl)}
    s.free()
    # quality of the full retrieval (outside the timed region)
    s = ctx.compress(x, eb, interp=args.interp)
    st = s.retrieve(eb=eb)
    err = st.tensor().double() - x.double()
    max_err = float(err.abs().max())
    mse = float((err * err).mean())
    psnr = 20 * math.log10(rng) - 10 * math.log10(mse) if mse > 0 else float("inf")
    del err
    st.free()
    s.free()
    lat.sort()
    p50 = lat[len(lat) // 2] if lat else None
    p99 = lat[min(len(lat) - 1, int(math.ceil(0.99 * len(lat))) - 1)] if lat else None

    # roofline of the dominant kernel: algorithmic bytes per launch
    alg_bytes, alg_targets, kname = launch_bytes(dom_op, dom_pass, pinfo, shape, itemsize, args.interp)
    traffic = counted_traffic(dom_op, pinfo[dom_pass]["level"], shape, itemsize, args.interp)
    dom_list = dom_c if dom_op == "compress" else dom_r
    dom_avg_ms = sum(dom_list) / len(dom_list)
    achieved = alg_bytes / (dom_avg_ms * 1e-3) / 1e9
    # whole calls: compression moves n s + C (field in, stream out), a full
    # retrieval L_E + n s (every stream byte in, field out); median call time
    c_med = sorted(step_c)[len(step_c) // 2]
    r_med = sorted(step_r)[len(step_r) // 2]
    call_c = n * itemsize + stream_bytes
    call_r = stream_bytes + n * itemsize
    whole = {"compress": {"alg_bytes": call_c, "ms": round(c_med, 4),
                          "GBps": round(call_c / (c_med * 1e-3) / 1e9, 2),
                          "frac": round(call_c / (c_med * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4)},
             "retrieve": {"alg_bytes": call_r, "ms": round(r_med, 4),
                          "GBps": round(call_r / (r_med * 1e-3) / 1e9, 2),
                          "frac": round(call_r / (r_med * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4)}}

    out = {
        "metric": "compress & retrieve GB/s (fp32 in) at eb=1e-4*range; p50/p99 retrieval latency",
        "value": round(gb / (ms_per_step / 1e3), 3),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if itemsize == 4 else "f64",
        "data": "synthetic",
        "config": {"workload": f"{'x'.join(map(str, shape))} {'f32' if itemsize == 4 else 'f64'} "
                               f"Gaussian random field P(k)~k^-5/3, {args.interp}, eb={args.rel_eb:g}*range, "
                               "compress + full retrieve",
                   "eb_abs": eb, "stream_bytes": stream_bytes,
                   "compression_ratio": round(n * itemsize / stream_bytes, 4),
                   "n_passes": P},
        "compress_GBps": round(gb / (tc / args.steps), 3),
        "retrieve_GBps": round(gb / (tr / args.steps), 3),
        "retrieve_latency_ms": {"p50": p50 and round(p50, 4), "p99": p99 and round(p99, 4), "calls": L,
                                "planner_median": round(sorted(plan_ms)[len(plan_ms) // 2], 4) if plan_ms else None,
                                "partial": part},
        "step_ms": {"compress_median": round(sorted(step_c)[len(step_c) // 2], 4),
                    "compress_min": round(min(step_c), 4),
                    "retrieve_median": round(sorted(step_r)[len(step_r) // 2], 4),
                    "retrieve_min": round(min(step_r), 4)},
        "quality": {"max_abs_err": max_err, "within_eb": max_err <= eb, "psnr_db": round(psnr, 3)},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBPS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": traffic,
                     "kernel": kname, "alg_bytes_per_launch": int(alg_bytes),
                     "alg_bytes_per_target": round(alg_bytes / max(1, alg_targets), 4),
                     "targets_per_launch": int(alg_targets),
                     "avg_launch_ms": round(dom_avg_ms, 5), "whole_call": whole},
        "pass_ms": {"compress": [round(v, 4) for v in c_ms], "retrieve": [round(v, 4) for v in r_ms]},
        "launch": {"column_rows_by_level": tuned, "autotuned": tuned is not None and not args.column_rows},
    }

    if not args.no_cpu_baseline:
        out["cpu_baseline"], out["parity"] = cpu_baseline(x, eb, args, ctx)
    print(json.dumps(out), flush=True)
    ctx.close()


def blobs_main(args):
    """The 64^3 float32 smooth field (8 Gaussian blobs + sine product +
    N(0, 1e-3) noise, seed 0), cubic, eb = 1e-4 * range: per step one
    compression and retrievals at 1e-2, 1e-3 and 1e-4 * range; per-call
    latencies; the oracle on the same field (one core) with the parity of
    the stream and of each retrieval."""
    import hashlib

    import numpy as np
    import torch

    import fieldgen
    import paper_2502_04093_amd as pkg
    from oracle import codec

    xn = fieldgen.blobs_64()
    x = torch.from_numpy(xn).to("cuda:0")
    rng = fieldgen.value_range(xn)
    eb = 1e-4 * rng
    rels = (1e-2, 1e-3, 1e-4)
    ctx = pkg.Context(0)
    lat = {"compress": [], **{f"retrieve eb={r:g}*range": [] for r in rels}}

    def step(record):
        t0 = time.perf_counter()
        s = ctx.compress(x, eb)
        t1 = time.perf_counter()
        if record:
            lat["compress"].append((t1 - t0) * 1e3)
        for r in rels:
            t0 = time.perf_counter()
            st = s.retrieve(eb=r * rng)
            t1 = time.perf_counter()
            if record:
                lat[f"retrieve eb={r:g}*range"].append((t1 - t0) * 1e3)
            st.free()
        s.free()

    for _ in range(max(1, args.warmup)):
        step(False)
    torch.cuda.synchronize()
    T0 = time.perf_counter()
    for _ in range(args.steps):
        step(True)
    torch.cuda.synchronize()
    T1 = time.perf_counter()
    ms = (T1 - T0) * 1e3 / args.steps

    def pct(v, q):
        v = sorted(v)
        return round(v[min(len(v) - 1, max(0, int(math.ceil(q * len(v))) - 1))], 4)

    lat_out = {k: {"p50": pct(v, 0.5), "p99": pct(v, 0.99), "calls": len(v)} for k, v in lat.items()}
    gb = xn.nbytes / 1e9
    # the oracle on the same field, and the parity of the GPU results
    t0 = time.perf_counter()
    buf = codec.compress(xn, eb)
    tc = time.perf_counter() - t0
    s = ctx.compress(x, eb)
    got = s.to_bytes()
    par = {"stream_sha256": hashlib.sha256(got).hexdigest()[:16], "stream_equal_oracle": got == buf}
    tr = {}
    for r in rels:
        t0 = time.perf_counter()
        o = codec.retrieve(buf, "eb", r * rng)
        tr[r] = time.perf_counter() - t0
        st = s.retrieve(eb=r * rng)
        f = st.tensor()
        par[f"retrieve eb={r:g}*range equal_oracle"] = f.cpu().numpy().tobytes() == o.field.tobytes()
        par[f"retrieve eb={r:g}*range max_err"] = float((f.double() - x.double()).abs().max())
        st.free()
    s.free()
    out = {
        "metric": "compress + 3 retrievals GB/s (fp32 in), 64^3 smooth field",
        "value": round(gb / (ms * 1e-3), 3), "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "64^3 f32 smooth field (8 Gaussian blobs, sine product, N(0,1e-3) "
                               "noise, seed 0), cubic, eb=1e-4*range, compress + retrievals at "
                               "1e-2/1e-3/1e-4*range",
                   "stream_bytes": len(got)},
        "latency_ms": lat_out,
        "cpu_baseline": {"value": round(gb / (tc + sum(tr.values())), 5), "unit": "GB/s", "cores": 1,
                         "kind": "oracle", "host_cpus": os.cpu_count(), "host_cpu_model": cpu_model(),
                         "sample": f"the whole field: compress {tc:.3f} s + retrievals "
                                   + " / ".join(f"{tr[r]:.3f}" for r in rels) + " s"},
        "parity": par,
    }
    print(json.dumps(out), flush=True)
    ctx.close()


def climate_batch_main(args):
    """--fields (default 20) float32 climate fields of 1800x3600 (odd ones
    30 % masked) at eb = 1e-3 * range each: per step one batched compress and
    batched retrievals at 1, 2 and 4 bits per value; then the same work one
    field per call."""
    import torch

    import fieldgen
    import paper_2502_04093_amd as pkg

    n = args.fields if args.fields != 8 else 20
    print(f"[bench] generating {n} climate fields 1800x3600", file=sys.stderr, flush=True)
    xs = [torch.from_numpy(fieldgen.climate_2d(i)).to("cuda:0") for i in range(n)]
    ebs = [1e-3 * float(x.max().double() - x.min().double()) for x in xs]
    ctx = pkg.Context(0)
    schedule = None
    if not args.no_autotune:
        # the batch schedule for this shape (direct launches or graph
        # replays), used by the batched calls (automatic mode)
        schedule = ctx.autotune_batch(xs[0], ebs[0], copies=n)
        ctx.set_batch_graphs("auto")

    def batched():
        ss = ctx.compress_batch(xs, ebs)
        for br in (1.0, 2.0, 4.0):
            for st in ctx.retrieve_batch(ss, bitrate=[br] * n):
                st.free()
        for s in ss:
            s.free()

    def plain():
        for x, e in zip(xs, ebs):
            s = ctx.compress(x, e)
            for br in (1.0, 2.0, 4.0):
                s.retrieve(bitrate=br).free()
            s.free()

    def timed(fn):
        for _ in range(max(1, args.warmup)):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / args.steps

    tb = timed(batched)
    tp = timed(plain)
    gb = n * xs[0].numel() * 4 / 1e9
    out = {
        "metric": "batched compress + 3 bitrate retrievals GB/s (fp32 in), climate fields",
        "value": round(gb / tb, 3), "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(tb * 1e3, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{n} x 1800x3600 f32 climate (zonal bands + k^-3 noise, odd "
                               "fields 30 % masked), cubic, eb=1e-3*range, batched compress + "
                               "retrievals at 1/2/4 bits per value"},
        "plain_GBps": round(gb / tp, 3), "plain_ms_per_step": round(tp * 1e3, 4),
        "batch_speedup": round(tp / tb, 4), "batch_schedule": schedule,
    }
    print(json.dumps(out), flush=True)
    ctx.close()


def batch_main(args):
    """Several float64 log-normal fields (P(k) ~ k^-2, 256x384x384) at eb =
    1e-5 * range each: batched compress + batched full retrieve per step,
    then the same work one field per call."""
    import torch

    import fieldgen
    import paper_2502_04093_amd as pkg

    shape = (256, 384, 384)
    n = args.fields
    print(f"[bench] generating {n} fields {shape} f64", file=sys.stderr, flush=True)
    xs = [fieldgen.lognormal_torch(shape, seed=i) for i in range(n)]
    ebs = [1e-5 * float(x.max() - x.min()) for x in xs]
    ctx = pkg.Context(0)
    schedule = None
    if not args.no_autotune:
        ctx.autotune(xs[0], ebs[0])
        # the batch schedule (direct or graph replays, persistent grid) for
        # this shape, used by the batched calls below (automatic mode)
        schedule = ctx.autotune_batch(xs[0], ebs[0], copies=n)
        ctx.set_batch_graphs("auto")

    def batched():
        ss = ctx.compress_batch(xs, ebs)
        sts = ctx.retrieve_batch(ss, eb=ebs)
        for st in sts:
            st.free()
        for s in ss:
            s.free()

    def plain():
        for x, e in zip(xs, ebs):
            s = ctx.compress(x, e)
            st = s.retrieve(eb=e)
            st.free()
            s.free()

    def timed(fn):
        for _ in range(max(1, args.warmup)):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / args.steps

    tb = timed(batched)
    tp = timed(plain)
    # the batched retrieval alone, direct level launches and graph replays
    ss = ctx.compress_batch(xs, ebs)

    def retrieve_only():
        for st in ctx.retrieve_batch(ss, eb=ebs):
            st.free()

    def compress_only():
        for s in ctx.compress_batch(xs, ebs):
            s.free()

    ctx.set_batch_graphs(False)
    tr_direct = timed(retrieve_only)
    tc_direct = timed(compress_only)
    ctx.set_batch_graphs(True)
    tr_graph = timed(retrieve_only)
    tc_graph = timed(compress_only)
    ctx.set_batch_graphs(False)
    for s in ss:
        s.free()
    gb = n * xs[0].numel() * 8 / 1e9
    out = {
        "metric": "batched compress & retrieve GB/s (fp64 in), 8 fields, eb=1e-5*range",
        "value": round(gb / tb, 3), "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(tb * 1e3, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{n} x 256x384x384 f64 log-normal exp(1.5 GRF(k^-2)), cubic, "
                               "eb=1e-5*range each, batched compress + full retrieve"},
        "plain_GBps": round(gb / tp, 3), "plain_ms_per_step": round(tp * 1e3, 4),
        "batch_speedup": round(tp / tb, 4),
        "batched_retrieve_ms": {"direct_launches": round(tr_direct * 1e3, 4),
                                "graph_replay": round(tr_graph * 1e3, 4),
                                "graphs": ctx.graph_stats()},
        "batched_compress_ms": {"direct_launches": round(tc_direct * 1e3, 4),
                                "graph_replay": round(tc_graph * 1e3, 4)},
        "batch_schedule": schedule,
    }
    print(json.dumps(out), flush=True)
    ctx.close()


def entropy_main(args):
    """Entropy stage.  (1) The 512^3 float32 field at --rel-eb * range:
    serialized size raw and entropy coded, device time of the coding call
    (codes every block, gathers the coded payload) and of loading the coded
    bytes (upload + decode) beside loading the raw bytes.  (2) --fields
    1800x3600 float32 climate fields (odd ones 30 % masked) at 1e-3 * range:
    compression ratios, and retrievals at 1, 2 and 4 bits per value planned on
    raw plane sizes and on coded ones (max error, PSNR)."""
    import numpy as np
    import torch

    import fieldgen
    import paper_2502_04093_amd as pkg

    ctx = pkg.Context(0)
    shape = tuple(args.shape)
    print(f"[bench] generating {shape} field", file=sys.stderr, flush=True)
    x = fieldgen.grf_torch(shape, -5.0 / 6.0, args.seed)
    rng = float(x.max().double() - x.min().double())
    eb = args.rel_eb * rng

    def sync_time(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        return r, time.perf_counter() - t0

    t_code, t_load_raw, t_load_coded = [], [], []
    raw_b = coded_b = None
    for it in range(args.warmup + args.steps):
        s = ctx.compress(x, eb)
        if raw_b is None:
            raw_b = s.to_bytes()
        _, tc = sync_time(s.entropy_code)
        if coded_b is None:
            coded_b = s.to_bytes()
        s.free()
        s1, tr = sync_time(lambda: ctx.stream_from_bytes(raw_b))
        s2, td = sync_time(lambda: ctx.stream_from_bytes(coded_b))
        s1.free()
        s2.free()
        if it >= args.warmup:
            t_code.append(tc)
            t_load_raw.append(tr)
            t_load_coded.append(td)
        print(f"[bench] entropy step {it}: code {tc * 1e3:.2f} ms, load raw {tr * 1e3:.2f} ms, "
              f"load coded {td * 1e3:.2f} ms", file=sys.stderr, flush=True)
    nbytes = x.numel() * 4
    med = lambda v: float(np.median(v))
    big = {
        "shape": list(shape), "rel_eb": args.rel_eb,
        "raw_stream_bytes": len(raw_b), "coded_stream_bytes": len(coded_b),
        "cr_raw": round(nbytes / len(raw_b), 4), "cr_coded": round(nbytes / len(coded_b), 4),
        "code_ms": round(med(t_code) * 1e3, 3),
        "code_GBps_of_field": round(nbytes / med(t_code) / 1e9, 2),
        "load_raw_ms": round(med(t_load_raw) * 1e3, 3),
        "load_coded_ms": round(med(t_load_coded) * 1e3, 3),
    }
    del x
    torch.cuda.empty_cache()

    climate = []
    for f in range(args.fields):
        xf = fieldgen.climate_2d(f)
        xd = torch.from_numpy(xf).to("cuda:0")
        e = 1e-3 * fieldgen.value_range(xf)
        r = fieldgen.value_range(xf)
        s_raw = ctx.compress(xd, e)
        s_cod = ctx.compress(xd, e).entropy_code()
        row = {"field": f, "masked": bool(f % 2), "cr_raw": round(xf.nbytes / s_raw.nbytes, 3),
               "cr_coded": round(xf.nbytes / s_cod.nbytes, 3)}
        xd64 = xd.double()
        for br in (1.0, 2.0, 4.0):
            for tag, s in (("raw", s_raw), ("coded", s_cod)):
                st = s.retrieve(bitrate=br)
                err = (st.tensor().double() - xd64)
                mx = float(err.abs().max())
                mse = float((err * err).mean())
                psnr = 20 * math.log10(r) - 10 * math.log10(mse) if mse > 0 else float("inf")
                row[f"br{br:g}_{tag}_maxerr"] = mx
                row[f"br{br:g}_{tag}_psnr"] = round(psnr, 2)
                st.free()
        s_raw.free()
        s_cod.free()
        climate.append(row)
        print(f"[bench] climate field {f}: {row}", file=sys.stderr, flush=True)
    mean = lambda k: round(float(np.mean([c[k] for c in climate])), 3)
    summary = {"cr_raw": mean("cr_raw"), "cr_coded": mean("cr_coded")}
    for br in ("1", "2", "4"):
        for tag in ("raw", "coded"):
            summary[f"br{br}_{tag}_psnr"] = mean(f"br{br}_{tag}_psnr")
    out = {
        "metric": "entropy-coded compression ratio, 512^3 f32 GRF, eb=1e-4*range",
        "value": big["cr_coded"], "unit": "x", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": big["code_ms"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": f"entropy stage: {'x'.join(map(str, shape))} f32 GRF k^-5/3 at "
                               f"eb={args.rel_eb:g}*range; {args.fields} x 1800x3600 f32 climate "
                               "fields at eb=1e-3*range, bitrate 1/2/4"},
        "field512": big, "climate_mean": summary, "climate": climate,
    }
    print(json.dumps(out), flush=True)
    ctx.close()


def variants_main(args):
    """The paper's variants on the 512^3 float32 field compressed at 1e-6 *
    range.  (1) Plane groups: bytes loaded and bound for error-bound targets
    1e-2 .. 1e-5 * range, and bound and max error for bitrates 1, 2, 4, with
    per-pass groups and with the paper's per-level groups.  (2) The
    progressive run 1e-2 -> 1e-3 -> 1e-4 -> 1e-5 -> 1e-6 * range refined in
    the recompute form and in the additive form: device time per step, bound,
    max error and the largest difference between the two reconstructions,
    beside a fresh retrieval to the same target.  (3) The non-progressive head
    L_p = 0..4 (the top levels always loaded): stream size, bytes loaded and
    bound at 1e-2 and 1e-4 * range, bound and error at 1 bit per value."""
    import numpy as np
    import torch

    import fieldgen
    import paper_2502_04093_amd as pkg

    ctx = pkg.Context(0)
    shape = tuple(args.shape)
    print(f"[bench] generating {shape} field", file=sys.stderr, flush=True)
    x = fieldgen.grf_torch(shape, -5.0 / 6.0, args.seed)
    xd = x.double()
    r = float(x.max().double() - x.min().double())
    s = ctx.compress(x, 1e-6 * r)
    groups = []
    for rel in (1e-2, 1e-3, 1e-4, 1e-5):
        row = {"target": f"eb={rel:g}*range"}
        for tag, lg in (("pass", False), ("level", True)):
            st = s.retrieve(eb=rel * r, level_groups=lg)
            row[f"{tag}_loaded_bytes"] = int(st.info.bytes_loaded)
            row[f"{tag}_bound"] = st.info.bound
            st.free()
        groups.append(row)
        print(f"[bench] groups {row}", file=sys.stderr, flush=True)
    for br in (1.0, 2.0, 4.0):
        row = {"target": f"bitrate={br:g}"}
        for tag, lg in (("pass", False), ("level", True)):
            st = s.retrieve(bitrate=br, level_groups=lg)
            row[f"{tag}_bound"] = st.info.bound
            row[f"{tag}_maxerr"] = float((st.tensor().double() - xd).abs().max())
            st.free()
        groups.append(row)
        print(f"[bench] groups {row}", file=sys.stderr, flush=True)

    refine = []
    a = s.retrieve(eb=1e-2 * r)
    b = s.retrieve(eb=1e-2 * r)
    for rel in (1e-3, 1e-4, 1e-5, 1e-6):
        ia = a.refine(eb=rel * r)
        ib = b.refine_additive(eb=rel * r)
        # a fresh retrieval to the same target (the same plan) for comparison
        fr = s.retrieve(eb=rel * r)
        fresh_ms = fr.info.t_device_ms
        same_plan = fr.plan == a.plan
        fr.free()
        ta, tb = a.tensor().double(), b.tensor().double()
        row = {"target": f"eb={rel:g}*range",
               "recompute_ms": round(ia.t_device_ms, 3), "additive_ms": round(ib.t_device_ms, 3),
               "fresh_retrieve_ms": round(fresh_ms, 3), "fresh_same_plan": bool(same_plan),
               "recompute_bound": ia.bound, "additive_bound": ib.bound,
               "recompute_maxerr": float((ta - xd).abs().max()),
               "additive_maxerr": float((tb - xd).abs().max()),
               "max_abs_difference": float((ta - tb).abs().max()),
               "bytes_read": int(ib.bytes_read)}
        refine.append(row)
        print(f"[bench] refine {row}", file=sys.stderr, flush=True)
        del ta, tb
    a.free()
    b.free()
    s.free()
    # the non-progressive head (L_p of Alg. 1): the top levels always loaded
    head = []
    for npl in (0, 1, 2, 3, 4):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sh = ctx.compress(x, 1e-6 * r, nonprog_levels=npl)
        torch.cuda.synchronize()
        row = {"nonprog_levels": npl, "stream_bytes": int(sh.nbytes),
               "compress_ms": round((time.perf_counter() - t0) * 1e3, 3)}
        for rel in (1e-2, 1e-4):
            st = sh.retrieve(eb=rel * r)
            row[f"eb={rel:g}*range"] = {"bytes_loaded": int(st.info.bytes_loaded), "bound": st.info.bound,
                                        "device_ms": round(st.info.t_device_ms, 3)}
            st.free()
        for br in (1.0,):
            st = sh.retrieve(bitrate=br)
            row[f"bitrate={br:g}"] = {"bound": st.info.bound,
                                     "maxerr": float((st.tensor().double() - xd).abs().max())}
            st.free()
        sh.free()
        head.append(row)
        print(f"[bench] nonprog {row}", file=sys.stderr, flush=True)
    out = {
        "metric": "paper variants on 512^3 f32 GRF compressed at eb=1e-6*range",
        "value": round(sum(r_["additive_ms"] for r_ in refine), 3), "unit": "ms (additive refine steps)",
        "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": round(sum(r_["recompute_ms"] for r_ in refine), 3),
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "per-pass vs per-level plane groups; recompute vs additive "
                               "refinement 1e-2 -> 1e-6 * range"},
        "plane_groups": groups, "refinement": refine, "nonprog_head": head,
    }
    print(json.dumps(out), flush=True)
    ctx.close()


def serve_main(args):
    """Serving mix: resident float32 fields of sizes U{64^3, 128^3, 256^3,
    512^3, 1800x3600} (each a rolled, scaled and shifted copy of one of 4 base
    fields per size class), compressed at 1e-6 * range.  Requests arrive as a
    Poisson process; each picks a field; 30 % refine the state of an earlier
    retrieval of that field to a tighter target, the rest are retrievals with an
    error bound (log-uniform 1e-6..1e-2 * range) or a bitrate (0.5..8 bits per
    value), half each.  Served through ipc_server (continuous batching, device
    memory budget), then the same trace one request at a time in arrival order.
    Latency = completion - arrival."""
    import threading

    import numpy as np
    import torch

    import fieldgen
    import paper_2502_04093_amd as pkg

    rng = np.random.default_rng(5)
    classes = [(64, 64, 64), (128, 128, 128), (256, 256, 256), (512, 512, 512), (1800, 3600)]
    nf = args.fields if args.fields != 8 else 40
    print(f"[bench] generating and compressing {nf} resident fields", file=sys.stderr, flush=True)
    ctx = pkg.Context(0)
    bases = {}
    streams, ranges, sizes = [], [], []
    for i in range(nf):
        c = int(rng.integers(len(classes)))
        shape = classes[c]
        key = (c, i % 4)
        if key not in bases:
            amp = -5.0 / 6.0 if len(shape) == 3 else -1.5
            bases[key] = fieldgen.grf_torch(shape, amp, seed=100 * c + i % 4)
        shifts = tuple(int(rng.integers(n)) for n in shape)
        x = torch.roll(bases[key], shifts, dims=tuple(range(len(shape)))) * float(rng.uniform(0.5, 2)) \
            + float(rng.uniform(-1, 1))
        r = float(x.max().double() - x.min().double())
        streams.append(ctx.compress(x.contiguous(), 1e-6 * r))
        ranges.append(r)
        sizes.append(x.numel() * 4)
        del x
    bases.clear()
    torch.cuda.empty_cache()
    # the trace: (arrival s, field, kind, value, refine_of)
    R = args.requests
    t = np.cumsum(rng.exponential(1.0 / args.rate, size=R))
    trace, last_ret = [], {}
    for k in range(R):
        f = int(rng.integers(nf))
        if f in last_ret and rng.random() < 0.3 and t[k] - t[last_ret[f]] > 0.002:
            j = last_ret.pop(f)
            trace.append((t[k], f, "refine", None, j))
            continue
        if rng.random() < 0.5:
            trace.append((t[k], f, "eb", ranges[f] * 10 ** rng.uniform(-6, -2), None))
        else:
            trace.append((t[k], f, "bitrate", float(rng.uniform(0.5, 8)), None))
        last_ret[f] = k
    # tighter refinement targets: a tenth of the retrieved bound (fixed below)
    uses = {}
    for k, (_, _, kind, _, j) in enumerate(trace):
        if kind == "refine":
            uses[j] = k

    def pct(v, q):
        v = sorted(v)
        return v[min(len(v) - 1, int(np.ceil(q * len(v))) - 1)]

    # served
    srv = pkg.Server(ctx, budget_bytes=int(args.budget_gib * (1 << 30)), max_batch=64,
                     batch_graphs=not args.direct_batches)
    tickets = [None] * R
    states = [None] * R
    done_ev = [threading.Event() for _ in range(R)]
    lat = [0.0] * R
    t_done = [0.0] * R

    def waiter():
        for k in range(R):
            while tickets[k] is None:
                time.sleep(0.0001)
            kind, j = trace[k][2], trace[k][4]
            st, info, ms = srv.wait(tickets[k], stream=streams[trace[k][1]],
                                    state=states[j] if kind == "refine" else None)
            t_done[k] = time.perf_counter()
            lat[k] = ms
            if kind == "refine":
                srv.release(st)
            elif k in uses:
                states[k] = st
            else:
                srv.release(st)
            done_ev[k].set()

    wt = threading.Thread(target=waiter)
    wt.start()
    T0 = time.perf_counter()
    for k, (ta, f, kind, val, j) in enumerate(trace):
        d = T0 + ta - time.perf_counter()
        if d > 0:
            time.sleep(d)
        if kind == "refine":
            done_ev[j].wait()
            tickets[k] = srv.submit(state=states[j], eb=states[j].bound * 0.1)
        else:
            tickets[k] = srv.submit(stream=streams[f], **{kind: val})
    wt.join()
    T1 = max(t_done)
    stats = srv.stats()
    srv.close()
    served = {"requests_per_s": round(R / (T1 - T0), 2), "p50_ms": round(pct(lat, 0.5), 4),
              "p99_ms": round(pct(lat, 0.99), 4), "batches": stats["batches"],
              "peak_budget_GiB": round(stats["peak"] / (1 << 30), 3),
              "batch_graphs": not args.direct_batches, "graphs": ctx.graph_stats()}
    ctx.set_batch_graphs(False)
    # plain: one request at a time, in arrival order
    pstates = [None] * R
    plat = []
    T0 = time.perf_counter()
    for k, (ta, f, kind, val, j) in enumerate(trace):
        arr = T0 + ta
        d = arr - time.perf_counter()
        if d > 0:
            time.sleep(d)
        if kind == "refine":
            st = pstates[j]
            st.refine(eb=st.bound * 0.1)
            st.free()
            pstates[j] = None
        else:
            st = streams[f].retrieve(**{kind: val})
            torch.cuda.synchronize()
            if k in uses:
                pstates[k] = st
            else:
                st.free()
        plat.append((time.perf_counter() - arr) * 1e3)
    T1 = time.perf_counter()
    plain = {"requests_per_s": round(R / (T1 - T0), 2), "p50_ms": round(pct(plat, 0.5), 4),
             "p99_ms": round(pct(plat, 0.99), 4)}
    out = {
        "metric": "serving requests/s and p50/p99 latency (resident-field request mix)",
        "value": served["requests_per_s"], "unit": "requests/s", "n_gpus": 1, "steps": R,
        "warmup": 0, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{nf} resident f32 fields U{{64^3,128^3,256^3,512^3,1800x3600}}, "
                               f"eb=1e-6*range; {R} Poisson requests at {args.rate:g}/s, 30 % "
                               "refines; budget " + f"{args.budget_gib:g} GiB"},
        "served": served, "plain": plain,
        "speedup_requests_per_s": round(served["requests_per_s"] / plain["requests_per_s"], 4),
    }
    print(json.dumps(out), flush=True)
    for s in streams:
        s.free()
    ctx.close()


def launch_bytes(op, launch, pinfo, shape, itemsize, interp):
    """Algorithmic HBM bytes of one launch: what the method must move for the
    targets the launch predicts, nothing for the work of the layout.

    Per target that is its value (compression reads it from the input field,
    retrieval writes it to the output) plus its share of the stream (the
    planes of the launch's passes, written by compression, read by a full
    retrieval).  Summed over the launches of a call this is the call's n * s
    plus its plane bytes, the whole-call figure less the fixed part of the
    stream (header, tables, anchors, outliers).  Coarse-grid reads, halo
    re-reads and the rewrite of coarse points are the kernel's overhead, seen
    in the counted traffic, not algorithmic bytes.
    """
    group = [i for i, p in enumerate(pinfo) if p["launch_pass"] == launch]
    planes = sum(sum(pinfo[i]["plane_bytes"]) for i in group)
    targets = sum(pinfo[i]["n_targets"] for i in group)
    tname = "float" if itemsize == 4 else "double"
    if len(group) == 1:
        return targets * itemsize + planes, targets, f"k_{op}_pass<{tname},{interp}> pass {launch}"
    lev = pinfo[launch]["level"]
    return targets * itemsize + planes, targets, f"k_level3_{op}<{tname},{interp}> level {lev}"


def counted_traffic(op, level, shape, itemsize, interp):
    """HBM bytes per launch from the committed counter summaries under profiles/
    (FETCH_SIZE + WRITE_SIZE, scaled by a plain copy of known size), or None when
    no summary covers this launch or the kernel source changed since it was taken."""
    import glob
    import hashlib
    src = os.path.join(ROOT, "paper_2502_04093_amd", "csrc", "level3.hip")
    try:
        h = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    except OSError:
        return None
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        for line in open(path):
            if not line.startswith("traffic-json: "):
                continue
            d = json.loads(line[len("traffic-json: "):])
            if (d.get("source_sha256_16") == h and list(d.get("shape", [])) == list(shape)
                    and d.get("dtype") == ("f32" if itemsize == 4 else "f64")
                    and d.get("interp") == interp):
                v = d.get("bytes_per_launch", {}).get(f"{op}|level {level}")
                if v is not None:
                    return int(v)
    return None


def cpu_model():
    """The host CPU's model name (first processor of /proc/cpuinfo)."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(x, eb, args, ctx):
    """The oracle (plain NumPy, one core) on a cubic corner of the same field,
    and the parity of the GPU path on that corner: its stream and full
    retrieval compared byte for byte with the oracle's."""
    import hashlib

    import numpy as np
    from oracle import codec
    e = min(args.cpu_sample, *x.shape) if x.dim() == 3 else None
    sub = x[:e, :e, :e] if x.dim() == 3 else x
    xs = np.ascontiguousarray(sub.cpu().numpy())
    print(f"[bench] cpu baseline: oracle on {xs.shape}", file=sys.stderr, flush=True)
    interp = 1 if args.interp == "cubic" else 0
    t0 = time.perf_counter()
    buf = codec.compress(xs, eb, interp=interp)
    t1 = time.perf_counter()
    ref = codec.retrieve(buf, "eb", eb)
    t2 = time.perf_counter()
    gb = xs.nbytes / 1e9
    base = {"value": round(gb / (t2 - t0), 5), "unit": "GB/s", "cores": 1, "kind": "oracle",
            "host_cpus": os.cpu_count(), "host_cpu_model": cpu_model(),
            "sample": f"{'x'.join(map(str, xs.shape))} corner of the same field, same eb; "
                      f"compress {t1 - t0:.2f} s + full retrieve {t2 - t1:.2f} s",
            "compress_GBps": round(gb / (t1 - t0), 5), "retrieve_GBps": round(gb / (t2 - t1), 5)}
    s = ctx.compress(sub.contiguous(), eb, interp=args.interp)
    got = s.to_bytes()
    st = s.retrieve(eb=eb)
    fld = st.tensor().cpu().numpy().tobytes()
    st.free()
    s.free()
    parity = {"sample": f"{'x'.join(map(str, xs.shape))} corner",
              "stream_sha256": hashlib.sha256(got).hexdigest()[:16],
              "stream_equal_oracle": got == buf,
              "retrieval_equal_oracle": fld == ref.field.tobytes()}
    if x.dim() == 3:
        parity["full_size_sampled"] = sampled_parity(x, eb, args, ctx)
    return base, parity


def sampled_parity(x, eb, args, ctx, n=64):
    """The whole field in the timed launch configuration: n random outputs of
    its full retrieval against the pointwise oracle (each evaluated through
    its dependency cone)."""
    import numpy as np
    import torch
    from oracle.pointwise import Cone
    rng = np.random.default_rng(12345)
    pts = np.stack([rng.integers(0, d, size=n) for d in x.shape], axis=1)
    cone = Cone(x.cpu().numpy(), eb, 1 if args.interp == "cubic" else 0)
    s = ctx.compress(x, eb, interp=args.interp)
    st = s.retrieve(eb=eb)
    idx = torch.from_numpy(pts).to(x.device)
    got = st.tensor()[idx[:, 0], idx[:, 1], idx[:, 2]].cpu().numpy()
    st.free()
    s.free()
    ref = np.array([cone.xhat(tuple(int(v) for v in p)) for p in pts], dtype=got.dtype)
    return {"points": n, "cone_points": cone.cone_size(), "equal_oracle": got.tobytes() == ref.tobytes()}


if __name__ == "__main__":
    main()
