#!/usr/bin/env python3
"""Benchmark of the fused Array-OL downscaler on one MI355X.

One step = one pass of the fused horizontal+vertical downscale over a batch
of 300 synthetic 1920x1080 I420 frames (luma 1920x1080, chroma 960x540,
3/8 in both directions with 11 taps) resident in HBM, as one launch. The
JSON line reports output Mpixel/s (luma output pixels, 720x405 per frame),
the HBM roofline of the fused kernel, the bf16 matrix-core form of the same
batch with its max-abs error against the float64 oracle, and the CPU oracle
timed on a bounded sample on the host's cores.

    python bench.py [--gpus 1] [--steps 50] [--warmup 100]
"""

from __future__ import annotations

import argparse
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "output Mpixel/s & % HBM peak: plain int vs BF16-MFMA batched (err ≤1e-3)"
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
H, W = 1080, 1920
P, Q, TAPS = 3, 8, 11
SEED = 20110322


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# ------------------------------------------------------------------ inputs

def make_frames(n):
    import synthgen
    return synthgen.yuv420_frames(SEED, n, H, W)


def alg_bytes_per_frame(in_es, out_es):
    """Algorithmic HBM bytes of one I420 frame: every input element read once, every output written once."""
    ch, cw = H // 2, W // 2
    oy = (P * -(-H // Q), P * -(-W // Q))
    oc = (P * -(-ch // Q), P * -(-cw // Q))
    n_in = H * W + 2 * ch * cw
    n_out = oy[0] * oy[1] + 2 * oc[0] * oc[1]
    return n_in * in_es + n_out * out_es, oy


# ------------------------------------------------------------------ HBM traffic from counters

KERNEL_SOURCES = ["paper_1103_4881_amd/csrc/band.hip", "paper_1103_4881_amd/csrc/aol_internal.h"]
TRAFFIC_FILE = "profiles/k_band_u8_i420_1080p_300f_traffic.json"


def kernel_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def traffic_bytes():
    """HBM bytes per launch of the fused kernel from the committed rocprofv3 counter summary
    (FETCH_SIZE and WRITE_SIZE, each scaled by the same counter on a plain 1 GiB copy), or None
    when the kernel sources changed since the counters were taken."""
    path = os.path.join(ROOT, TRAFFIC_FILE)
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    if t.get("kernel_sha256") != kernel_hash():
        return None
    return int(t["fetch_kib"] * 1024 * t["fetch_scale"] + t["write_kib"] * 1024 * t["write_scale"])


# ------------------------------------------------------------------ GPU timing

def time_launches(launch, steps, warmup, stream):
    """Warm up, then time `steps` launches: wall clock around them (synchronised on both
    sides) and per-launch HIP events on the launch stream."""
    import torch
    for _ in range(warmup):
        launch()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s, e in ev:
        s.record(stream)
        launch()
        e.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per = [s.elapsed_time(e) for s, e in ev]  # ms
    return wall / steps * 1e3, float(np.mean(per)), float(np.median(per))


def bench_u8(Yh, Uh, Vh, steps, warmup):
    import torch
    import paper_1103_4881_amd as aol
    import synthgen
    n = Yh.shape[0]
    c = synthgen.design_taps(P, Q, TAPS)
    f = aol.Polyphase(P, Q, c)
    plan = aol.DownscalePlan([(H, W), (H // 2, W // 2), (H // 2, W // 2)], f, f, "u8")
    ins = [torch.from_numpy(a).cuda() for a in (Yh, Uh, Vh)]
    outs = [torch.empty((n,) + s, dtype=torch.uint8, device="cuda") for s in plan.out_shapes]
    stream = torch.cuda.current_stream()
    ms_step, ms_kernel, ms_med = time_launches(lambda: plan.run(ins, outs), steps, warmup, stream)
    bpf, oy = alg_bytes_per_frame(1, 1)
    res = dict(ms_step=ms_step, ms_kernel=ms_kernel, ms_kernel_median=ms_med, bytes=bpf * n,
               out_pixels=n * oy[0] * oy[1], plan=plan, ins=ins, outs=outs)
    return res


def bench_float(ins_u8, steps, warmup, fmt="bf16", check_frames=(0,)):
    """The matrix-core form on the same frames: 16-bit normalised pixels in, float32 out."""
    import torch
    import paper_1103_4881_amd as aol
    import synthgen
    from oracle import polyphase as pp
    n = ins_u8[0].shape[0]
    c = synthgen.design_taps(P, Q, TAPS)
    f = aol.Polyphase(P, Q, c)
    plan = aol.DownscalePlan([(H, W), (H // 2, W // 2), (H // 2, W // 2)], f, f, fmt)
    tdt = torch.bfloat16 if fmt == "bf16" else torch.float16
    # k/255 rounded to nearest in float32, then to the 16-bit format (nearest even)
    ins = [(x.float() / 255.0).to(tdt) for x in ins_u8]
    outs = [torch.empty((n,) + s, dtype=torch.float32, device="cuda") for s in plan.out_shapes]
    stream = torch.cuda.current_stream()
    ms_step, ms_kernel, ms_med = time_launches(lambda: plan.run(ins, outs), steps, warmup, stream)
    # max-abs error against the float64 oracle on the identical 16-bit inputs
    of = pp.Filter(P, Q, c)
    errs = []
    for fr in check_frames:
        for x16, y in zip(ins, outs):
            xin = x16[fr].float().cpu().numpy().astype(np.float64)
            ref = pp.downscale_f64(xin, of, of)
            errs.append(float(np.abs(y[fr].cpu().numpy().astype(np.float64) - ref).max()))
    bpf, oy = alg_bytes_per_frame(2, 4)
    return dict(ms_step=ms_step, ms_kernel=ms_kernel, ms_kernel_median=ms_med, bytes=bpf * n,
                out_pixels=n * oy[0] * oy[1], max_abs_err=max(errs), err_frames=list(check_frames))


# ------------------------------------------------------------------ batch of streams

BATCH_SEED = 2011
BATCH_STREAMS = 64
BATCH_FRAMES = 30


def bench_batch(fmt="u8", steps=BATCH_FRAMES, warmup=BATCH_FRAMES):
    """64 streams of uneven sizes/ratios/taps, 30 frames each; one step = one frame of every
    stream = one pointer-table update + one graph launch of the persistent kernel."""
    import torch
    import paper_1103_4881_amd as aol
    import synthgen
    mix = synthgen.stream_mix(BATCH_SEED, BATCH_STREAMS)
    filt = {}
    streams = []
    for st in mix:
        key = (st.p, st.q, st.taps)
        if key not in filt:
            filt[key] = aol.Polyphase(st.p, st.q, synthgen.design_taps(st.p, st.q, st.taps))
        streams.append((st.h, st.w, filt[key], filt[key]))
    plan = aol.BatchPlan(streams, fmt)
    # distinct buffers for every frame of every stream (each step reads memory no earlier step read)
    g = synthgen.rng_for(BATCH_SEED, 1)
    ins, outs = [], []
    for i, st in enumerate(mix):
        base = torch.from_numpy(synthgen.gradient_plane(g, st.h, st.w)).cuda()
        if fmt != "u8":
            base = (base.float() / 255.0).to(torch.bfloat16 if fmt == "bf16" else torch.float16)
        ins.append([base.clone() for _ in range(BATCH_FRAMES)])
        odt = torch.uint8 if fmt == "u8" else torch.float32
        outs.append([torch.empty(plan.out_shapes[i], dtype=odt, device="cuda") for _ in range(BATCH_FRAMES)])
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        plan.set_pointers([ins[i][0] for i in range(len(mix))], [outs[i][0] for i in range(len(mix))], s)
        plan.autotune(s)
        graph = plan.graph(s)

        # pointer arrays of every frame, checked once (a serving loop keeps them the same way)
        tables = [plan.pointer_arrays([ins[i][k] for i in range(len(mix))], [outs[i][k] for i in range(len(mix))])
                  for k in range(BATCH_FRAMES)]

        def step(k):
            plan.set_pointer_arrays(tables[k % BATCH_FRAMES], s)
            aol.aol_graph_launch(graph, s)

        for k in range(warmup):
            step(k)
        s.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        t0 = time.perf_counter()
        for k, (a, b) in enumerate(ev):
            a.record(s)
            step(k)
            b.record(s)
        s.synchronize()
        wall = time.perf_counter() - t0
    per = [a.elapsed_time(b) for a, b in ev]
    in_es, out_es = (1, 1) if fmt == "u8" else (2, 4)
    bytes_step = sum(h * w * in_es + oh * ow * out_es for (h, w), (oh, ow) in zip(plan.shapes, plan.out_shapes))
    px_step = sum(oh * ow for (oh, ow) in plan.out_shapes)
    ms_step = wall / steps * 1e3
    ms_kernel = float(np.mean(per))
    res = {"value": round(px_step / (ms_step / 1e3) / 1e6, 1), "unit": "Mpixel/s", "ms_per_step": round(ms_step, 4),
           "steps": steps, "streams": len(mix), "frames_per_stream": BATCH_FRAMES,
           "bytes_per_step": bytes_step, "out_pixels_per_step": px_step,
           "roofline": {"bound": "hbm", "achieved": round(bytes_step / (ms_kernel / 1e3) / 1e9, 1), "peak": HBM_PEAK_GBS,
                        "unit": "GB/s", "frac": round(bytes_step / (ms_kernel / 1e3) / 1e9 / HBM_PEAK_GBS, 4)},
           "schedule": json.loads(plan.schedule())}
    # correctness of the last step on a few streams against the oracle
    from oracle import polyphase as pp
    k = (warmup + steps - 1) % BATCH_FRAMES
    errs = []
    for i in range(0, len(mix), 16):
        st = mix[i]
        of = pp.Filter(st.p, st.q, synthgen.design_taps(st.p, st.q, st.taps))
        x = ins[i][k].float().cpu().numpy()
        y = outs[i][k].float().cpu().numpy()
        if fmt == "u8":
            errs.append(float(np.abs(y - pp.downscale_u8(x.astype(np.uint8), of, of)).max()))
        else:
            errs.append(float(np.abs(y - pp.downscale_f64(x.astype(np.float64), of, of)).max()))
    res["max_abs_err_sampled_streams"] = max(errs)
    plan.close()
    del ins, outs
    torch.cuda.empty_cache()
    return res


# ------------------------------------------------------------------ generic repetition

GEN_SHAPE = (64, 1024, 1024)


def bench_generic(steps=10, warmup=20):
    """64x1024x1024 float32, random non-identity tiler, 5x5 weighted sum."""
    import torch
    import paper_1103_4881_amd as aol
    import synthgen
    from oracle import generic as gn
    from oracle.arrayol import Tiler
    rt = synthgen.random_tiler(BATCH_SEED, array_shape=GEN_SHAPE, pat_shape=(5, 5))
    A = synthgen.rng_for(BATCH_SEED, 1).uniform(-1, 1, size=GEN_SHAPE).astype(np.float32)
    w = synthgen.rng_for(BATCH_SEED, 2).uniform(-1, 1, size=(5, 5)).astype(np.float32)
    tin = aol.make_tiler(rt.array_shape, rt.rep_shape, rt.pat_shape, rt.origin, rt.paving, rt.fitting)
    plan = aol.WeightedSumPlan(tin, aol.identity_out_tiler(rt.rep_shape), w)
    x = torch.from_numpy(A).cuda()
    y = torch.empty(plan.out_shape, dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream()
    ms_step, ms_kernel, _ = time_launches(lambda: plan.run(x, y), steps, warmup, stream)
    # footprint: every input element some pattern element reads (bitmap on the device,
    # a few large batched index computations)
    R = rt.rep_shape
    seen = torch.zeros(int(np.prod(GEN_SHAPE)), dtype=torch.bool, device="cuda")
    S = torch.tensor(GEN_SHAPE, device="cuda").view(3, 1, 1, 1, 1)
    strides = [GEN_SHAPE[1] * GEN_SHAPE[2], GEN_SHAPE[2], 1]
    P = torch.tensor(rt.paving, device="cuda")
    F = torch.tensor(rt.fitting, device="cuda")
    o = torch.tensor(rt.origin, device="cuda")
    pat = torch.stack(torch.meshgrid(torch.arange(5, device="cuda"), torch.arange(5, device="cuda"),
                                     indexing="ij")).reshape(2, -1)  # [2, 25]
    foff = (F.view(3, 2, 1) * pat.view(1, 2, 25)).sum(1).view(3, 1, 1, 1, 25)
    r1 = torch.arange(R[1], device="cuda").view(1, 1, -1, 1, 1)
    r2 = torch.arange(R[2], device="cuda").view(1, 1, 1, -1, 1)
    for c0 in range(0, R[0], 32):
        r0 = torch.arange(c0, min(c0 + 32, R[0]), device="cuda").view(1, -1, 1, 1, 1)
        v = (o.view(3, 1, 1, 1, 1) + P[:, 0].view(3, 1, 1, 1, 1) * r0 + P[:, 1].view(3, 1, 1, 1, 1) * r1
             + P[:, 2].view(3, 1, 1, 1, 1) * r2 + foff)
        v = torch.remainder(v, S)
        flat = v[0] * strides[0] + v[1] * strides[1] + v[2]
        seen[flat.reshape(-1)] = True
    footprint = int(seen.sum().item())
    n_out = int(np.prod(R))
    alg_bytes = 4 * footprint + 4 * n_out
    # sampled parity against the float64 oracle
    g = synthgen.rng_for(BATCH_SEED, 3)
    rs = np.stack([g.integers(0, n, size=4000) for n in R])
    ref, mag = gn.weighted_sum_at(A, Tiler(rt.array_shape, rt.origin, rt.paving.tolist(), rt.fitting.tolist(),
                                           rt.pat_shape), w, rs)
    got = y.cpu().numpy()[tuple(rs)].astype(np.float64)
    rel = float((np.abs(got - ref) / np.maximum(mag, 1e-30)).max())
    gbs = alg_bytes / (ms_kernel / 1e3) / 1e9
    plan.close()
    return {"value": round(n_out / (ms_step / 1e3) / 1e9, 3), "unit": "Goutput/s", "ms_per_step": round(ms_step, 4),
            "outputs": n_out, "footprint_elems": footprint, "alg_bytes": alg_bytes,
            "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(gbs / HBM_PEAK_GBS, 4)},
            "max_rel_err_sampled": rel, "tolerance_rel": 1e-5,
            "tiler": {"paving": rt.paving.tolist(), "fitting": rt.fitting.tolist(), "origin": list(rt.origin),
                      "rep_shape": list(R)}}


# ------------------------------------------------------------------ CPU oracle baseline

_CPU_FRAMES = None


def _cpu_one(i):
    from oracle import polyphase as pp
    import synthgen
    c = synthgen.design_taps(P, Q, TAPS)
    f = pp.Filter(P, Q, c)
    Y, U, V = _CPU_FRAMES
    for a in (Y[i], U[i], V[i]):
        pp.downscale_u8(a, f, f)
    return i


def cpu_baseline(n_frames, repeats):
    """The CPU oracle (vectorised NumPy definition) over a sample of frames, one process per core;
    the sample is passed `repeats` times so that the timed CPU work lasts 10-30 s."""
    global _CPU_FRAMES
    _CPU_FRAMES = make_frames(n_frames)
    cores = max(1, min(16, os.cpu_count() or 1))
    ctx = mp.get_context("fork")
    with ctx.Pool(cores) as pool:
        pool.map(_cpu_one, range(min(cores, n_frames)))  # warm the workers (imports)
        t0 = time.perf_counter()
        pool.map(_cpu_one, [i % n_frames for i in range(n_frames * repeats)], chunksize=1)
        dt = time.perf_counter() - t0
    _, oy = alg_bytes_per_frame(1, 1)
    done = n_frames * repeats
    return dict(value=done * oy[0] * oy[1] / dt / 1e6, unit="Mpixel/s", cores=cores, kind="oracle",
                sample=f"{n_frames} I420 1920x1080 frames of the same workload, each downscaled {repeats} times "
                       f"({done} frames), integer oracle (numpy), {cores} processes, {dt:.1f} s")


# ------------------------------------------------------------------ main

def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--frames", type=int, default=300)
    ap.add_argument("--cpu-frames", type=int, default=384)
    ap.add_argument("--cpu-repeats", type=int, default=10)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-float", action="store_true")
    ap.add_argument("--only", choices=["u8", "bf16", "batch", "generic"], default=None,
                    help="run one workload only (for profiling)")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-generic", action="store_true")
    ap.add_argument("--hash", action="store_true", help="print the fused kernel's source hash and exit")
    ap.add_argument("--copy-calib", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy 3 times (scale for HBM byte counters)")
    args = ap.parse_args()
    if args.hash:
        print(kernel_hash())
        return
    if args.copy_calib:
        import torch
        src = torch.ones(1 << 30, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calib_bytes": 1 << 30, "launches": 3}))
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (frames and streams are "
              "independent repetitions; see the sharding notes). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    cpu = None
    if not args.no_cpu:  # before the GPU is initialised: the pool forks this process
        t = time.time()
        cpu = cpu_baseline(args.cpu_frames, args.cpu_repeats)
        log(f"cpu baseline in {time.time() - t:.1f} s: {cpu['value']:.1f} Mpixel/s")

    import torch
    torch.cuda.set_device(0)
    t = time.time()
    Yh, Uh, Vh = make_frames(args.frames)
    log(f"generated {args.frames} I420 frames in {time.time() - t:.1f} s")

    out = {"metric": METRIC}
    u8 = None
    if args.only in (None, "u8"):
        u8 = bench_u8(Yh, Uh, Vh, args.steps, args.warmup)
        log(f"u8 fused: {u8['ms_step']:.3f} ms/step, kernel {u8['ms_kernel']:.3f} ms")
    fl = None
    if not args.no_float and args.only in (None, "bf16"):
        import torch as _t
        ins_u8 = u8["ins"] if u8 else [_t.from_numpy(a).cuda() for a in (Yh, Uh, Vh)]
        if u8:
            del u8["outs"]
            _t.cuda.empty_cache()
        fl = bench_float(ins_u8, args.steps, args.warmup, "bf16")
        log(f"bf16 fused: {fl['ms_step']:.3f} ms/step, kernel {fl['ms_kernel']:.3f} ms, err {fl['max_abs_err']:.2e}")

    extra = {}
    if not args.no_batch and args.only in (None, "batch"):
        extra["batch_u8"] = bench_batch("u8")
        log(f"batch u8: {extra['batch_u8']['ms_per_step']:.3f} ms/step")
        if not args.no_float:
            extra["batch_bf16"] = bench_batch("bf16")
            log(f"batch bf16: {extra['batch_bf16']['ms_per_step']:.3f} ms/step")
    if not args.no_generic and args.only in (None, "generic"):
        extra["generic"] = bench_generic()
        log(f"generic: {extra['generic']['ms_per_step']:.3f} ms/step")
    if args.only in ("batch", "generic"):
        print(json.dumps({"metric": METRIC, **extra}), flush=True)
        return

    main_res = u8 if u8 else fl
    dtype = "u8" if u8 else "bf16"
    value = main_res["out_pixels"] / (main_res["ms_step"] / 1e3) / 1e6
    gbs = main_res["bytes"] / (main_res["ms_kernel"] / 1e3) / 1e9
    out.update({
        "value": round(value, 1),
        "unit": "Mpixel/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(main_res["ms_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
        "config": {"workload": f"I420 1920x1080 x{args.frames} frames, 3/8 both axes, 11 taps, fused H+V",
                   "frames": args.frames, "height": H, "width": W, "p": P, "q": Q, "taps": TAPS,
                   "parallelism": "single GPU"},
        "hbm_frac": round(main_res["bytes"] / (main_res["ms_step"] / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
        "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": traffic_bytes() if u8 else None,
                     "kernel": "aol::k_band<u8>" if u8 else "aol::k_band<bf16>",
                     "alg_bytes_per_launch": main_res["bytes"],
                     "kernel_ms_mean": round(main_res["ms_kernel"], 4)},
    })
    if fl and u8:
        fgbs = fl["bytes"] / (fl["ms_kernel"] / 1e3) / 1e9
        out["bf16"] = {"value": round(fl["out_pixels"] / (fl["ms_step"] / 1e3) / 1e6, 1), "unit": "Mpixel/s",
                       "ms_per_step": round(fl["ms_step"], 4), "max_abs_err": fl["max_abs_err"], "tolerance": 1e-3,
                       "err_frames": fl["err_frames"],
                       "roofline": {"bound": "hbm", "achieved": round(fgbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                    "frac": round(fgbs / HBM_PEAK_GBS, 4), "alg_bytes_per_launch": fl["bytes"]}}
    out.update(extra)
    if cpu:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
