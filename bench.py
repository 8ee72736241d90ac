#!/usr/bin/env python3
"""Benchmark of the fused Array-OL downscaler on one MI355X.

One step = one pass of the fused horizontal+vertical downscale over a batch
of 300 synthetic 1920x1080 I420 frames (luma 1920x1080, chroma 960x540,
3/8 in both directions with 11 taps) resident in HBM, as one launch. The
JSON line reports output Mpixel/s (luma output pixels, 720x405 per frame),
the HBM roofline of the fused kernel, the bf16 matrix-core form of the same
batch with its max-abs error against the float64 oracle, and the CPU oracle
timed on a bounded sample on the host's cores.

    python bench.py [--gpus 1] [--steps 20] [--warmup 5]
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


def cpu_baseline(n_frames):
    """The CPU oracle (vectorised NumPy definition) over a sample of frames, one process per core."""
    global _CPU_FRAMES
    _CPU_FRAMES = make_frames(n_frames)
    cores = max(1, min(16, os.cpu_count() or 1))
    ctx = mp.get_context("fork")
    with ctx.Pool(cores) as pool:
        pool.map(_cpu_one, range(min(cores, n_frames)))  # warm the workers (imports)
        t0 = time.perf_counter()
        pool.map(_cpu_one, range(n_frames), chunksize=1)
        dt = time.perf_counter() - t0
    _, oy = alg_bytes_per_frame(1, 1)
    return dict(value=n_frames * oy[0] * oy[1] / dt / 1e6, unit="Mpixel/s", cores=cores, kind="oracle",
                sample=f"{n_frames} I420 1920x1080 frames, integer oracle (numpy), {cores} processes, {dt:.2f} s")


# ------------------------------------------------------------------ main

def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--frames", type=int, default=300)
    ap.add_argument("--cpu-frames", type=int, default=384)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-float", action="store_true")
    ap.add_argument("--only", choices=["u8", "bf16"], default=None, help="run one kernel only (for profiling)")
    ap.add_argument("--copy-calib", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy 3 times (scale for HBM byte counters)")
    args = ap.parse_args()
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
        cpu = cpu_baseline(args.cpu_frames)
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
                     "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": "k_fused<u8>" if u8 else "k_fused<bf16>",
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
    if cpu:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
