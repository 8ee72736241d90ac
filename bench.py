#!/usr/bin/env python3
"""Benchmark of the fused Array-OL downscaler on one MI355X.

One step = one pass of the fused horizontal+vertical downscale over a batch
of 300 synthetic 1920x1080 I420 frames (luma 1920x1080, chroma 960x540,
3/8 in both directions with 11 taps) resident in HBM, as one launch. The
JSON line reports output Mpixel/s (luma output pixels, 720x405 per frame),
the HBM roofline of the fused kernel (against the 8 TB/s datasheet figure
and a copy measured on the same GPU), a bit-exactness check of sampled
frames of the timed launch against the oracle, and beside it:

  * config1: latency of one 640x480 frame (cache resident, not an HBM figure);
  * bf16 / fp16: the matrix-core form of the same batch, max-abs error
    against the float64 oracle per plane and per checked frame;
  * batch_u8 / batch_bf16: 64 uneven streams, one launch per step in a graph,
    plus the subset of their 1920x1080 streams;
  * generic: the 5x5 weighted-sum repetition over a 64x1024x1024 array;
  * cpu_baseline: the CPU oracle on a bounded sample (all granted cores, one
    process, and the Array-OL interpreter on the 640x480 frame).

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
WARM_SECONDS = 0.5  # launches before every timed region, so the clocks have ramped up


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


def check_frames(n):
    return sorted({0, n // 2, n - 1})


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

def warm(launch, warmup, sync):
    """`warmup` launches, then more until WARM_SECONDS have passed (clock ramp after idle)."""
    for _ in range(warmup):
        launch()
    sync()
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < WARM_SECONDS:
        for _ in range(10):
            launch()
        sync()


def time_launches(launch, steps, warmup, stream):
    """Warm up, then time `steps` launches back to back: the wall clock around them
    (synchronised on both sides) and two HIP events on the launch stream, one before the
    first and one after the last (the mean launch duration over the timed region). Then
    `steps` more, each between two events, for the median (events between the launches
    lengthen the steps they bracket, so they stay out of the timed region)."""
    import torch
    warm(launch, warmup, torch.cuda.synchronize)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(steps):
        launch()
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    mean = e0.elapsed_time(e1) / steps
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    for s, e in ev:
        s.record(stream)
        launch()
        e.record(stream)
    torch.cuda.synchronize()
    per = [s.elapsed_time(e) for s, e in ev]  # ms
    return wall / steps * 1e3, float(mean), float(np.median(per))


def copy_peak(n_bytes=1 << 30, reps=20):
    """HBM bandwidth of a plain device-to-device copy (torch's copy kernel) on this GPU:
    2 * n_bytes per launch over the median HIP-event duration."""
    import torch
    src = torch.ones(n_bytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    stream = torch.cuda.current_stream()
    _, _, med = time_launches(lambda: dst.copy_(src), reps, 5, stream)
    del src, dst
    torch.cuda.empty_cache()
    return 2 * n_bytes / (med / 1e3) / 1e9


def bench_u8(Yh, Uh, Vh, steps, warmup):
    import torch
    import paper_1103_4881_amd as aol
    import synthgen
    from oracle import polyphase as pp
    n = Yh.shape[0]
    c = synthgen.design_taps(P, Q, TAPS)
    f = aol.Polyphase(P, Q, c)
    plan = aol.DownscalePlan([(H, W), (H // 2, W // 2), (H // 2, W // 2)], f, f, "u8")
    ins = [torch.from_numpy(a).cuda() for a in (Yh, Uh, Vh)]
    outs = [torch.empty((n,) + s, dtype=torch.uint8, device="cuda") for s in plan.out_shapes]
    stream = torch.cuda.current_stream()
    ms_step, ms_kernel, ms_med = time_launches(lambda: plan.run(ins, outs), steps, warmup, stream)
    # the timed launch's outputs, sampled frames against the integer oracle (every element)
    of = pp.Filter(P, Q, c)
    mism, checked = 0, 0
    for fr in check_frames(n):
        for a, o in zip((Yh, Uh, Vh), outs):
            ref = pp.downscale_u8(a[fr], of, of)
            mism += int((o[fr].cpu().numpy() != ref).sum())
            checked += ref.size
    bpf, oy = alg_bytes_per_frame(1, 1)
    return dict(ms_step=ms_step, ms_kernel=ms_kernel, ms_kernel_median=ms_med, bytes=bpf * n,
                out_pixels=n * oy[0] * oy[1], plan=plan, ins=ins, outs=outs, schedule=plan.schedule(n),
                mismatches=mism, checked_elements=checked, checked_frames=check_frames(n))


def bench_unfused(u8, Yh, Uh, Vh, steps, warmup):
    """The unfused form (a horizontal and a vertical row-pass kernel, the uint8 intermediate
    through HBM) on the same frames and plan, with a workspace for all frames (one launch per
    pass): outputs identical to the fused launch's, and the time and bytes fusion saves."""
    import torch
    plan = u8["plan"]
    ins = u8["ins"]
    n = ins[0].shape[0]
    work = torch.empty(plan.workspace_bytes() * n, dtype=torch.uint8, device="cuda")
    outs = [torch.empty((n,) + s, dtype=torch.uint8, device="cuda") for s in plan.out_shapes]
    stream = torch.cuda.current_stream()
    ms_step, ms_kernel, ms_med = time_launches(lambda: plan.run_unfused(ins, outs, work), steps, warmup, stream)
    same = all(torch.equal(a, b) for a, b in zip(outs, u8["outs"]))
    # bytes: the fused launch's, plus the intermediate written once and read once
    ch, cw = H // 2, W // 2
    z = H * (P * -(-W // Q)) + 2 * ch * (P * -(-cw // Q))
    bytes_unf = u8["bytes"] + 2 * z * n
    del work, outs
    torch.cuda.empty_cache()
    gbs = bytes_unf / (ms_kernel / 1e3) / 1e9
    return {"ms_per_step": round(ms_step, 4), "ms_two_passes_mean": round(ms_kernel, 4),
            "ms_two_passes_median": round(ms_med, 4), "identical_to_fused": bool(same),
            "bytes_per_step": bytes_unf, "intermediate_bytes": 2 * z * n,
            "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(gbs / HBM_PEAK_GBS, 4)},
            "fusion_gain": {"time": round(ms_step / u8["ms_step"], 3),
                            "bytes": round(bytes_unf / u8["bytes"], 3)}}


LIN_FRAMES = 30
VALU_MAC_PEAK = 256 * 64 * 2 * 2.4e9  # v_dot2_i32_i16: 2 MACs per lane, a wave64 instruction per CU and cycle


def _frames_spec(spec, frames):
    """A tiler spec with a leading frame dimension in the array and the repetition space."""
    import synthgen
    paving = [[1] + [0] * len(spec.paving[0])] + [[0] + list(row) for row in spec.paving]
    fitting = [[0] * len(spec.fitting[0])] + [list(row) for row in spec.fitting]
    return synthgen.TilerSpec((frames,) + tuple(spec.array_shape), (0,) + tuple(spec.origin), paving, fitting,
                              spec.pat_shape)


def bench_linear(steps=20, warmup=10, n=LIN_FRAMES):
    """The linear integer repetition (wider elementary tasks): interleaved RGB 1920x1080 frames to
    planar colour components (3 -> 3 per pixel), the composition back to RGB, and a non-separable
    2-D polyphase downscale of luma frames (3/8 on both axes, 11 x 11 kernels per output phase:
    a 17 x 17 window -> 3 x 3 outputs per repetition); frames as a repetition dimension."""
    import torch
    import paper_1103_4881_amd as aol
    import synthgen
    from oracle import linear as ln
    from oracle.arrayol import Tiler
    h, w = H, W
    ot = lambda sp: Tiler(sp.array_shape, sp.origin, sp.paving, sp.fitting, sp.pat_shape)
    at = lambda sp, rep: aol.make_tiler(sp.array_shape, rep, sp.pat_shape, sp.origin, sp.paving, sp.fitting)
    res = {}
    stream = torch.cuda.current_stream()
    rgb = np.stack([synthgen.uniform_frame(SEED + 7 + f, h, 3 * w) for f in range(n)])
    rep0, tin0, tout0 = synthgen.rgb_to_planar_tilers(h, w)
    rep20, tin20, tout20 = synthgen.planar_to_rgb_tilers(h, w)
    rep_p, tin_p, tout_p, _, span = synthgen.polyphase2d_tilers(h, w, P, Q, TAPS)
    Wp = synthgen.polyphase2d_weights(SEED, P, Q, TAPS)
    x_rgb = torch.from_numpy(rgb).cuda()
    planar = torch.empty((n, 3, h, w), dtype=torch.uint8, device="cuda")
    back = torch.empty((n, h, 3 * w), dtype=torch.uint8, device="cuda")
    luma = x_rgb.view(n, h, 3 * w)[:, :, :w].contiguous()
    down = torch.empty((n, P * -(-h // Q), P * -(-w // Q)), dtype=torch.uint8, device="cuda")
    cases = [("rgb_to_planar_ycc", x_rgb, planar, rep0, tin0, tout0, synthgen.RGB_TO_YCC_W, synthgen.RGB_TO_YCC_BIAS),
             ("planar_ycc_to_rgb", planar, back, rep20, tin20, tout20, synthgen.YCC_TO_RGB_W,
              synthgen.YCC_TO_RGB_BIAS),
             ("polyphase2d_3_8_11x11", luma, down, rep_p, tin_p, tout_p, Wp, None)]
    for name, x, y, rep1, ti1, to1, Wt, bias in cases:
        rep, ti, to = (n,) + tuple(rep1), _frames_spec(ti1, n), _frames_spec(to1, n)
        plan = aol.LinearPlan(at(ti, rep), at(to, rep), Wt, bias)
        ms_step, ms_kernel, ms_med = time_launches(lambda: plan.run(x, y), steps, warmup, stream)
        plan.close()
        torch.cuda.synchronize()
        n_in, n_out = int(np.prod(ti1.pat_shape)), int(np.prod(to1.pat_shape))
        nrep = int(np.prod(rep))
        alg_bytes = x.numel() + y.numel()  # every input element read once, every output written once
        mism = 0
        xh = x.cpu().numpy()
        yh = y.cpu().numpy()
        for f in (0, n - 1):
            ref, _ = ln.linear_u8(xh[f], ot(ti1), Wt, bias, ot(to1), rep1)
            mism += int((yh[f] != ref).sum())
        gbs = alg_bytes / (ms_kernel / 1e3) / 1e9
        macs = nrep * n_in * n_out
        e = {"ms_per_step": round(ms_step, 4), "kernel_ms_median": round(ms_med, 4), "frames": n,
             "repetitions": nrep, "pattern_in": n_in, "pattern_out": n_out, "alg_bytes": alg_bytes,
             "hbm": {"achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(gbs / HBM_PEAK_GBS, 4)},
             "mismatches_first_last_frame": mism}
        tmac = macs / (ms_kernel / 1e3) / 1e12
        e["alu"] = {"achieved": round(tmac, 2), "peak": round(VALU_MAC_PEAK / 1e12, 1), "unit": "TMAC/s",
                    "frac": round(tmac * 1e12 / VALU_MAC_PEAK, 4), "macs_per_launch": macs}
        e["bound"] = "hbm" if e["hbm"]["frac"] >= e["alu"]["frac"] else "alu"
        res[name] = e
        log(f"linear {name}: {ms_step:.3f} ms/step, {gbs:.0f} GB/s, {tmac:.1f} TMAC/s, mismatches {mism}")
    del x_rgb, planar, back, luma, down
    torch.cuda.empty_cache()
    return res


CIF_FRAMES = 2000


def bench_cif(n=CIF_FRAMES):
    """The paper's own workload: I420 CIF frames (352x288 luma), 3/8 along lines and 4/9 along
    columns (-> 132x128), frames in host memory. The host-to-host pipeline in four forms: one
    frame at a time with no overlap (pageable, then pinned host memory), one frame at a time with
    four frames in flight, and groups of 50 frames with three groups in flight (pinned). Stage
    times are sums of per-group GPU events; `transfer_share` is the copies' part of the stage
    time, `overlap` the stage time over the span from the first copy to the last."""
    import torch
    import paper_1103_4881_amd as aol
    import synthgen
    from oracle import polyphase as pp
    planes = synthgen.yuv420_frames(SEED + 1, n, 288, 352)
    ch, cv = synthgen.design_taps(3, 8, 11), synthgen.design_taps(4, 9, 11)
    plan = aol.DownscalePlan([(288, 352), (144, 176), (144, 176)], aol.Polyphase(3, 8, ch),
                             aol.Polyphase(4, 9, cv), "u8")
    pinned_in = [torch.from_numpy(a).pin_memory() for a in planes]
    pageable_in = [torch.from_numpy(a) for a in planes]
    res = {"frames": n, "in": "352x288 I420", "out": "132x128 I420", "h": "3/8, 11 taps", "v": "4/9, 11 taps",
           "bytes_in": n * (288 * 352 + 2 * 144 * 176), "bytes_out": n * (128 * 132 + 2 * 64 * 66), "forms": {}}
    of, ov = pp.Filter(3, 8, ch), pp.Filter(4, 9, cv)
    mism = 0
    for name, batch, depth, pinned in [("per_frame_serial_pageable", 1, 1, False), ("per_frame_serial", 1, 1, True),
                                       ("per_frame_overlapped", 1, 4, True), ("groups_of_50", 50, 3, True)]:
        ins = pinned_in if pinned else pageable_in
        outs = [torch.empty((n,) + s, dtype=torch.uint8, pin_memory=pinned) for s in plan.out_shapes]
        pipe = aol.Pipeline(plan, batch, depth)
        pipe.run([t[:2 * batch] for t in ins], [o[:2 * batch] for o in outs])  # warm-up
        st = pipe.run(ins, outs)
        pipe.close()
        for fr in check_frames(n):
            for o, a in zip(outs, planes):
                mism += int((o[fr].numpy() != pp.downscale_u8(a[fr], of, ov)).sum())
        stage = st["h2d_ms"] + st["kernel_ms"] + st["d2h_ms"]
        res["forms"][name] = {
            "batch_frames": batch, "depth": depth, "host_memory": "pinned" if pinned else "pageable",
            "wall_ms": round(st["wall_ms"], 2), "span_ms": round(st["span_ms"], 2),
            "h2d_ms": round(st["h2d_ms"], 2), "kernel_ms": round(st["kernel_ms"], 2), "d2h_ms": round(st["d2h_ms"], 2),
            "transfer_share": round((st["h2d_ms"] + st["d2h_ms"]) / stage, 3),
            "overlap": round(stage / st["span_ms"], 3) if st["span_ms"] > 0 else None,
            "frames_per_s": round(n / (st["wall_ms"] / 1e3), 1),
            "h2d_gbs": round(st["h2d_bytes"] / (st["h2d_ms"] / 1e3) / 1e9, 2),
            "d2h_gbs": round(st["d2h_bytes"] / (st["d2h_ms"] / 1e3) / 1e9, 2)}
        log(f"cif {name}: {st['wall_ms']:.1f} ms wall, h2d {st['h2d_ms']:.1f} kernel {st['kernel_ms']:.1f} "
            f"d2h {st['d2h_ms']:.1f} ms")
    res["mismatches_sampled_frames"] = mism
    plan.close()
    return res


def bench_config1(reps=100, warmup=200):
    """One 640x480 uniform random frame -> 180x240 (3/8, 11 taps): launch latency. The 350 KB
    working set stays in the caches, so this is a latency figure, not an HBM measurement."""
    import torch
    import paper_1103_4881_amd as aol
    import synthgen
    from oracle import polyphase as pp
    X = synthgen.uniform_frame(2024, 480, 640)
    c = synthgen.design_taps(P, Q, TAPS)
    f = aol.Polyphase(P, Q, c)
    plan = aol.DownscalePlan([(480, 640)], f, f, "u8")
    x = torch.from_numpy(X).cuda()[None]
    y = torch.empty((1, 180, 240), dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()
    _, mean, med = time_launches(lambda: plan.run([x], [y]), reps, warmup, stream)
    ok = bool(np.array_equal(y[0].cpu().numpy(), pp.downscale_u8(X, pp.Filter(P, Q, c), pp.Filter(P, Q, c))))
    sched = plan.schedule(1)
    plan.close()
    return {"us_median": round(med * 1e3, 2), "us_mean": round(mean * 1e3, 2), "launches": reps,
            "out_mpixel_per_s": round(180 * 240 / (med / 1e3) / 1e6, 1), "bit_exact": ok,
            "note": "one 640x480 frame; 350 KB working set, cache resident: latency, not HBM throughput",
            "schedule": sched}


def bench_float(ins_u8, steps, warmup, fmt="bf16"):
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
    # max-abs error against the float64 oracle on the identical 16-bit inputs, per plane and frame
    of = pp.Filter(P, Q, c)
    errs = {}
    for fr in check_frames(n):
        for name, x16, y in zip("YUV", ins, outs):
            xin = x16[fr].float().cpu().numpy().astype(np.float64)
            ref = pp.downscale_f64(xin, of, of)
            errs[f"{name}{fr}"] = float(np.abs(y[fr].cpu().numpy().astype(np.float64) - ref).max())
    bpf, oy = alg_bytes_per_frame(2, 4)
    plan.close()
    del ins, outs
    torch.cuda.empty_cache()
    return dict(ms_step=ms_step, ms_kernel=ms_kernel, ms_kernel_median=ms_med, bytes=bpf * n,
                out_pixels=n * oy[0] * oy[1], max_abs_err=max(errs.values()), err_per_plane_frame=errs)


def float_entry(fl):
    fgbs = fl["bytes"] / (fl["ms_kernel"] / 1e3) / 1e9
    return {"value": round(fl["out_pixels"] / (fl["ms_step"] / 1e3) / 1e6, 1), "unit": "Mpixel/s",
            "ms_per_step": round(fl["ms_step"], 4), "kernel_ms_median": round(fl["ms_kernel_median"], 4),
            "max_abs_err": fl["max_abs_err"], "tolerance": 1e-3,
            "max_abs_err_per_plane_frame": fl["err_per_plane_frame"],
            "roofline": {"bound": "hbm", "achieved": round(fgbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(fgbs / HBM_PEAK_GBS, 4), "alg_bytes_per_launch": fl["bytes"]}}


# ------------------------------------------------------------------ batch of streams

BATCH_SEED = 2011
BATCH_STREAMS = 64
BATCH_FRAMES = 30


def bench_batch(fmt="u8", steps=BATCH_FRAMES, warmup=BATCH_FRAMES, only_size=None):
    """64 streams of uneven sizes/ratios/taps, 30 frames each; one step = one frame of every
    stream = one launch of the persistent kernel over that frame slot's buffer set.
    only_size=(h, w): the subset of the mix's streams of that size."""
    import torch
    import paper_1103_4881_amd as aol
    import synthgen
    from oracle import polyphase as pp
    mix = synthgen.stream_mix(BATCH_SEED, BATCH_STREAMS)
    if only_size:
        mix = [s for s in mix if (s.h, s.w) == tuple(only_size)]
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

        # one buffer set (pointer table) per frame slot, made once, as a serving loop over a
        # ring of frame buffers keeps them: a step is one launch of the persistent kernel
        # (measured faster than a pointer update + launch, or one graph launch per slot)
        sets = [plan.buffers(plan.pointer_arrays([ins[i][k] for i in range(len(mix))],
                                                 [outs[i][k] for i in range(len(mix))]))
                for k in range(BATCH_FRAMES)]
        count = [0]

        def step():
            plan.run_buffers(sets[count[0] % BATCH_FRAMES], s)
            count[0] += 1

        ms_step, ms_kernel, ms_med = time_launches(step, steps, warmup, s)

        # consecutive steps on two streams (they write different frame slots and share only
        # read-only tables): the next step's workgroups start on the compute units the
        # previous step's last workgroups leave idle
        s2 = torch.cuda.Stream()
        pair = (s, s2)

        def step2():
            plan.run_buffers(sets[count[0] % BATCH_FRAMES], pair[count[0] & 1])
            count[0] += 1

        warm(step2, warmup, torch.cuda.synchronize)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            step2()
        torch.cuda.synchronize()
        ms_two = (time.perf_counter() - t0) / steps * 1e3
    in_es, out_es = (1, 1) if fmt == "u8" else (2, 4)
    bytes_step = sum(h * w * in_es + oh * ow * out_es for (h, w), (oh, ow) in zip(plan.shapes, plan.out_shapes))
    px_step = sum(oh * ow for (oh, ow) in plan.out_shapes)
    gbs = bytes_step / (ms_kernel / 1e3) / 1e9
    res = {"value": round(px_step / (ms_step / 1e3) / 1e6, 1), "unit": "Mpixel/s", "ms_per_step": round(ms_step, 4),
           "step_ms_median": round(ms_med, 4), "step_ms_mean": round(ms_kernel, 4),
           "steps": steps, "streams": len(mix), "frames_per_stream": BATCH_FRAMES,
           "bytes_per_step": bytes_step, "out_pixels_per_step": px_step,
           "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS,
                        "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4),
                        "frac_median": round(bytes_step / (ms_med / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
                        "frac_wall": round(bytes_step / (ms_step / 1e3) / 1e9 / HBM_PEAK_GBS, 4)},
           "schedule": json.loads(plan.schedule()),
           "two_streams": {"ms_per_step": round(ms_two, 4), "value": round(px_step / (ms_two / 1e3) / 1e6, 1),
                           "frac_wall": round(bytes_step / (ms_two / 1e3) / 1e9 / HBM_PEAK_GBS, 4)}}
    # the last step's outputs of every stream against the oracle
    k = (count[0] - 1) % BATCH_FRAMES
    errs = []
    for i, st in enumerate(mix):
        of = pp.Filter(st.p, st.q, synthgen.design_taps(st.p, st.q, st.taps))
        x = ins[i][k].float().cpu().numpy()
        y = outs[i][k].float().cpu().numpy()
        if fmt == "u8":
            errs.append(float(np.abs(y - pp.downscale_u8(x.astype(np.uint8), of, of)).max()))
        else:
            errs.append(float(np.abs(y - pp.downscale_f64(x.astype(np.float64), of, of)).max()))
    res["max_abs_err_all_streams"] = max(errs)
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
    ms_step, ms_kernel, ms_med = time_launches(lambda: plan.run(x, y), steps, warmup, stream)
    # footprint: every input element some pattern element reads (bitmap on the device,
    # a few large batched index computations)
    R = rt.rep_shape
    seen = torch.zeros(int(np.prod(GEN_SHAPE)), dtype=torch.bool, device="cuda")
    S = torch.tensor(GEN_SHAPE, device="cuda").view(3, 1, 1, 1, 1)
    strides = [GEN_SHAPE[1] * GEN_SHAPE[2], GEN_SHAPE[2], 1]
    Pv = torch.tensor(rt.paving, device="cuda")
    F = torch.tensor(rt.fitting, device="cuda")
    o = torch.tensor(rt.origin, device="cuda")
    pat = torch.stack(torch.meshgrid(torch.arange(5, device="cuda"), torch.arange(5, device="cuda"),
                                     indexing="ij")).reshape(2, -1)  # [2, 25]
    foff = (F.view(3, 2, 1) * pat.view(1, 2, 25)).sum(1).view(3, 1, 1, 1, 25)
    r1 = torch.arange(R[1], device="cuda").view(1, 1, -1, 1, 1)
    r2 = torch.arange(R[2], device="cuda").view(1, 1, 1, -1, 1)
    for c0 in range(0, R[0], 32):
        r0 = torch.arange(c0, min(c0 + 32, R[0]), device="cuda").view(1, -1, 1, 1, 1)
        v = (o.view(3, 1, 1, 1, 1) + Pv[:, 0].view(3, 1, 1, 1, 1) * r0 + Pv[:, 1].view(3, 1, 1, 1, 1) * r1
             + Pv[:, 2].view(3, 1, 1, 1, 1) * r2 + foff)
        v = torch.remainder(v, S)
        flat = v[0] * strides[0] + v[1] * strides[1] + v[2]
        seen[flat.reshape(-1)] = True
    footprint = int(seen.sum().item())
    del seen
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
    del x, y
    torch.cuda.empty_cache()
    return {"value": round(n_out / (ms_step / 1e3) / 1e9, 3), "unit": "Goutput/s", "ms_per_step": round(ms_step, 4),
            "kernel_ms_median": round(ms_med, 4), "outputs": n_out, "footprint_elems": footprint,
            "alg_bytes": alg_bytes,
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


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(n_frames, repeats, single_frames):
    """The CPU oracle (vectorised NumPy definition, one BLAS thread per process) over a sample
    of frames: one process per granted core (at most 16, the host share of one GPU), the sample
    passed `repeats` times so the timed CPU work lasts 10-30 s; then one process alone (the
    analogue of a sequential program) on `single_frames` frames; then the Array-OL interpreter
    on the 640x480 frame."""
    global _CPU_FRAMES
    from oracle import polyphase as pp
    import synthgen
    _CPU_FRAMES = make_frames(n_frames)
    granted = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    cores = max(1, min(16, granted))
    ctx = mp.get_context("fork")
    with ctx.Pool(cores) as pool:
        pool.map(_cpu_one, range(min(cores, n_frames)))  # warm the workers (imports)
        t0 = time.perf_counter()
        pool.map(_cpu_one, [i % n_frames for i in range(n_frames * repeats)], chunksize=1)
        dt = time.perf_counter() - t0
    _, oy = alg_bytes_per_frame(1, 1)
    done = n_frames * repeats
    # one process
    _cpu_one(0)
    t0 = time.perf_counter()
    for i in range(single_frames):
        _cpu_one(i % n_frames)
    dt1 = time.perf_counter() - t0
    # the interpreter (pure Python loops over repetitions) on the 640x480 frame
    X = synthgen.uniform_frame(2024, 480, 640)
    f = pp.Filter(P, Q, synthgen.design_taps(P, Q, TAPS))
    t0 = time.perf_counter()
    Yi, _, _ = pp.downscale_u8_interp(X, f, f)
    dti = time.perf_counter() - t0
    return dict(value=done * oy[0] * oy[1] / dt / 1e6, unit="Mpixel/s", cores=cores, kind="oracle",
                sample=f"{n_frames} I420 1920x1080 frames of the same workload, each downscaled {repeats} times "
                       f"({done} frames), integer oracle (numpy), {cores} processes, {dt:.1f} s",
                cpu_model=_cpu_model(), os_cpu_count=os.cpu_count(), granted_cpus=granted,
                single_process={"value": single_frames * oy[0] * oy[1] / dt1 / 1e6, "unit": "Mpixel/s",
                                "frames": single_frames, "seconds": round(dt1, 2)},
                interpreter_config1={"seconds": round(dti, 3), "frame": "640x480 -> 180x240",
                                     "out_mpixel_per_s": 180 * 240 / dti / 1e6})


# ------------------------------------------------------------------ main

def main():
    global WARM_SECONDS
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--frames", type=int, default=300)
    ap.add_argument("--cpu-frames", type=int, default=384)
    ap.add_argument("--cpu-repeats", type=int, default=10)
    ap.add_argument("--cpu-single-frames", type=int, default=64)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-float", action="store_true")
    ap.add_argument("--only", choices=["u8", "unfused", "bf16", "fp16", "batch", "generic", "linear", "config1", "cif"], default=None,
                    help="run one workload only (for profiling)")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-generic", action="store_true")
    ap.add_argument("--warm-seconds", type=float, default=WARM_SECONDS,
                    help="extra warm-up time before each timed region (0 under a counter profiler)")
    ap.add_argument("--hash", action="store_true", help="print the fused kernel's source hash and exit")
    ap.add_argument("--copy-calib", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy 3 times (scale for HBM byte counters)")
    args = ap.parse_args()
    WARM_SECONDS = args.warm_seconds
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
    if not args.no_cpu and args.only is None:  # before the GPU is initialised: the pool forks this process
        t = time.time()
        cpu = cpu_baseline(args.cpu_frames, args.cpu_repeats, args.cpu_single_frames)
        log(f"cpu baseline in {time.time() - t:.1f} s: {cpu['value']:.1f} Mpixel/s")

    import torch
    torch.cuda.set_device(0)
    out = {"metric": METRIC}
    extra = {}
    if args.only is None:
        extra["copy_peak_gbs"] = round(copy_peak(), 1)
        log(f"copy: {extra['copy_peak_gbs']} GB/s")
    if args.only in (None, "cif"):
        extra["paper_cif_pipeline"] = bench_cif()
        if args.only:
            print(json.dumps({"metric": METRIC, **extra}), flush=True)
            return
    if args.only in (None, "config1"):
        extra["config1"] = bench_config1()
        log(f"config1: {extra['config1']['us_median']} us")
        if args.only:
            print(json.dumps({"metric": METRIC, **extra}), flush=True)
            return
    t = time.time()
    Yh, Uh, Vh = make_frames(args.frames)
    log(f"generated {args.frames} I420 frames in {time.time() - t:.1f} s")

    u8 = None
    if args.only in (None, "u8", "unfused"):
        u8 = bench_u8(Yh, Uh, Vh, args.steps, args.warmup)
        log(f"u8 fused: {u8['ms_step']:.3f} ms/step, kernel {u8['ms_kernel']:.3f} ms, "
            f"mismatches {u8['mismatches']}")
    if u8 and args.only in (None, "unfused"):
        extra["unfused_u8"] = bench_unfused(u8, Yh, Uh, Vh, args.steps, args.warmup)
        log(f"unfused u8: {extra['unfused_u8']['ms_per_step']:.3f} ms/step, identical "
            f"{extra['unfused_u8']['identical_to_fused']}")
    fl = {}
    if not args.no_float and args.only in (None, "bf16", "fp16"):
        ins_u8 = u8["ins"] if u8 else [torch.from_numpy(a).cuda() for a in (Yh, Uh, Vh)]
        if u8:
            del u8["outs"]
            torch.cuda.empty_cache()
        for fmt in ("bf16", "fp16"):
            if args.only in (None, fmt):
                fl[fmt] = bench_float(ins_u8, args.steps, args.warmup, fmt)
                log(f"{fmt} fused: {fl[fmt]['ms_step']:.3f} ms/step, kernel {fl[fmt]['ms_kernel']:.3f} ms, "
                    f"err {fl[fmt]['max_abs_err']:.2e}")
        del ins_u8
    if u8:
        u8.pop("ins", None)
        u8.pop("outs", None)
        u8["plan"].close()
        torch.cuda.empty_cache()

    if not args.no_batch and args.only in (None, "batch"):
        extra["batch_u8"] = bench_batch("u8")
        log(f"batch u8: {extra['batch_u8']['ms_per_step']:.3f} ms/step, two streams {extra['batch_u8']['two_streams']['ms_per_step']:.3f}")
        extra["batch_u8_1080p_subset"] = bench_batch("u8", only_size=(1080, 1920))
        log(f"batch u8 1080p subset: {extra['batch_u8_1080p_subset']['ms_per_step']:.3f} ms/step, two streams {extra['batch_u8_1080p_subset']['two_streams']['ms_per_step']:.3f}")
        if not args.no_float:
            extra["batch_bf16"] = bench_batch("bf16")
            log(f"batch bf16: {extra['batch_bf16']['ms_per_step']:.3f} ms/step, two streams {extra['batch_bf16']['two_streams']['ms_per_step']:.3f}")
    if not args.no_generic and args.only in (None, "generic"):
        extra["generic"] = bench_generic()
        log(f"generic: {extra['generic']['ms_per_step']:.3f} ms/step")
    if not args.no_generic and args.only in (None, "linear"):
        extra["linear_u8"] = bench_linear()
    if args.only in ("batch", "generic", "linear"):
        print(json.dumps({"metric": METRIC, **extra}), flush=True)
        return

    if u8:
        main_res, dtype = u8, "u8"
    else:
        dtype = next(iter(fl))
        main_res = fl[dtype]
    value = main_res["out_pixels"] / (main_res["ms_step"] / 1e3) / 1e6
    gbs = main_res["bytes"] / (main_res["ms_kernel"] / 1e3) / 1e9
    copy = extra.get("copy_peak_gbs")
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
                     "copy_peak": copy, "frac_of_copy": round(gbs / copy, 4) if copy else None,
                     "kernel": "aol::k_band<u8>" if u8 else f"aol::k_band<{dtype}>",
                     "alg_bytes_per_launch": main_res["bytes"],
                     "kernel_ms_mean": round(main_res["ms_kernel"], 4),
                     "kernel_ms_median": round(main_res["ms_kernel_median"], 4)},
    })
    if u8:
        out["parity"] = {"mismatches": u8["mismatches"], "checked_elements": u8["checked_elements"],
                         "checked_frames": u8["checked_frames"], "against": "integer oracle, every element"}
        out["schedule"] = u8["schedule"]
    for fmt, res in fl.items():
        if res is not main_res:
            out[fmt] = float_entry(res)
    out.update(extra)
    if cpu:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
