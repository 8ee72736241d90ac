"""GPU parity of the fused downscaler against the CPU oracle.

Integer path: bit-exact. Float path: max-abs error against the float64
oracle evaluated on the identical bf16/fp16 inputs, within 1e-3 normalised
pixels (the kernel keeps a hi/lo intermediate and float32 accumulation, so
the observed error is around 1e-6; the bound is the stated tolerance).
"""

import numpy as np
import pytest

import synthgen
from oracle import polyphase as pp

import torch

import paper_1103_4881_amd as aol  # a missing library fails the suite (no skip)

pytestmark = pytest.mark.gpu

FLOAT_TOL = 1e-3


def _filters(p, q, T, kind="design", seed=0, starts=None):
    if kind == "design":
        c = synthgen.design_taps(p, q, T)
    elif kind == "raw":
        # phases whose taps have different sums: a different rounding bias per output phase
        g = synthgen.rng_for(seed, 6)
        c = g.integers(-60, 120, size=(p, T))
    else:
        g = synthgen.rng_for(seed, 5)
        c = g.integers(-300, 400, size=(p, T))
        c[:, 0] += 256 - c.sum(axis=1)
        c = np.clip(c, -2047, 2047)
    return aol.Polyphase(p, q, c, starts), pp.Filter(p, q, c, starts)


FILLS = (0x00, 0xFF)  # output sentinels: an element left unwritten differs between the two runs


def _run_u8(planes_np, hf, vf, tile=None, in_pitch_pad=0, out_pitch_pad=0):
    """planes_np: list of uint8 arrays [F, H, W]. Runs the plan once per sentinel fill of the
    outputs (0x00, then 0xFF), requires both runs to agree on every output element (so every
    element was written) and to leave the row padding alone; returns uint8 [F, MH, MW] per plane."""
    shapes = [a.shape[1:] for a in planes_np]
    out_shapes = [aol.aol_downscale_output_shape(h, w, hf, vf) for (h, w) in shapes]
    ins, ip, op = [], [], []
    for a, (oh, ow) in zip(planes_np, out_shapes):
        F, H, W = a.shape
        buf = torch.full((F, H, W + in_pitch_pad), 77, dtype=torch.uint8, device="cuda")
        buf[:, :, :W] = torch.from_numpy(a).cuda()
        ins.append(buf[:, :, :W])
        ip.append(W + in_pitch_pad)
        op.append(ow + out_pitch_pad)
    plan = aol.DownscalePlan(shapes, hf, vf, "u8", in_pitches=ip, out_pitches=op)
    if tile:
        plan.set_tile(*tile)
    runs = []
    for fill in FILLS:
        outs = [torch.full((a.shape[0], oh, ow + out_pitch_pad), fill, dtype=torch.uint8, device="cuda")
                for a, (oh, ow) in zip(planes_np, out_shapes)]
        plan.run(ins, [o[:, :, :s[1]] for o, s in zip(outs, out_shapes)])
        torch.cuda.synchronize()
        res = []
        for o, (oh, ow) in zip(outs, out_shapes):
            o = o.cpu().numpy()
            if out_pitch_pad:
                assert (o[:, :, ow:] == fill).all(), "write outside the output rows"
            res.append(o[:, :, :ow])
        runs.append(res)
    for a, b in zip(*runs):
        np.testing.assert_array_equal(a, b, err_msg="outputs differ between sentinel fills (unwritten elements)")
    plan.close()
    return runs[0]


def test_config1_vga_frame_bit_exact():
    """One 640x480 uniform random frame, 3/8 with 11 taps on both axes -> 180x240."""
    X = synthgen.uniform_frame(2024, 480, 640)
    hf, of = _filters(3, 8, 11)
    (Y,) = _run_u8([X[None]], hf, hf)
    ref = pp.downscale_u8(X, of, of)
    assert Y.shape == (1, 180, 240)
    np.testing.assert_array_equal(Y[0], ref)


CASES = [
    # (h, w, p, q, T, kind, starts)
    (1, 1, 3, 8, 11, "design", None),
    (3, 5, 3, 8, 11, "random", None),
    (17, 9, 1, 2, 8, "design", None),
    (31, 47, 2, 3, 16, "random", None),
    (45, 130, 4, 9, 7, "random", [-3, 0, 2, 5]),
    (64, 64, 1, 1, 1, "design", None),
    (100, 37, 5, 3, 6, "random", None),
    (129, 257, 3, 8, 16, "random", None),
    (240, 200, 16, 64, 32, "random", None),
    (77, 333, 3, 5, 13, "random", [-9, -4, 0]),
    (540, 960, 3, 8, 11, "design", None),
    (96, 256, 3, 8, 11, "raw", None),
    (70, 150, 2, 3, 9, "raw", None),
]


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}x{c[1]}-{c[2]}_{c[3]}-T{c[4]}-{c[5]}" for c in CASES])
def test_odd_shapes_and_ratios_bit_exact(case):
    h, w, p, q, T, kind, starts = case
    hf, of = _filters(p, q, T, kind, seed=h * 7 + w, starts=starts)
    vf, ov = _filters(p, q, T, kind, seed=h * 3 + w + 1, starts=starts)
    X = synthgen.uniform_frame(h, h, w, idx=w)[None].repeat(2, axis=0)
    X[1] = 255 - X[1]
    (Y,) = _run_u8([X], hf, vf)
    np.testing.assert_array_equal(Y, pp.downscale_u8(X, of, ov))


def test_unaligned_pitches_and_guard_bytes():
    hf, of = _filters(3, 8, 11)
    vf, ov = _filters(1, 2, 8)
    X = synthgen.uniform_frame(5, 70, 150, idx=1)[None]
    (Y,) = _run_u8([X], hf, vf, in_pitch_pad=3, out_pitch_pad=5)
    np.testing.assert_array_equal(Y, pp.downscale_u8(X, of, ov))


@pytest.mark.parametrize("p,q,T", [(16, 24, 9), (16, 32, 16)])
def test_sixteen_blocks_per_period(p, q, T):
    # p = 16 (the largest): 16 block positions per period shared by the horizontal pass's shares
    hf, of = _filters(p, q, T)
    X = synthgen.uniform_frame(17, 100, 240, idx=3)[None]
    (Y,) = _run_u8([X], hf, hf)
    np.testing.assert_array_equal(Y, pp.downscale_u8(X, of, of))


@pytest.mark.parametrize("p,q", [(9, 16), (12, 16), (16, 24)])
def test_many_block_positions_with_int8_taps(p, q):
    """More block positions per period than compute waves (p > 8) with taps that fit int8 and
    one K-step: the loading waves take no share of the horizontal pass and each compute wave
    takes two (the second reading its coefficient operands from LDS)."""
    T = 8
    c = np.full((p, T), 32)  # each phase sums to 256, every tap within int8
    hf, of = aol.Polyphase(p, q, c), pp.Filter(p, q, c)
    plan = aol.DownscalePlan([(140, 416)], hf, hf, "u8")
    sched = plan.schedule(2)
    plan.close()
    assert sched["kernel"] == "band" and sched["split"] == 0 and sched["kmax"] == 1, sched
    X = np.stack([synthgen.uniform_frame(19 + p + f, 140, 416, idx=4) for f in range(2)])
    (Y,) = _run_u8([X], hf, hf)
    np.testing.assert_array_equal(Y, pp.downscale_u8(X, of, of))


def test_two_kstep_filters_many_units_per_workgroup():
    # 3/8 with 16 taps: blocks with one and with two K-steps, column bands, several
    # units per workgroup (a regression: an unused K-step was accumulated)
    hf, of = _filters(3, 8, 16)
    F = 6
    planes = [synthgen.uniform_frame(31 + f, 1080, 1920, idx=0) for f in range(F)]
    X = np.stack(planes)
    (Y,) = _run_u8([X], hf, hf)
    for f in range(F):
        np.testing.assert_array_equal(Y[f], pp.downscale_u8(X[f:f + 1], of, of)[0], err_msg=f"frame {f}")


@pytest.mark.parametrize("w,out_pad", [(512, 0), (512, 4), (512, 8), (400, 4), (464, 0)])
def test_output_pitches_paired_stores(w, out_pad):
    # output rows of 192 / 150 / 174 bytes with pitches that are and are not
    # multiples of 8, odd and even counts of 16-column output blocks
    hf, of = _filters(3, 8, 11)
    vf, ov = _filters(3, 8, 11)
    X = synthgen.uniform_frame(8, 96, w, idx=2)[None]
    (Y,) = _run_u8([X], hf, vf, out_pitch_pad=out_pad)
    np.testing.assert_array_equal(Y, pp.downscale_u8(X, of, ov))


@pytest.mark.parametrize("w,out_pad", [(1280, 0), (1275, 0), (1280, 1), (1280, 2), (1278, 0)])
def test_output_pitches_split_taps(w, out_pad):
    """2/3 with split taps, three frames: output rows of 854 / 850 / 852 bytes with pitches
    6, 2, 0 and 4 modulo 8 and odd ones (dword, half-word and byte stores)."""
    hf, of = _filters(2, 3, 14)
    X = np.stack([synthgen.uniform_frame(40 + f, 96, w, idx=3) for f in range(3)])
    probe = aol.DownscalePlan([(96, w)], hf, hf, "u8")
    sched = probe.schedule(3)
    probe.close()
    assert sched["kernel"] == "band" and sched["split"] == 1, sched
    (Y,) = _run_u8([X], hf, hf, out_pitch_pad=out_pad)
    np.testing.assert_array_equal(Y, pp.downscale_u8(X, of, of))


def test_i420_frames_every_tile_shape_identical():
    """Three planes, several frames, every tile shape: identical bytes (independent elementary tasks)."""
    Yp, Up, Vp = synthgen.yuv420_frames(7, 3, 360, 640)
    hf, of = _filters(3, 8, 11)
    ref = [pp.downscale_u8(a, of, of) for a in (Yp, Up, Vp)]
    # includes tiles whose output count per side (3*8=24, 3*2=6) is not a multiple of the 16-wide blocks
    for tile in [(16, 16), (32, 16), (16, 32), (32, 32), (64, 16), (32, 8), (16, 8), (64, 4), (2, 2), (16, 3)]:
        got = _run_u8([Yp, Up, Vp], hf, hf, tile=tile)
        for g, r in zip(got, ref):
            np.testing.assert_array_equal(g, r)


def test_1080p_i420_six_frames_every_frame():
    """Six I420 1080p frames in one launch (short segments: few frames); every output of
    every frame checked."""
    n = 6
    Yp, Up, Vp = synthgen.yuv420_frames(11, n, 1080, 1920)
    hf, of = _filters(3, 8, 11)
    got = _run_u8([Yp, Up, Vp], hf, hf)
    assert got[0].shape == (n, 405, 720) and got[1].shape == (n, 204, 360)
    for f in range(n):
        for g, a in zip(got, (Yp, Up, Vp)):
            np.testing.assert_array_equal(g[f], pp.downscale_u8(a[f], of, of), err_msg=f"frame {f}")


# The benchmark's workload: 300 I420 1080p frames (seed, filter and plan as in bench.py)
BENCH_SEED, BENCH_FRAMES = 20110322, 300


def test_headline_launch_300_frames():
    """The launch bench.py times: 300 I420 1920x1080 frames, 3/8 with 11 taps on both axes, the
    automatic schedule (segments of up to 64 repetitions: 7 units per frame, 2100 items dealt over
    the workgroups). Runs twice, outputs pre-filled with 0x00 and with 0xFF: the two runs agree on
    all 300 frames (every output written); sampled frames equal the oracle on every element."""
    n = BENCH_FRAMES
    Yp, Up, Vp = synthgen.yuv420_frames(BENCH_SEED, n, 1080, 1920)
    c = synthgen.design_taps(3, 8, 11)
    f = aol.Polyphase(3, 8, c)
    of = pp.Filter(3, 8, c)
    plan = aol.DownscalePlan([(1080, 1920), (540, 960), (540, 960)], f, f, "u8")
    sched = plan.schedule(n)
    assert sched["kernel"] == "band" and sched["seg"] == 64 and sched["units_per_frame"] == 7, sched
    assert sched["items"] == 7 * n and sched["split"] == 0 and sched["kmax"] == 1, sched
    ins = [torch.from_numpy(a).cuda() for a in (Yp, Up, Vp)]
    runs = []
    for fill in FILLS:
        outs = [torch.full((n,) + s, fill, dtype=torch.uint8, device="cuda") for s in plan.out_shapes]
        plan.run(ins, outs)
        torch.cuda.synchronize()
        runs.append(outs)
    for j, (a, b) in enumerate(zip(*runs)):
        assert torch.equal(a, b), f"plane {j}: outputs differ between sentinel fills"
    g = synthgen.rng_for(BENCH_SEED, 77)
    frames = sorted({0, 1, n // 2 - 1, n // 2, n - 2, n - 1, *g.integers(0, n, size=4).tolist()})
    for fr in frames:
        for j, (o, a) in enumerate(zip(runs[0], (Yp, Up, Vp))):
            np.testing.assert_array_equal(o[fr].cpu().numpy(), pp.downscale_u8(a[fr], of, of),
                                          err_msg=f"frame {fr} plane {j}")
    plan.close()


def test_first_run_captured_in_a_graph():
    """A plan's very first run, captured in a graph and replayed: run calls only enqueue (no
    allocation, copy or synchronisation), so the capture holds the whole launch."""
    Yp, Up, Vp = synthgen.yuv420_frames(19, 3, 270, 480)
    hf, of = _filters(3, 8, 11)
    plan = aol.DownscalePlan([a.shape[1:] for a in (Yp, Up, Vp)], hf, hf, "u8")
    ins = [torch.from_numpy(a).cuda() for a in (Yp, Up, Vp)]
    outs = [torch.full((3,) + s, 0xA5, dtype=torch.uint8, device="cuda") for s in plan.out_shapes]
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        plan.run(ins, outs)
    refs = [pp.downscale_u8(a, of, of) for a in (Yp, Up, Vp)]
    for rep, fill in enumerate((0x00, 0xFF, 0x00)):
        for o in outs:
            o.fill_(fill)  # eager work between the replays
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        for j, (o, r) in enumerate(zip(outs, refs)):
            np.testing.assert_array_equal(o.cpu().numpy(), r, err_msg=f"replay {rep} plane {j}")
    del graph
    plan.close()


@pytest.mark.parametrize("fmt", ["u8", "bf16"])
@pytest.mark.parametrize("p,q,tile", [(5, 3, (16, 5)), (2, 3, (16, 7)), (3, 8, (4, 3)), (1, 2, (8, 9))])
def test_tiles_with_partial_output_blocks(fmt, p, q, tile):
    """Tiles whose p*tile outputs leave a partial 16-wide block: no writes into the neighbouring tile."""
    X = synthgen.uniform_frame(p * 10 + q, 150, 170)[None]
    hf, of = _filters(p, q, 9)
    if fmt == "u8":
        (Y,) = _run_u8([X], hf, hf, tile=tile)
        np.testing.assert_array_equal(Y, pp.downscale_u8(X, of, of))
    else:
        (o,), (b,) = _run_f([X], hf, hf, fmt, tile=tile)
        assert np.abs(o - pp.downscale_f64(_decode(b, fmt), of, of)).max() <= FLOAT_TOL


def test_constant_frames_map_to_themselves():
    for (p, q, T) in [(3, 8, 11), (2, 3, 16), (1, 2, 8)]:
        hf, _ = _filters(p, q, T, "random", seed=T)
        X = np.broadcast_to(np.arange(256, dtype=np.uint8)[:, None, None], (256, 24, 40)).copy()
        (Y,) = _run_u8([X], hf, hf)
        assert (Y == np.arange(256, dtype=np.uint8)[:, None, None]).all()


# ------------------------------------------------------------------ float path

def _run_f(planes_u8, hf, vf, fmt, tile=None):
    shapes = [a.shape[1:] for a in planes_u8]
    plan = aol.DownscalePlan(shapes, hf, vf, fmt)
    if tile:
        plan.set_tile(*tile)
    ins, outs, bits = [], [], []
    for a, (oh, ow) in zip(planes_u8, plan.out_shapes):
        b = synthgen.normalised(a, fmt)
        bits.append(b)
        ins.append(torch.from_numpy(b.view(np.int16)).cuda())
        outs.append(torch.full((a.shape[0], oh, ow), float("nan"), dtype=torch.float32, device="cuda"))
    plan.run(ins, outs)
    torch.cuda.synchronize()
    plan.close()
    return [o.cpu().numpy() for o in outs], bits


def _decode(bits, fmt):
    if fmt == "bf16":
        return (bits.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    return bits.view(np.float16).astype(np.float64)


@pytest.mark.parametrize("fmt", ["bf16", "fp16"])
def test_float_path_within_tolerance(fmt):
    Yp, Up, Vp = synthgen.yuv420_frames(3, 2, 270, 480)
    hf, of = _filters(3, 8, 11)
    outs, bits = _run_f([Yp, Up, Vp], hf, hf, fmt)
    for o, b in zip(outs, bits):
        ref = pp.downscale_f64(_decode(b, fmt), of, of)
        assert np.isfinite(o).all()
        err = np.abs(o - ref).max()
        print(f"{fmt} plane {o.shape}: max-abs error {err:.3e}")
        assert err <= FLOAT_TOL


@pytest.mark.parametrize("fmt", ["bf16", "fp16"])
@pytest.mark.parametrize("case", [(33, 71, 2, 3, 16), (19, 5, 1, 2, 8), (130, 300, 3, 8, 11), (40, 75, 2, 3, 14)])
def test_float_path_odd_shapes(fmt, case):
    h, w, p, q, T = case
    hf, of = _filters(p, q, T)
    X = synthgen.uniform_frame(h, h, w)[None]
    (o,), (b,) = _run_f([X], hf, hf, fmt)
    ref = pp.downscale_f64(_decode(b, fmt), of, of)
    assert np.abs(o - ref).max() <= FLOAT_TOL


@pytest.mark.parametrize("band,seg", [(0, 0), (16, 16), (64, 16), (128, 64), (32, 32)])
def test_band_schedules_bit_exact(band, seg):
    """Band kernel: column bands with halo chunks, several segment lengths, I420 frames."""
    Yp, Up, Vp = synthgen.yuv420_frames(13, 2, 270, 700)
    hf, of = _filters(3, 8, 11)
    vf, ov = _filters(2, 3, 14)
    shapes = [a.shape[1:] for a in (Yp, Up, Vp)]
    plan = aol.DownscalePlan(shapes, hf, vf, "u8")
    plan.set_band(band, seg)
    ins = [torch.from_numpy(a).cuda() for a in (Yp, Up, Vp)]
    for fill in FILLS:
        outs = [torch.full((2,) + s, fill, dtype=torch.uint8, device="cuda") for s in plan.out_shapes]
        plan.run(ins, outs)
        torch.cuda.synchronize()
        for o, a in zip(outs, (Yp, Up, Vp)):
            np.testing.assert_array_equal(o.cpu().numpy(), pp.downscale_u8(a, of, ov), err_msg=f"fill {fill}")
    plan.close()


@pytest.mark.parametrize("fmt,band,seg", [("bf16", 0, 0), ("bf16", 32, 16), ("fp16", 16, 48)])
def test_band_schedules_float(fmt, band, seg):
    Yp, _, _ = synthgen.yuv420_frames(17, 2, 200, 520)
    hf, of = _filters(3, 8, 11)
    plan = aol.DownscalePlan([Yp.shape[1:]], hf, hf, fmt)
    plan.set_band(band, seg)
    b = synthgen.normalised(Yp, fmt)
    ins = [torch.from_numpy(b.view(np.int16)).cuda()]
    outs = [torch.full((2,) + plan.out_shapes[0], float("nan"), dtype=torch.float32, device="cuda")]
    plan.run(ins, outs)
    torch.cuda.synchronize()
    ref = pp.downscale_f64(_decode(b, fmt), of, of)
    got = outs[0].cpu().numpy()
    assert np.isfinite(got).all()
    assert np.abs(got - ref).max() <= FLOAT_TOL
    plan.close()
