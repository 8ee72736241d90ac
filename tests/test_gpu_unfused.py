"""GPU parity of the unfused downscaler (two row passes, intermediate through device memory).

Integer path only: bit-exact against the oracle on every element, and identical to the fused
kernel. Outputs are pre-filled with 0x00 and then 0xFF: both runs must agree (every element
written) and row padding must be left alone. Frames run in groups that fit the workspace; the
tests give workspaces of one, two and all frames.
"""

import numpy as np
import pytest

import synthgen
from oracle import polyphase as pp

import torch

import paper_1103_4881_amd as aol  # a missing library fails the suite (no skip)

pytestmark = pytest.mark.gpu

FILLS = (0x00, 0xFF)


def _filters(p, q, T, kind="design", seed=0, starts=None):
    if kind == "design":
        c = synthgen.design_taps(p, q, T)
    else:  # taps beyond int8 (split operands) with phases of different sums
        g = synthgen.rng_for(seed, 5)
        c = g.integers(-300, 400, size=(p, T))
        c[:, 0] += 256 - c.sum(axis=1)
        c = np.clip(c, -2047, 2047)
    return aol.Polyphase(p, q, c, starts), pp.Filter(p, q, c, starts)


def _workspace(plan, frames):
    per = plan.workspace_bytes()
    return torch.empty(per * frames, dtype=torch.uint8, device="cuda"), per


def _run(planes_np, hf, vf, ws_frames=None, in_pitch_pad=0, out_pitch_pad=0, fused_too=True):
    """Runs the unfused form once per sentinel fill; returns the outputs (uint8 [F, MH, MW] per
    plane) after checking that both fills agree, padding is untouched and (fused_too) the fused
    kernel gives the same bytes."""
    shapes = [a.shape[1:] for a in planes_np]
    out_shapes = [aol.aol_downscale_output_shape(h, w, hf, vf) for (h, w) in shapes]
    F = planes_np[0].shape[0]
    ins, ip, op = [], [], []
    for a, (oh, ow) in zip(planes_np, out_shapes):
        _, H, W = a.shape
        buf = torch.full((F, H, W + in_pitch_pad), 77, dtype=torch.uint8, device="cuda")
        buf[:, :, :W] = torch.from_numpy(a).cuda()
        ins.append(buf[:, :, :W])
        ip.append(W + in_pitch_pad)
        op.append(ow + out_pitch_pad)
    plan = aol.DownscalePlan(shapes, hf, vf, "u8", in_pitches=ip, out_pitches=op)
    work, per = _workspace(plan, ws_frames or F)
    runs = []
    for fill in FILLS:
        outs = [torch.full((F, oh, ow + out_pitch_pad), fill, dtype=torch.uint8, device="cuda")
                for (oh, ow) in out_shapes]
        work.fill_(fill)  # stale workspace contents must not matter
        plan.run_unfused(ins, [o[:, :, :s[1]] for o, s in zip(outs, out_shapes)], work)
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
    if fused_too:
        outs = [torch.full((F, oh, ow + out_pitch_pad), 0x5A, dtype=torch.uint8, device="cuda")
                for (oh, ow) in out_shapes]
        plan.run(ins, [o[:, :, :s[1]] for o, s in zip(outs, out_shapes)])
        torch.cuda.synchronize()
        for j, (o, u, (oh, ow)) in enumerate(zip(outs, runs[0], out_shapes)):
            np.testing.assert_array_equal(o.cpu().numpy()[:, :, :ow], u, err_msg=f"plane {j}: fused != unfused")
    plan.close()
    return runs[0]


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
    (480, 640, 3, 8, 11, "design", None),
    (540, 960, 3, 8, 11, "design", None),
    (288, 352, 3, 8, 11, "design", None),
    (300, 700, 2, 3, 16, "random", None),
]


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}x{c[1]}-{c[2]}_{c[3]}-T{c[4]}-{c[5]}" for c in CASES])
def test_shapes_and_ratios_bit_exact(case):
    h, w, p, q, T, kind, starts = case
    hf, of = _filters(p, q, T, kind, seed=h * 7 + w, starts=starts)
    vf, ov = _filters(p, q, T, kind, seed=h * 3 + w + 1, starts=starts)
    X = synthgen.uniform_frame(h, h, w, idx=w)[None].repeat(3, axis=0)
    X[1] = 255 - X[1]
    X[2] = X[2] // 3
    (Y,) = _run([X], hf, vf, ws_frames=2)  # two groups of frames: 2 + 1
    np.testing.assert_array_equal(Y, pp.downscale_u8(X, of, ov))


def test_paper_cif_ratios():
    """The paper's CIF frames: 352x288 with 3/8 along lines and 4/9 along columns -> 132x128."""
    hf, of = _filters(3, 8, 11)
    vf, ov = _filters(4, 9, 11)
    Yp, Up, Vp = synthgen.yuv420_frames(5, 4, 288, 352)
    got = _run([Yp, Up, Vp], hf, vf, ws_frames=1)
    assert got[0].shape == (4, 128, 132)
    for g, a in zip(got, (Yp, Up, Vp)):
        np.testing.assert_array_equal(g, pp.downscale_u8(a, of, ov))


def test_unaligned_pitches_and_guard_bytes():
    """Input pitch not a multiple of 16 (byte-wise gathers), output pitch not a multiple of 4."""
    hf, of = _filters(3, 8, 11)
    vf, ov = _filters(1, 2, 8)
    X = synthgen.uniform_frame(5, 70, 150, idx=1)[None].repeat(2, axis=0)
    X[1] = 255 - X[1]
    (Y,) = _run([X], hf, vf, in_pitch_pad=3, out_pitch_pad=5)
    np.testing.assert_array_equal(Y, pp.downscale_u8(X, of, ov))


def test_constant_frames_map_to_themselves():
    for (p, q, T) in [(3, 8, 11), (2, 3, 16), (1, 2, 8)]:
        hf, _ = _filters(p, q, T, "random", seed=T)
        X = np.broadcast_to(np.arange(256, dtype=np.uint8)[:, None, None], (256, 24, 40)).copy()
        (Y,) = _run([X], hf, hf, ws_frames=100, fused_too=False)
        assert (Y == np.arange(256, dtype=np.uint8)[:, None, None]).all()


def test_1080p_i420_workload_groups_of_frames():
    """The benchmark's workload (300 I420 1920x1080 frames, 3/8, 11 taps) in groups of 52
    frames (a 64 MiB workspace): all frames equal the fused kernel's; sampled frames (first and
    last of several groups) equal the oracle on every element."""
    n = 300
    Yp, Up, Vp = synthgen.yuv420_frames(20110322, n, 1080, 1920)
    c = synthgen.design_taps(3, 8, 11)
    f = aol.Polyphase(3, 8, c)
    of = pp.Filter(3, 8, c)
    plan = aol.DownscalePlan([(1080, 1920), (540, 960), (540, 960)], f, f, "u8")
    per = plan.workspace_bytes()
    group = (64 << 20) // per
    assert group == 52, per
    work = torch.empty(64 << 20, dtype=torch.uint8, device="cuda")
    ins = [torch.from_numpy(a).cuda() for a in (Yp, Up, Vp)]
    fused = [torch.full((n,) + s, 0x00, dtype=torch.uint8, device="cuda") for s in plan.out_shapes]
    unf = [torch.full((n,) + s, 0xFF, dtype=torch.uint8, device="cuda") for s in plan.out_shapes]
    plan.run(ins, fused)
    plan.run_unfused(ins, unf, work)
    torch.cuda.synchronize()
    for j, (a, b) in enumerate(zip(fused, unf)):
        assert torch.equal(a, b), f"plane {j}: fused and unfused outputs differ"
    for fr in (0, group - 1, group, 2 * group + 7, n - 1):
        for j, (o, a) in enumerate(zip(unf, (Yp, Up, Vp))):
            np.testing.assert_array_equal(o[fr].cpu().numpy(), pp.downscale_u8(a[fr], of, of),
                                          err_msg=f"frame {fr} plane {j}")
    plan.close()


def test_errors():
    hf, _ = _filters(3, 8, 11)
    plan = aol.DownscalePlan([(64, 64)], hf, hf, "u8")
    x = torch.zeros((2, 64, 64), dtype=torch.uint8, device="cuda")
    y = torch.zeros((2,) + plan.out_shapes[0], dtype=torch.uint8, device="cuda")
    per = plan.workspace_bytes()
    assert per == 24 * 128  # 24 transposed rows of 64 lines padded to 128 bytes
    small = torch.empty(per - 1, dtype=torch.uint8, device="cuda")
    with pytest.raises(aol.AolError) as e:
        plan.run_unfused([x], [y], small)
    assert e.value.status == aol.AOL_ERR_INVALID
    big = torch.empty(per * 2 + 256, dtype=torch.uint8, device="cuda")
    with pytest.raises(aol.AolError) as e:
        plan.run_unfused([x], [y], big[1:])  # not 256-byte aligned
    assert e.value.status == aol.AOL_ERR_INVALID
    with pytest.raises(aol.AolError) as e:
        aol.aol_downscale_u8_unfused(plan._h, 2, [x.data_ptr()], [x.stride(0)], [y.data_ptr()], [y.stride(0)], 0,
                                     per * 2)
    assert e.value.status == aol.AOL_ERR_INVALID
    plan.close()
    fplan = aol.DownscalePlan([(64, 64)], hf, hf, "bf16")
    with pytest.raises(aol.AolError) as e:
        fplan.workspace_bytes()
    assert e.value.status == aol.AOL_ERR_INVALID
    fplan.close()
