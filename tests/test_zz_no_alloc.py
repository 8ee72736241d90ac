"""GPU test of the allocation-free entry point (aol_downscale_u8_unfused_static): the unfused
downscale with its intermediate in the library's static 64 MiB device workspace, called through
the C ABI and compared with the workspace entry point (aol_downscale_u8_unfused) on two calls in a
row, the second with a smaller input; sampled frames also against the oracle."""

import numpy as np
import pytest

import synthgen
from oracle import polyphase as pp

import torch

import paper_1103_4881_amd as aol  # a missing library fails the suite (no skip)

pytestmark = pytest.mark.gpu

STATIC_BYTES = 64 << 20


def _call(plan, ins, outs, static):
    if static:
        aol.aol_downscale_u8_unfused_static(plan._h, ins[0].shape[0], [t.data_ptr() for t in ins],
                                            [t.stride(0) for t in ins], [o.data_ptr() for o in outs],
                                            [o.stride(0) for o in outs])
    else:
        work = torch.empty(plan.workspace_bytes() * ins[0].shape[0], dtype=torch.uint8, device="cuda")
        aol.aol_downscale_u8_unfused(plan._h, ins[0].shape[0], [t.data_ptr() for t in ins],
                                     [t.stride(0) for t in ins], [o.data_ptr() for o in outs],
                                     [o.stride(0) for o in outs], work.data_ptr(), work.numel())
        torch.cuda.synchronize()
        del work
    torch.cuda.synchronize()


def _check(planes, hf, vf, of, ov, sample):
    shapes = [a.shape[1:] for a in planes]
    plan = aol.DownscalePlan(shapes, hf, vf, "u8")
    n = planes[0].shape[0]
    ins = [torch.from_numpy(a).cuda() for a in planes]
    ref_out = [torch.full((n,) + s, 0x00, dtype=torch.uint8, device="cuda") for s in plan.out_shapes]
    st_out = [torch.full((n,) + s, 0xFF, dtype=torch.uint8, device="cuda") for s in plan.out_shapes]
    _call(plan, ins, ref_out, static=False)
    _call(plan, ins, st_out, static=True)
    for j, (a, b) in enumerate(zip(ref_out, st_out)):
        assert torch.equal(a, b), f"plane {j}: static-workspace outputs differ from the workspace entry point's"
    for fr in sample:
        for j, (o, a) in enumerate(zip(st_out, planes)):
            np.testing.assert_array_equal(o[fr].cpu().numpy(), pp.downscale_u8(a[fr], of, ov),
                                          err_msg=f"frame {fr} plane {j}")
    per = plan.workspace_bytes()
    plan.close()
    return per


def test_static_workspace_two_calls_second_smaller():
    c = synthgen.design_taps(3, 8, 11)
    f, of = aol.Polyphase(3, 8, c), pp.Filter(3, 8, c)
    # call 1: 60 I420 1080p frames, more than the static workspace holds at once (groups of 52 + 8)
    planes = synthgen.yuv420_frames(601, 60, 1080, 1920)
    per = _check(planes, f, f, of, of, sample=(0, 51, 52, 59))
    assert STATIC_BYTES // per == 52
    # call 2: a smaller input (one 480x640 plane, 3 frames, 4/9 vertically) over the same
    # workspace, which still holds the first call's intermediates
    cv = synthgen.design_taps(4, 9, 11)
    X = np.stack([synthgen.uniform_frame(602 + k, 480, 640) for k in range(3)])
    _check([X], f, aol.Polyphase(4, 9, cv), of, pp.Filter(4, 9, cv), sample=(0, 1, 2))


def test_static_workspace_frame_too_large():
    """One frame whose intermediate exceeds the 64 MiB static workspace is refused (no launch)."""
    c = synthgen.design_taps(3, 8, 11)
    f = aol.Polyphase(3, 8, c)
    plan = aol.DownscalePlan([(16384, 16384)], f, f, "u8")
    assert plan.workspace_bytes() > STATIC_BYTES
    x = torch.zeros(16, dtype=torch.uint8, device="cuda")  # never read: the call fails before any launch
    with pytest.raises(aol.AolError) as e:
        aol.aol_downscale_u8_unfused_static(plan._h, 1, [x.data_ptr()], [0], [x.data_ptr()], [0])
    assert e.value.status == aol.AOL_ERR_UNSUPPORTED
    plan.close()
