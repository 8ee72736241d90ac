"""GPU tests of the host-to-host frame pipeline (frames in host memory, copies overlapped with
the fused kernel) on the paper's CIF workload: 352x288 I420 frames, 3/8 along lines and 4/9 along
columns (352x288 -> 132x128). Outputs are bit-exact against the oracle and identical to the
device-resident launch; outputs are pre-filled with 0x00 and 0xFF (every element written)."""

import numpy as np
import pytest

import synthgen
from oracle import polyphase as pp

import torch

import paper_1103_4881_amd as aol  # a missing library fails the suite (no skip)

pytestmark = pytest.mark.gpu

CIF = (288, 352)


def _cif_plan():
    ch = synthgen.design_taps(3, 8, 11)
    cv = synthgen.design_taps(4, 9, 11)
    hf, vf = aol.Polyphase(3, 8, ch), aol.Polyphase(4, 9, cv)
    plan = aol.DownscalePlan([CIF, (144, 176), (144, 176)], hf, vf, "u8")
    return plan, pp.Filter(3, 8, ch), pp.Filter(4, 9, cv)


@pytest.mark.parametrize("batch,depth,pinned", [(1, 1, True), (1, 4, True), (7, 3, True), (16, 2, False)])
def test_cif_pipeline_bit_exact(batch, depth, pinned):
    n = 40
    planes = synthgen.yuv420_frames(1103, n, *CIF)
    plan, oh, ov = _cif_plan()
    assert plan.out_shapes[0] == (128, 132) and plan.out_shapes[1] == (64, 66)
    pipe = aol.Pipeline(plan, batch, depth)
    ins = [torch.from_numpy(a).pin_memory() if pinned else torch.from_numpy(a) for a in planes]
    refs = [pp.downscale_u8(a, oh, ov) for a in planes]
    for fill in (0x00, 0xFF):
        outs = [torch.full((n,) + s, fill, dtype=torch.uint8, pin_memory=pinned) for s in plan.out_shapes]
        st = pipe.run(ins, outs)
        for j, (o, r) in enumerate(zip(outs, refs)):
            np.testing.assert_array_equal(o.numpy(), r, err_msg=f"plane {j} fill {fill}")
        assert st["frames"] == n and st["groups"] == -(-n // batch)
        assert st["h2d_bytes"] == n * (288 * 352 + 2 * 144 * 176)
        assert st["d2h_bytes"] == n * (128 * 132 + 2 * 64 * 66)
        assert st["h2d_ms"] > 0 and st["kernel_ms"] > 0 and st["d2h_ms"] > 0 and st["span_ms"] > 0
    pipe.close()
    plan.close()


def test_pipeline_equals_device_launch_and_reuses_slots():
    """More groups than slots (each slot reused many times), and a second run on the same
    pipeline: the outputs equal one device-resident launch over the same frames."""
    n = 61
    planes = synthgen.yuv420_frames(7, n, *CIF)
    plan, _, _ = _cif_plan()
    dev_in = [torch.from_numpy(a).cuda() for a in planes]
    dev_out = [torch.empty((n,) + s, dtype=torch.uint8, device="cuda") for s in plan.out_shapes]
    plan.run(dev_in, dev_out)
    torch.cuda.synchronize()
    pipe = aol.Pipeline(plan, 4, 3)
    ins = [torch.from_numpy(a).pin_memory() for a in planes]
    for rep in range(2):
        outs = [torch.full((n,) + s, 0xA5 ^ rep, dtype=torch.uint8, pin_memory=True) for s in plan.out_shapes]
        st = pipe.run(ins, outs)
        assert st["groups"] == 16
        for j, (o, d) in enumerate(zip(outs, dev_out)):
            np.testing.assert_array_equal(o.numpy(), d.cpu().numpy(), err_msg=f"run {rep} plane {j}")
    pipe.close()
    plan.close()


def test_pipeline_errors():
    plan, _, _ = _cif_plan()
    for batch, depth in [(0, 2), (1, 0), (1, 65)]:
        with pytest.raises(aol.AolError) as e:
            aol.Pipeline(plan, batch, depth)
        assert e.value.status == aol.AOL_ERR_INVALID
    pipe = aol.Pipeline(plan, 2, 2)
    ins = [torch.zeros((3,) + s, dtype=torch.uint8) for s in plan.shapes]
    outs = [torch.zeros((3,) + s, dtype=torch.uint8) for s in plan.out_shapes]
    with pytest.raises(aol.AolError) as e:  # frame strides smaller than a frame
        aol.aol_pipeline_run_u8(pipe._h, 3, [t.data_ptr() for t in ins], [1, 1, 1], [o.data_ptr() for o in outs],
                                [o.stride(0) for o in outs])
    assert e.value.status == aol.AOL_ERR_INVALID
    st = pipe.run([t[:0] for t in ins], [o[:0] for o in outs])  # no frames: nothing to do
    assert st["groups"] == 0 and st["frames"] == 0
    pipe.close()
    plan.close()
    c = synthgen.design_taps(3, 8, 11)
    fplan = aol.DownscalePlan([CIF], aol.Polyphase(3, 8, c), aol.Polyphase(3, 8, c), "bf16")
    with pytest.raises(ValueError):
        aol.Pipeline(fplan, 1, 2)
    with pytest.raises(aol.AolError) as e:
        aol.aol_pipeline_create(fplan._h, 1, 2)
    assert e.value.status == aol.AOL_ERR_INVALID
    fplan.close()
