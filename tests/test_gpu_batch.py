"""GPU parity of the batched downscaler (many streams, one launch per step,
optionally a captured graph) against the CPU oracle: integer bit-exact,
float within 1e-3 normalised pixels of the float64 oracle."""

import json

import numpy as np
import pytest

import synthgen
from oracle import polyphase as pp

import torch

import paper_1103_4881_amd as aol  # a missing library fails the suite (no skip)

pytestmark = pytest.mark.gpu
FILLS = (0x00, 0xFF)  # output sentinels: an element left unwritten differs between the two runs

MIX = [  # (h, w, p, q, taps, kind)
    (96, 200, 3, 8, 11, "design"),
    (61, 130, 1, 2, 8, "design"),
    (120, 97, 2, 3, 16, "design"),
    (33, 64, 2, 3, 13, "random"),  # taps beyond int8: split operands, run as a second launch
    (250, 330, 3, 8, 16, "design"),
    (17, 19, 1, 2, 9, "random"),
]


def _filt(p, q, T, kind, seed):
    if kind == "design":
        c = synthgen.design_taps(p, q, T)
    else:
        g = synthgen.rng_for(seed, 5)
        c = g.integers(-300, 400, size=(p, T))
        c[:, 0] += 256 - c.sum(axis=1)
    return aol.Polyphase(p, q, c), pp.Filter(p, q, c)


def _streams(mix, seed=0):
    out = []
    for i, (h, w, p, q, T, kind) in enumerate(mix):
        hf, of = _filt(p, q, T, kind, seed + i)
        vf, ov = _filt(p, q, T, kind, seed + 100 + i)
        out.append((h, w, hf, vf, of, ov))
    return out


def _frames(mix, n, seed):
    return [[synthgen.uniform_frame(seed + f, h, w, idx=i) for f in range(n)] for i, (h, w, *_) in enumerate(mix)]


@pytest.mark.parametrize("fill", FILLS)
def test_batch_u8_run_and_graph_bit_exact(fill):
    st = _streams(MIX)
    plan = aol.BatchPlan([(h, w, hf, vf) for (h, w, hf, vf, _, _) in st], "u8")
    steps = 3
    frames = _frames(MIX, steps, 7)
    ins = [[torch.from_numpy(fr).cuda() for fr in fs] for fs in frames]
    outs = [[torch.full(plan.out_shapes[i], fill, dtype=torch.uint8, device="cuda") for _ in range(steps)]
            for i in range(len(st))]
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        # step 0 as a plain launch, steps 1.. through one captured graph
        plan.set_pointers([ins[i][0] for i in range(len(st))], [outs[i][0] for i in range(len(st))], s)
        plan.run(s)
        g = plan.graph(s)
        # pointer arrays built once, as a serving loop keeps them; step 2 uses them twice
        tables = [plan.pointer_arrays([ins[i][k] for i in range(len(st))], [outs[i][k] for i in range(len(st))])
                  for k in range(steps)]
        for k in list(range(1, steps)) + [steps - 1]:
            plan.set_pointer_arrays(tables[k], s)
            aol.aol_graph_launch(g, s)
    s.synchronize()
    for i, (h, w, hf, vf, of, ov) in enumerate(st):
        for k in range(steps):
            np.testing.assert_array_equal(outs[i][k].cpu().numpy(), pp.downscale_u8(frames[i][k], of, ov),
                                          err_msg=f"stream {i} step {k}")
    plan.close()


@pytest.mark.parametrize("fill", FILLS)
def test_batch_graphs_with_pointers_per_frame_slot(fill):
    """One graph per frame slot, each with its own pointer table: replayed in turn
    and out of order, with eager work between replays; every output against the oracle."""
    st = _streams(MIX, seed=5)
    plan = aol.BatchPlan([(h, w, hf, vf) for (h, w, hf, vf, _, _) in st], "u8")
    slots = 3
    frames = _frames(MIX, slots, 13)
    ins = [[torch.from_numpy(fr).cuda() for fr in fs] for fs in frames]
    outs = [[torch.full(plan.out_shapes[i], fill, dtype=torch.uint8, device="cuda") for _ in range(slots)]
            for i in range(len(st))]
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        graphs = [plan.graph_with_pointers(plan.pointer_arrays([ins[i][k] for i in range(len(st))],
                                                               [outs[i][k] for i in range(len(st))]), s)
                  for k in range(slots)]
        for rep, k in enumerate([0, 1, 2, 1, 0, 2]):
            for i in range(len(st)):
                outs[i][k].fill_(fill)  # eager work between the replays; the replay rewrites the slot
            aol.aol_graph_launch(graphs[k], s)
            s.synchronize()
            for i, (h, w, hf, vf, of, ov) in enumerate(st):
                np.testing.assert_array_equal(outs[i][k].cpu().numpy(), pp.downscale_u8(frames[i][k], of, ov),
                                              err_msg=f"replay {rep} slot {k} stream {i}")
    plan.close()


@pytest.mark.parametrize("fill", FILLS)
def test_batch_buffer_sets_per_frame_slot(fill):
    """One buffer set per frame slot, run in turn and out of order, across a schedule change,
    with the plan's own table pointed elsewhere: every output against the oracle; a set is
    refused by another plan."""
    st = _streams(MIX, seed=6)
    plan = aol.BatchPlan([(h, w, hf, vf) for (h, w, hf, vf, _, _) in st], "u8")
    slots = 3
    frames = _frames(MIX, slots + 1, 17)
    ins = [[torch.from_numpy(fr).cuda() for fr in fs] for fs in frames]
    outs = [[torch.full(plan.out_shapes[i], fill, dtype=torch.uint8, device="cuda") for _ in range(slots + 1)]
            for i in range(len(st))]
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        sets = [plan.buffers(plan.pointer_arrays([ins[i][k] for i in range(len(st))],
                                                 [outs[i][k] for i in range(len(st))])) for k in range(slots)]
        # the plan's own table: the spare slot, which no buffer-set run may touch
        plan.set_pointers([ins[i][slots] for i in range(len(st))], [outs[i][slots] for i in range(len(st))], s)
        for rep, k in enumerate([0, 1, 2, 1, 0, 2]):
            if rep == 3:
                plan.set_schedule(32, 150 * 1024)
            for i in range(len(st)):
                outs[i][k].fill_(fill)
            plan.run_buffers(sets[k], s)
            s.synchronize()
            for i, (h, w, hf, vf, of, ov) in enumerate(st):
                np.testing.assert_array_equal(outs[i][k].cpu().numpy(), pp.downscale_u8(frames[i][k], of, ov),
                                              err_msg=f"run {rep} slot {k} stream {i}")
        for i in range(len(st)):
            assert bool((outs[i][slots] == fill).all()), f"stream {i}: the plan's own buffers were written"
        other = aol.BatchPlan([(h, w, hf, vf) for (h, w, hf, vf, _, _) in st], "u8")
        with pytest.raises(aol.AolError) as ei:
            other.run_buffers(sets[0], s)
        assert ei.value.status == aol.AOL_ERR_INVALID
        other.close()
    plan.close()


@pytest.mark.parametrize("fill", FILLS)
def test_batch_buffer_sets_on_two_streams(fill):
    """Buffer sets run on two streams in turn with no wait between them (the sets write
    different frame slots), and a schedule change issued while those launches may still
    run: every slot against the oracle, before and after the change."""
    st = _streams(MIX, seed=8)
    plan = aol.BatchPlan([(h, w, hf, vf) for (h, w, hf, vf, _, _) in st], "u8")
    slots = 4
    first = _frames(MIX, slots, 23)
    second = _frames(MIX, slots, 41)
    ins = [[torch.from_numpy(fr).cuda() for fr in fs] for fs in first]
    outs = [[torch.full(plan.out_shapes[i], fill, dtype=torch.uint8, device="cuda") for _ in range(slots)]
            for i in range(len(st))]
    sets = [plan.buffers(plan.pointer_arrays([ins[i][k] for i in range(len(st))],
                                             [outs[i][k] for i in range(len(st))])) for k in range(slots)]
    pair = (torch.cuda.Stream(), torch.cuda.Stream())
    torch.cuda.synchronize()
    for k in range(slots):
        plan.run_buffers(sets[k], pair[k & 1])
    plan.set_schedule(32, 76 * 1024)  # waits for the launches above before rewriting tables
    torch.cuda.synchronize()
    for i, (h, w, hf, vf, of, ov) in enumerate(st):
        for k in range(slots):
            np.testing.assert_array_equal(outs[i][k].cpu().numpy(), pp.downscale_u8(first[i][k], of, ov),
                                          err_msg=f"first pass slot {k} stream {i}")
    for i in range(len(st)):
        for k in range(slots):
            ins[i][k].copy_(torch.from_numpy(second[i][k]))
            outs[i][k].fill_(fill)
    torch.cuda.synchronize()
    for r in range(2 * slots):  # a slot returns to the same stream, so its two runs stay ordered
        plan.run_buffers(sets[r % slots], pair[r & 1])
    torch.cuda.synchronize()
    for i, (h, w, hf, vf, of, ov) in enumerate(st):
        for k in range(slots):
            np.testing.assert_array_equal(outs[i][k].cpu().numpy(), pp.downscale_u8(second[i][k], of, ov),
                                          err_msg=f"second pass slot {k} stream {i}")
    plan.close()


@pytest.mark.parametrize("fill", FILLS)
def test_batch_autotune_keeps_results(tmp_path, fill):
    st = _streams(MIX[:4], seed=3)
    cache = str(tmp_path / "tune.txt")
    plan = aol.BatchPlan([(h, w, hf, vf) for (h, w, hf, vf, _, _) in st], "u8", tune_cache=cache)
    frames = _frames(MIX[:4], 1, 11)
    ins = [torch.from_numpy(fs[0]).cuda() for fs in frames]
    outs = [torch.full(plan.out_shapes[i], fill, dtype=torch.uint8, device="cuda") for i in range(len(st))]
    plan.set_pointers(ins, outs)
    plan.autotune()
    sched = plan.schedule()
    plan.run()
    torch.cuda.synchronize()
    for i, (h, w, hf, vf, of, ov) in enumerate(st):
        np.testing.assert_array_equal(outs[i].cpu().numpy(), pp.downscale_u8(frames[i][0], of, ov))
    plan.close()
    # a new plan over the same batch picks the tuned schedule from the cache
    plan2 = aol.BatchPlan([(h, w, hf, vf) for (h, w, hf, vf, _, _) in st], "u8", tune_cache=cache)
    assert plan2.schedule() == sched
    plan2.close()


@pytest.mark.parametrize("fmt", ["bf16", "fp16"])
def test_batch_float_within_tolerance(fmt):
    mix = [m for m in MIX if m[5] == "design"]
    st = _streams(mix)
    plan = aol.BatchPlan([(h, w, hf, vf) for (h, w, hf, vf, _, _) in st], fmt)
    frames = _frames(mix, 1, 5)
    bits = [synthgen.normalised(fs[0], fmt) for fs in frames]
    ins = [torch.from_numpy(b.view(np.int16)).cuda() for b in bits]
    outs = [torch.full(plan.out_shapes[i], float("nan"), dtype=torch.float32, device="cuda") for i in range(len(st))]
    plan.set_pointers(ins, outs)
    plan.run()
    torch.cuda.synchronize()
    for i, (h, w, hf, vf, of, ov) in enumerate(st):
        x = ((bits[i].astype(np.uint32) << 16).view(np.float32).astype(np.float64) if fmt == "bf16"
             else bits[i].view(np.float16).astype(np.float64))
        ref = pp.downscale_f64(x, of, ov)
        got = outs[i].cpu().numpy()
        assert np.isfinite(got).all()
        assert np.abs(got - ref).max() <= 1e-3, (i, float(np.abs(got - ref).max()))
    plan.close()


@pytest.mark.parametrize("fill", FILLS)
def test_batch_64_streams_mix_one_step(fill):
    """The 64-stream mix (sizes 640x480..3840x2160, ratios 3/8, 1/2, 2/3, 8..16 taps): one step, all outputs."""
    mix = synthgen.stream_mix(2011, 64)
    filt = {}
    streams = []
    for s in mix:
        key = (s.p, s.q, s.taps)
        if key not in filt:
            c = synthgen.design_taps(s.p, s.q, s.taps)
            filt[key] = (aol.Polyphase(s.p, s.q, c), pp.Filter(s.p, s.q, c))
        streams.append((s.h, s.w, filt[key][0], filt[key][0]))
    plan = aol.BatchPlan(streams, "u8")
    g = synthgen.rng_for(2011, 9)
    frames = [synthgen.gradient_plane(g, s.h, s.w) for s in mix]
    ins = [torch.from_numpy(f).cuda() for f in frames]
    outs = [torch.full(plan.out_shapes[i], fill, dtype=torch.uint8, device="cuda") for i in range(len(mix))]
    plan.set_pointers(ins, outs)
    plan.run()
    torch.cuda.synchronize()
    for i, s in enumerate(mix):
        of = filt[(s.p, s.q, s.taps)][1]
        np.testing.assert_array_equal(outs[i].cpu().numpy(), pp.downscale_u8(frames[i], of, of), err_msg=f"stream {i}")
    plan.close()


@pytest.mark.parametrize("fill", FILLS)
def test_batch_int8_taps_streams_of_the_mix(fill):
    """The streams of the 64-stream mix whose filters fit int8 taps: the fast kernel instance with
    several filters, sizes and K-step counts in one launch, several units per workgroup."""
    mix = [s for s in synthgen.stream_mix(2011, 64)
           if np.abs(np.array(synthgen.design_taps(s.p, s.q, s.taps))).max() <= 127]
    filt = {}
    streams = []
    for s in mix:
        key = (s.p, s.q, s.taps)
        if key not in filt:
            c = synthgen.design_taps(s.p, s.q, s.taps)
            filt[key] = (aol.Polyphase(s.p, s.q, c), pp.Filter(s.p, s.q, c))
        streams.append((s.h, s.w, filt[key][0], filt[key][0]))
    plan = aol.BatchPlan(streams, "u8")
    assert '"launches": 1' in plan.schedule()
    g = synthgen.rng_for(2011, 10)
    frames = [synthgen.gradient_plane(g, s.h, s.w) for s in mix]
    ins = [torch.from_numpy(f).cuda() for f in frames]
    outs = [torch.full(plan.out_shapes[i], fill, dtype=torch.uint8, device="cuda") for i in range(len(mix))]
    plan.set_pointers(ins, outs)
    plan.run()
    torch.cuda.synchronize()
    for i, s in enumerate(mix):
        of = filt[(s.p, s.q, s.taps)][1]
        np.testing.assert_array_equal(outs[i].cpu().numpy(), pp.downscale_u8(frames[i], of, of), err_msg=f"stream {i}")
    plan.close()


# int8-tap and split-tap streams whose lines are whole 16-byte chunks: both parts in one launch
MIX_DUAL = [  # (h, w, p, q, taps, kind)
    (96, 208, 3, 8, 11, "design"),
    (61, 128, 1, 2, 8, "design"),
    (120, 96, 2, 3, 16, "design"),
    (33, 64, 2, 3, 13, "random"),
    (250, 336, 3, 8, 16, "design"),
    (140, 160, 5, 7, 9, "random"),
    (300, 512, 1, 2, 12, "random"),
]


@pytest.mark.parametrize("fill", FILLS)
def test_batch_int8_and_split_taps_in_one_launch(fill):
    """Streams with int8 taps and streams with split taps run as the two parts of one launch
    (each on its own workgroups), directly and through a graph over two steps."""
    st = _streams(MIX_DUAL, seed=40)
    plan = aol.BatchPlan([(h, w, hf, vf) for (h, w, hf, vf, _, _) in st], "u8")
    assert '"launches": 1' in plan.schedule(), plan.schedule()
    steps = 2
    frames = _frames(MIX_DUAL, steps, 31)
    ins = [[torch.from_numpy(fr).cuda() for fr in fs] for fs in frames]
    outs = [[torch.full(plan.out_shapes[i], fill, dtype=torch.uint8, device="cuda") for _ in range(steps)]
            for i in range(len(st))]
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        plan.set_pointers([ins[i][0] for i in range(len(st))], [outs[i][0] for i in range(len(st))], s)
        plan.run(s)
        g = plan.graph(s)
        plan.set_pointers([ins[i][1] for i in range(len(st))], [outs[i][1] for i in range(len(st))], s)
        aol.aol_graph_launch(g, s)
    s.synchronize()
    for i, (h, w, hf, vf, of, ov) in enumerate(st):
        for k in range(steps):
            np.testing.assert_array_equal(outs[i][k].cpu().numpy(), pp.downscale_u8(frames[i][k], of, ov),
                                          err_msg=f"stream {i} step {k}")
    plan.close()


def test_batch_64_streams_one_launch():
    """The 64-stream mix (int8-tap and split-tap filters) is scheduled as one launch."""
    _, _, streams = _mix64()
    plan = aol.BatchPlan(streams, "u8")
    assert '"launches": 1' in plan.schedule(), plan.schedule()
    plan.close()


def _mix64():
    mix = synthgen.stream_mix(2011, 64)
    filt = {}
    streams = []
    for s in mix:
        key = (s.p, s.q, s.taps)
        if key not in filt:
            c = synthgen.design_taps(s.p, s.q, s.taps)
            filt[key] = (aol.Polyphase(s.p, s.q, c), pp.Filter(s.p, s.q, c))
        streams.append((s.h, s.w, filt[key][0], filt[key][0]))
    return mix, filt, streams


# the schedules the autotuner times: segment lengths x LDS budgets (column bands)
TUNE_SEGS = (16, 32, 64, 128)
TUNE_BUDGETS = (150 * 1024, 76 * 1024)


def test_batch_every_tuner_candidate_identical():
    """The 64-stream mix under every schedule the autotuner may pick: each candidate's outputs
    equal the first candidate's on all 64 streams, and the first equals the oracle (results do
    not depend on the schedule)."""
    mix, filt, streams = _mix64()
    plan = aol.BatchPlan(streams, "u8")
    g = synthgen.rng_for(2011, 12)
    frames = [synthgen.gradient_plane(g, s.h, s.w) for s in mix]
    ins = [torch.from_numpy(f).cuda() for f in frames]
    first = None
    n_cand = 0
    for budget in TUNE_BUDGETS:
        for seg in TUNE_SEGS:
            try:
                plan.set_schedule(seg, budget)
            except aol.AolError as e:
                assert e.status == aol.AOL_ERR_UNSUPPORTED, e.msg
                continue
            n_cand += 1
            outs = [torch.full(plan.out_shapes[i], 0xFF if n_cand % 2 else 0x00, dtype=torch.uint8, device="cuda")
                    for i in range(len(mix))]
            plan.set_pointers(ins, outs)
            plan.run()
            torch.cuda.synchronize()
            if first is None:
                first = outs
                for i, s in enumerate(mix):
                    of = filt[(s.p, s.q, s.taps)][1]
                    np.testing.assert_array_equal(outs[i].cpu().numpy(), pp.downscale_u8(frames[i], of, of),
                                                  err_msg=f"stream {i}")
            else:
                for i in range(len(mix)):
                    assert torch.equal(outs[i], first[i]), f"seg {seg} budget {budget}: stream {i} differs"
    assert n_cand >= 4
    plan.close()


def test_batch_part_weights_give_identical_outputs():
    """The 64-stream mix (int8-tap and split-tap streams in one launch) with the workgroups divided
    between the two parts at skewed weights: every stream's output equals the oracle at each
    weight, and a weight out of range is refused with the last one kept."""
    mix, filt, streams = _mix64()
    plan = aol.BatchPlan(streams, "u8")
    g = synthgen.rng_for(2011, 13)
    frames = [synthgen.gradient_plane(g, s.h, s.w) for s in mix]
    ins = [torch.from_numpy(f).cuda() for f in frames]
    want = [pp.downscale_u8(frames[i], filt[(s.p, s.q, s.taps)][1], filt[(s.p, s.q, s.taps)][1])
            for i, s in enumerate(mix)]
    for k, wgt in enumerate((300, 1000, 2500)):
        plan.set_part_weight(wgt)
        sched = json.loads(plan.schedule())
        assert sched["part_weight"] == wgt and sched["launches"] == 1, sched
        outs = [torch.full(plan.out_shapes[i], 0xFF if k % 2 else 0x00, dtype=torch.uint8, device="cuda")
                for i in range(len(mix))]
        plan.set_pointers(ins, outs)
        plan.run()
        torch.cuda.synchronize()
        for i in range(len(mix)):
            np.testing.assert_array_equal(outs[i].cpu().numpy(), want[i], err_msg=f"weight {wgt}: stream {i}")
    with pytest.raises(aol.AolError) as ei:
        plan.set_part_weight(100)
    assert ei.value.status == aol.AOL_ERR_INVALID
    assert json.loads(plan.schedule())["part_weight"] == 2500
    plan.close()


def test_batch_graph_refused_after_reschedule():
    """A graph captured before the schedule changes is refused instead of running its old launch
    over the new tables; a graph captured afterwards runs."""
    st = _streams(MIX[:3])
    plan = aol.BatchPlan([(h, w, hf, vf) for (h, w, hf, vf, _, _) in st], "u8")
    frames = _frames(MIX[:3], 1, 21)
    ins = [torch.from_numpy(fs[0]).cuda() for fs in frames]
    outs = [torch.full(plan.out_shapes[i], 0, dtype=torch.uint8, device="cuda") for i in range(len(st))]
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        plan.set_pointers(ins, outs, s)
        g_old = plan.graph(s)
        plan.set_schedule(32, 76 * 1024)
        with pytest.raises(aol.AolError) as ei:
            aol.aol_graph_launch(g_old, s)
        assert ei.value.status == aol.AOL_ERR_INVALID
        g_new = plan.graph(s)
        aol.aol_graph_launch(g_new, s)
    s.synchronize()
    for i, (h, w, hf, vf, of, ov) in enumerate(st):
        np.testing.assert_array_equal(outs[i].cpu().numpy(), pp.downscale_u8(frames[i][0], of, ov))
    plan.close()
