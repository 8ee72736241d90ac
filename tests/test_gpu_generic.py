"""GPU parity of the generic Array-OL weighted-sum repetition against the
float64 oracle: |y - y64| <= 1e-5 * sum_i |w_i x_i| per output element
(float32 fused multiply-adds over at most 64 terms stay far inside it)."""

import numpy as np
import pytest

import synthgen
from oracle import generic as gn
from oracle.arrayol import Tiler

import torch

import paper_1103_4881_amd as aol  # a missing library fails the suite (no skip)

pytestmark = pytest.mark.gpu

REL = 1e-5


def _otiler(t):
    return Tiler(tuple(t.array_shape), tuple(t.origin), np.asarray(t.paving).tolist(),
                 np.asarray(t.fitting).tolist(), tuple(t.pat_shape))


def _atiler(rt):
    return aol.make_tiler(rt.array_shape, rt.rep_shape, rt.pat_shape, rt.origin, rt.paving, rt.fitting)


def _run(A, tin, tout, w):
    plan = aol.WeightedSumPlan(tin, tout, w)
    x = torch.from_numpy(A).cuda()
    y = torch.full(plan.out_shape, float("nan"), dtype=torch.float32, device="cuda")
    plan.run(x, y)
    torch.cuda.synchronize()
    plan.close()
    return y.cpu().numpy()


def _check(got, ref, mag):
    assert np.isfinite(got).all(), "an output element was not written"
    err = np.abs(got.astype(np.float64) - ref)
    bound = REL * np.maximum(mag, 1e-30)
    assert (err <= bound).all(), f"max rel err {float((err / bound).max()) * REL:.3e}"


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("shape,pat", [((7, 9, 11), (3, 2)), ((33, 70), (5, 5)), ((4, 6, 5, 8), (2, 3)),
                                       ((300,), (7,)), ((96, 130), (3, 3))])
def test_random_tilers_identity_output(seed, shape, pat):
    rt = synthgen.random_tiler(seed, array_shape=shape, pat_shape=pat)
    A = synthgen.rng_for(seed, 1).uniform(-1, 1, size=shape).astype(np.float32)
    w = synthgen.rng_for(seed, 2).uniform(-1, 1, size=pat).astype(np.float32)
    tin = _atiler(rt)
    tout = aol.identity_out_tiler(rt.rep_shape)
    got = _run(A, tin, tout, w)
    B, M, cnt = gn.weighted_sum_f64(A, _otiler(rt), w, _otiler_id(rt.rep_shape), rt.rep_shape)
    assert cnt.min() == 1 and cnt.max() == 1
    _check(got, B, M)


def _otiler_id(rep_shape):
    d = len(rep_shape)
    return Tiler(tuple(rep_shape), (0,) * d, np.eye(d, dtype=np.int64).tolist(), [[] for _ in range(d)], ())


def test_permuted_output_tiler():
    """Output written through a non-identity bijective tiler (transposed, shifted)."""
    rt = synthgen.random_tiler(3, array_shape=(20, 24), pat_shape=(3, 3))
    R = rt.rep_shape
    A = synthgen.rng_for(3, 1).uniform(-1, 1, size=rt.array_shape).astype(np.float32)
    w = synthgen.rng_for(3, 2).uniform(-1, 1, size=(3, 3)).astype(np.float32)
    # out[(2 + r1) mod R1, (5 + r0) mod R0]: a transposed, rotated output array
    oshape = (R[1], R[0])
    Pout = np.array([[0, 1], [1, 0]])
    tout_a = aol.make_tiler(oshape, R, (), (2, 5), Pout, np.zeros((2, 0), np.int64))
    tout_o = Tiler(oshape, (2, 5), Pout.tolist(), [[], []], ())
    got = _run(A, _atiler(rt), tout_a, w)
    B, M, cnt = gn.weighted_sum_f64(A, _otiler(rt), w, tout_o, R)
    assert cnt.min() == 1 and cnt.max() == 1
    _check(got, B, M)


def test_pattern_longer_than_array_wraps():
    A = synthgen.rng_for(9, 0).uniform(-1, 1, size=(3, 5)).astype(np.float32)
    tin = aol.make_tiler((3, 5), (3, 5), (4, 7), (1, 2), [[1, 0], [0, 1]], [[2, 0], [0, 3]])
    w = synthgen.rng_for(9, 1).uniform(-1, 1, size=(4, 7)).astype(np.float32)
    got = _run(A, tin, aol.identity_out_tiler((3, 5)), w)
    B, M, _ = gn.weighted_sum_f64(A, Tiler((3, 5), (1, 2), [[1, 0], [0, 1]], [[2, 0], [0, 3]], (4, 7)), w,
                                  _otiler_id((3, 5)), (3, 5))
    _check(got, B, M)


def test_full_size_64x1024x1024_sampled():
    """The 64x1024x1024 float32 array with a random tiler and 5x5 weights; 20000 sampled outputs."""
    rt = synthgen.random_tiler(2011, array_shape=(64, 1024, 1024), pat_shape=(5, 5))
    A = synthgen.rng_for(2011, 1).uniform(-1, 1, size=rt.array_shape).astype(np.float32)
    w = synthgen.rng_for(2011, 2).uniform(-1, 1, size=(5, 5)).astype(np.float32)
    plan = aol.WeightedSumPlan(_atiler(rt), aol.identity_out_tiler(rt.rep_shape), w)
    x = torch.from_numpy(A).cuda()
    y = torch.full(plan.out_shape, float("nan"), dtype=torch.float32, device="cuda")
    plan.run(x, y)
    torch.cuda.synchronize()
    yc = y.cpu().numpy()
    assert np.isfinite(yc).all()
    g = synthgen.rng_for(2011, 3)
    r = np.stack([g.integers(0, n, size=20000) for n in rt.rep_shape])
    ref, mag = gn.weighted_sum_at(A, _otiler(rt), w, r)
    _check(yc[tuple(r)], ref, mag)
    plan.close()


@pytest.mark.parametrize("seed", range(3))
def test_one_shot_entry_point_equals_plan(seed):
    """aol_weighted_sum_f32 (no plan, weights in the kernel arguments) and a plan's run both equal
    the oracle (a plan may group the sum by shared reads, so the two can differ in rounding)."""
    rt = synthgen.random_tiler(40 + seed, array_shape=(24, 40, 36), pat_shape=(5, 5))
    A = synthgen.rng_for(40 + seed, 1).uniform(-1, 1, size=rt.array_shape).astype(np.float32)
    w = synthgen.rng_for(40 + seed, 2).uniform(-1, 1, size=(5, 5)).astype(np.float32)
    tin, tout = _atiler(rt), aol.identity_out_tiler(rt.rep_shape)
    via_plan = _run(A, tin, tout, w)
    x = torch.from_numpy(A).cuda()
    y = torch.full(tuple(rt.rep_shape), float("nan"), dtype=torch.float32, device="cuda")
    aol.aol_weighted_sum_f32(tin, tout, w, x.data_ptr(), y.data_ptr())
    torch.cuda.synchronize()
    got = y.cpu().numpy()
    B, M, _ = gn.weighted_sum_f64(A, _otiler(rt), w, _otiler_id(rt.rep_shape), rt.rep_shape)
    _check(got, B, M)
    _check(via_plan, B, M)


# Fittings along the axis that the loop dimension's paving walks: neighbouring points share reads
# (classes of widths 3, 5 and 8, with gaps and reversed steps), and one too wide for sharing.
SHARED = [
    ((96, 130), (5, 5), [[1, 0], [0, 1]], [[1, 0], [0, 1]], (0, 0)),
    ((70, 64), (3, 3), [[1, 0], [0, 1]], [[1, 0], [0, 1]], (3, 60)),
    ((64, 96), (4, 3), [[1, 0], [0, 1]], [[2, 0], [0, 1]], (5, 7)),
    ((80, 72), (5, 2), [[1, 0], [0, 2]], [[-1, 0], [0, 1]], (79, 1)),
    ((50, 66), (9, 2), [[1, 0], [0, 1]], [[1, 0], [0, 1]], (2, 2)),
    ((12, 40, 48), (3, 5), [[1, 0, 0], [0, 1, 0], [0, 0, 1]], [[0, 0], [1, 0], [0, 1]], (0, 39, 5)),
]


@pytest.mark.parametrize("case", SHARED, ids=[f"{c[0]}-{c[1]}" for c in SHARED])
def test_shared_reads_along_the_loop_dimension(case):
    shape, pat, paving, fitting, origin = case
    P = np.array(paving)
    rep = tuple(int(-(-shape[d] // max(1, abs(P[d]).max()))) for d in range(len(shape)))
    A = synthgen.rng_for(sum(shape), 1).uniform(-1, 1, size=shape).astype(np.float32)
    w = synthgen.rng_for(sum(shape), 2).uniform(-1, 1, size=pat).astype(np.float32)
    tin = aol.make_tiler(shape, rep, pat, origin, paving, fitting)
    got = _run(A, tin, aol.identity_out_tiler(rep), w)
    B, M, cnt = gn.weighted_sum_f64(A, Tiler(shape, origin, paving, fitting, pat), w, _otiler_id(rep), rep)
    assert cnt.min() == 1 and cnt.max() == 1
    _check(got, B, M)
