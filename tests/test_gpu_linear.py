"""GPU parity of the linear integer repetition (uint8) against the CPU oracle: bit-exact.

Workloads: interleaved RGB to planar colour components and the composition back, both with
frames as a repetition dimension; non-separable 2-D polyphase filters with p x p outputs per
repetition; random tilers (strided, transposed and wrapping fittings) with random weights; a
multi-element interleaving output tiler. Every case runs on 16-byte aligned arrays (the staged form
where it applies) and on views one byte off (point by point); outputs are pre-filled with 0x00 and
0xFF: all four runs must agree (every element written once) and leave guard bytes untouched.
"""

import numpy as np
import pytest

import synthgen
from oracle import linear as ln
from oracle.arrayol import Tiler

import torch

import paper_1103_4881_amd as aol  # a missing library fails the suite (no skip)

pytestmark = pytest.mark.gpu


def _ot(spec):
    return Tiler(spec.array_shape, spec.origin, spec.paving, spec.fitting, spec.pat_shape)


def _at(spec, rep):
    return aol.make_tiler(spec.array_shape, rep, spec.pat_shape, spec.origin, spec.paving, spec.fitting)


def _run(X, tin, tout, rep, W, bias):
    """Both forms of the kernel: 16-byte aligned arrays (the staged form wherever the tilers allow
    it) and views one byte off alignment (point by point), each with two sentinel fills and guard
    bytes around the output that must stay untouched."""
    plan = aol.LinearPlan(_at(tin, rep), _at(tout, rep), W, bias)
    shape = tuple(tout.array_shape)
    n_in, n_out = int(X.size), int(np.prod(shape))
    outs = []
    for off in (0, 1):
        xb = torch.empty(n_in + 32, dtype=torch.uint8, device="cuda")
        x = xb[off:off + n_in].view(X.shape)
        x.copy_(torch.from_numpy(np.ascontiguousarray(X)))
        for fill in (0x00, 0xFF):
            yb = torch.full((n_out + 32,), fill, dtype=torch.uint8, device="cuda")
            plan.run(x, yb[off:off + n_out].view(shape))
            torch.cuda.synchronize()
            h = yb.cpu().numpy()
            assert (h[:off] == fill).all() and (h[off + n_out:] == fill).all(), "write outside the output"
            outs.append(h[off:off + n_out].reshape(shape))
    plan.close()
    for k in range(1, len(outs)):
        np.testing.assert_array_equal(outs[0], outs[k], err_msg=f"outputs differ between forms / fills ({k})")
    return outs[0]


def _oracle(X, tin, tout, rep, W, bias):
    B, cnt = ln.linear_u8(X, _ot(tin), W, bias, _ot(tout), rep)
    assert (cnt == 1).all()
    return B


def _frames_spec(spec, frames):
    """The same tiler with a leading frame dimension in the array and the repetition space."""
    d = len(spec.array_shape)
    paving = [[1] + [0] * len(spec.paving[0])] + [[0] + list(row) for row in spec.paving]
    fitting = [[0] * len(spec.fitting[0])] + [list(row) for row in spec.fitting]
    return synthgen.TilerSpec((frames,) + tuple(spec.array_shape), (0,) + tuple(spec.origin), paving, fitting,
                              spec.pat_shape)


@pytest.mark.parametrize("h,w", [(1, 1), (37, 53), (270, 480)])
def test_rgb_to_planar_ycc_and_back(h, w):
    X = synthgen.uniform_frame(h * 7 + w, h, 3 * w)
    rep, tin, tout = synthgen.rgb_to_planar_tilers(h, w)
    Y = _run(X, tin, tout, rep, synthgen.RGB_TO_YCC_W, synthgen.RGB_TO_YCC_BIAS)
    np.testing.assert_array_equal(Y, _oracle(X, tin, tout, rep, synthgen.RGB_TO_YCC_W, synthgen.RGB_TO_YCC_BIAS))
    rep2, tin2, tout2 = synthgen.planar_to_rgb_tilers(h, w)
    Z = _run(Y, tin2, tout2, rep2, synthgen.YCC_TO_RGB_W, synthgen.YCC_TO_RGB_BIAS)
    np.testing.assert_array_equal(Z, _oracle(Y, tin2, tout2, rep2, synthgen.YCC_TO_RGB_W, synthgen.YCC_TO_RGB_BIAS))


def test_rgb_frames_1080p_as_a_repetition_dimension():
    """Eight 1920x1080 RGB frames -> planar colour components in one launch (repetition space
    frames x lines x pixels), every element against the oracle; then the composition back."""
    F, h, w = 8, 1080, 1920
    X = np.stack([synthgen.uniform_frame(900 + f, h, 3 * w) for f in range(F)])
    rep0, tin0, tout0 = synthgen.rgb_to_planar_tilers(h, w)
    rep, tin, tout = (F,) + tuple(rep0), _frames_spec(tin0, F), _frames_spec(tout0, F)
    Y = _run(X, tin, tout, rep, synthgen.RGB_TO_YCC_W, synthgen.RGB_TO_YCC_BIAS)
    for f in (0, 5, 7):
        np.testing.assert_array_equal(Y[f], _oracle(X[f], tin0, tout0, rep0, synthgen.RGB_TO_YCC_W,
                                                    synthgen.RGB_TO_YCC_BIAS), err_msg=f"frame {f}")
    rep20, tin20, tout20 = synthgen.planar_to_rgb_tilers(h, w)
    rep2, tin2, tout2 = (F,) + tuple(rep20), _frames_spec(tin20, F), _frames_spec(tout20, F)
    Z = _run(Y, tin2, tout2, rep2, synthgen.YCC_TO_RGB_W, synthgen.YCC_TO_RGB_BIAS)
    for f in (0, 3, 7):
        np.testing.assert_array_equal(Z[f], _oracle(Y[f], tin20, tout20, rep20, synthgen.YCC_TO_RGB_W,
                                                    synthgen.YCC_TO_RGB_BIAS), err_msg=f"frame {f}")


@pytest.mark.parametrize("h,w,p,q,T", [(288, 352, 3, 8, 11), (101, 135, 3, 8, 11), (64, 90, 4, 9, 7),
                                       (33, 47, 2, 3, 5), (40, 40, 1, 2, 8), (17, 19, 1, 1, 3)])
def test_non_separable_2d_polyphase(h, w, p, q, T):
    X = synthgen.uniform_frame(h + w, h, w)
    rep, tin, tout, starts, span = synthgen.polyphase2d_tilers(h, w, p, q, T)
    W = synthgen.polyphase2d_weights(h * w, p, q, T)
    Y = _run(X, tin, tout, rep, W, None)
    np.testing.assert_array_equal(Y, _oracle(X, tin, tout, rep, W, None))


@pytest.mark.parametrize("rx,shift", [(255, 0), (256, 0), (257, 0), (200, 8 * 97), (256, 8 * 131 + 3)])
def test_rows_around_one_point_per_thread(rx, shift):
    """Rows of 255, 256 and 257 repetitions (the point-by-point kernel rotates a row's points over
    its threads only while each thread takes one point), and input origins moved along the row so
    that the points whose window crosses the left or right edge sit inside the row."""
    h, w, p, q, T = 19, 8 * rx, 3, 8, 11
    X = synthgen.uniform_frame(rx + shift, h, w)
    rep, tin, tout, _, _ = synthgen.polyphase2d_tilers(h, w, p, q, T)
    tin = synthgen.TilerSpec(tin.array_shape, (tin.origin[0], tin.origin[1] + shift), tin.paving, tin.fitting,
                             tin.pat_shape)
    W = synthgen.polyphase2d_weights(rx, p, q, T)
    Y = _run(X, tin, tout, rep, W, None)
    np.testing.assert_array_equal(Y, _oracle(X, tin, tout, rep, W, None))


@pytest.mark.parametrize("seed", range(6))
def test_random_tilers_and_weights(seed):
    """Random signed-permutation pavings with strides and a shear, fittings along distinct axes
    (strided, reversed), random origins, an identity output tiler, random weights and biases."""
    rt = synthgen.random_tiler(300 + seed, array_shape=(6, 23, 31), pat_shape=(3, 4))
    g = synthgen.rng_for(301 + seed, 0)
    X = g.integers(0, 256, size=rt.array_shape).astype(np.uint8)
    W = g.integers(-300, 300, size=(1, 12)).astype(np.int16)
    bias = g.integers(-5000, 5000, size=1).astype(np.int32)
    tin = synthgen.TilerSpec(rt.array_shape, rt.origin, rt.paving.tolist(), rt.fitting.tolist(), rt.pat_shape)
    d = len(rt.rep_shape)
    tout = synthgen.TilerSpec(tuple(rt.rep_shape), (0,) * d, np.eye(d, dtype=np.int64).tolist(),
                              np.zeros((d, 0), np.int64).tolist(), ())
    Y = _run(X, tin, tout, tuple(rt.rep_shape), W, bias)
    np.testing.assert_array_equal(Y, _oracle(X, tin, tout, tuple(rt.rep_shape), W, bias))


def test_interleaving_output_pattern_and_wrapping_input():
    """Two outputs per repetition written interleaved (output fitting 1, paving 2) from a 5 x 3
    input pattern that wraps the array's borders (origin -2, -1)."""
    h, w = 23, 29
    X = synthgen.uniform_frame(41, h, w)
    tin = synthgen.TilerSpec((h, w), (-2, -1), [[1, 0], [0, 1]], [[1, 0], [0, 1]], (5, 3))
    tout = synthgen.TilerSpec((h, 2 * w), (0, 0), [[1, 0], [0, 2]], [[0], [1]], (2,))
    g = synthgen.rng_for(42, 0)
    W = g.integers(-100, 200, size=(2, 15)).astype(np.int16)
    Y = _run(X, tin, tout, (h, w), W, np.array([300, -700], np.int32))
    np.testing.assert_array_equal(Y, _oracle(X, tin, tout, (h, w), W, np.array([300, -700])))


@pytest.mark.parametrize("h,w", [(5, 3001), (2, 2049), (3, 4096)])
def test_rgb_rows_of_several_chunks(h, w):
    """Rows longer than one staged chunk (2048 points): whole chunks, a partial last chunk."""
    X = synthgen.uniform_frame(h + w, h, 3 * w)
    rep, tin, tout = synthgen.rgb_to_planar_tilers(h, w)
    Y = _run(X, tin, tout, rep, synthgen.RGB_TO_YCC_W, synthgen.RGB_TO_YCC_BIAS)
    np.testing.assert_array_equal(Y, _oracle(X, tin, tout, rep, synthgen.RGB_TO_YCC_W, synthgen.RGB_TO_YCC_BIAS))
    rep2, tin2, tout2 = synthgen.planar_to_rgb_tilers(h, w)
    Z = _run(Y, tin2, tout2, rep2, synthgen.YCC_TO_RGB_W, synthgen.YCC_TO_RGB_BIAS)
    np.testing.assert_array_equal(Z, _oracle(Y, tin2, tout2, rep2, synthgen.YCC_TO_RGB_W, synthgen.YCC_TO_RGB_BIAS))


def test_wide_wrapping_pattern_mixes_clean_and_border_chunks():
    """A 5 x 3 pattern wrapping both borders on rows of 5000 points: the chunks at a row's ends
    cross a border (point by point), the middle ones do not (staged), rows at the top and bottom
    wrap vertically."""
    h, w = 9, 5000
    X = synthgen.uniform_frame(43, h, w)
    tin = synthgen.TilerSpec((h, w), (-2, -1), [[1, 0], [0, 1]], [[1, 0], [0, 1]], (5, 3))
    tout = synthgen.TilerSpec((h, 2 * w), (0, 0), [[1, 0], [0, 2]], [[0], [1]], (2,))
    g = synthgen.rng_for(44, 0)
    W = g.integers(-100, 200, size=(2, 15)).astype(np.int16)
    bias = np.array([-300, 900], np.int32)
    Y = _run(X, tin, tout, (h, w), W, bias)
    np.testing.assert_array_equal(Y, _oracle(X, tin, tout, (h, w), W, bias))


def test_outputs_interleaved_by_two_repetitions():
    """Repetition space (2, h, w): both k = 0 and k = 1 read in[y][x - 1 .. x + 1] and write
    out[y][2 x + k], so a row's outputs lie two elements apart (no dense output range: clean chunks
    store point by point from registers; rows of three chunks, the middle one clean)."""
    h, w = 11, 5000
    X = synthgen.uniform_frame(45, h, w)
    tin = synthgen.TilerSpec((h, w), (0, -1), [[0, 1, 0], [0, 0, 1]], [[0], [1]], (3,))
    tout = synthgen.TilerSpec((h, 2 * w), (0, 0), [[0, 1, 0], [1, 0, 2]], [[], []], ())
    W = np.array([[60, 120, 76]], np.int16)
    Y = _run(X, tin, tout, (2, h, w), W, np.array([-50], np.int32))
    np.testing.assert_array_equal(Y, _oracle(X, tin, tout, (2, h, w), W, np.array([-50])))


def test_errors():
    h, w = 4, 5
    rep, tin, tout = synthgen.rgb_to_planar_tilers(h, w)
    bad_out = synthgen.TilerSpec((3, h, w), (0, 0, 0), [[0, 0], [1, 0], [0, 0]], [[1], [0], [0]], (3,))
    with pytest.raises(aol.AolError) as e:  # every pixel of a line lands on the same output
        aol.LinearPlan(_at(tin, rep), _at(bad_out, rep), synthgen.RGB_TO_YCC_W)
    assert e.value.status == aol.AOL_ERR_INVALID
    with pytest.raises(aol.AolError) as e:  # sums beyond int32
        aol.LinearPlan(_at(tin, rep), _at(tout, rep), np.full((3, 3), 32767, np.int16), np.full(3, 2 ** 31 - 1))
    assert e.value.status == aol.AOL_ERR_UNSUPPORTED
    big = synthgen.TilerSpec((17 * h * w,), (0,), [[17 * w, 17]], [[1]], (17,))
    with pytest.raises(aol.AolError) as e:  # 17 outputs per repetition
        aol.LinearPlan(_at(synthgen.TilerSpec((h, w), (0, 0), [[1, 0], [0, 1]], [[], []], ()), rep),
                       _at(big, rep), np.ones((17, 1), np.int16))
    assert e.value.status == aol.AOL_ERR_UNSUPPORTED
