"""Pins of the linear integer repetition oracle (oracle/linear.py), CPU only.

Each pin is fixed by something other than the oracle's own formula:
numpy reshapes and transposes for interleaving (the tilers of RGB and planar
frames), scipy's circular correlation for a 2-D filter with identity tilers,
exhaustive constant-preserving invariants of the colour weights, the literal
interpreter with exact coverage on random tilers, and block sums of a 2 x 2
box filter by reshaping. The mutation tests at the end plant plausible
mistakes and check that a pin fails.
"""

import numpy as np
import pytest
import scipy.ndimage

import synthgen
from oracle import linear as ln
from oracle.arrayol import Tiler


def _t(spec):
    return Tiler(spec.array_shape, spec.origin, spec.paving, spec.fitting, spec.pat_shape)


def _rgb(h, w, seed=0):
    return synthgen.uniform_frame(seed, h, 3 * w)


def test_identity_weights_deinterleave_equals_transpose():
    h, w = 7, 11
    X = _rgb(h, w, 1)
    R, tin, tout = synthgen.rgb_to_planar_tilers(h, w)
    B, cnt = ln.linear_u8(X, _t(tin), 256 * np.eye(3, dtype=np.int64), None, _t(tout), R)
    assert (cnt == 1).all()
    np.testing.assert_array_equal(B, X.reshape(h, w, 3).transpose(2, 0, 1))


def test_identity_weights_interleave_equals_stack():
    h, w = 5, 9
    P = np.stack([synthgen.uniform_frame(2, h, w, idx=k) for k in range(3)])
    R, tin, tout = synthgen.planar_to_rgb_tilers(h, w)
    B, cnt = ln.linear_u8(P, _t(tin), 256 * np.eye(3, dtype=np.int64), None, _t(tout), R)
    assert (cnt == 1).all()
    np.testing.assert_array_equal(B, np.stack(list(P), axis=-1).reshape(h, 3 * w))


def test_channel_permutation_weights():
    h, w = 4, 6
    X = _rgb(h, w, 3)
    R, tin, tout = synthgen.rgb_to_planar_tilers(h, w)
    Wp = 256 * np.eye(3, dtype=np.int64)[[2, 0, 1]]  # out0 = B, out1 = R, out2 = G
    B, _ = ln.linear_u8(X, _t(tin), Wp, None, _t(tout), R)
    planes = X.reshape(h, w, 3).transpose(2, 0, 1)
    np.testing.assert_array_equal(B, planes[[2, 0, 1]])


def test_colour_weights_keep_every_grey_level():
    """Luma rows sum to 256 and chroma rows to 0 with offset 128: every grey (v, v, v) maps to
    (v, 128, 128) exactly, and back (the inverse rows sum to 256 with the offsets cancelling)."""
    v = np.arange(256, dtype=np.uint8)
    X = np.repeat(v, 3).reshape(1, 3 * 256)
    R, tin, tout = synthgen.rgb_to_planar_tilers(1, 256)
    B, _ = ln.linear_u8(X, _t(tin), synthgen.RGB_TO_YCC_W, synthgen.RGB_TO_YCC_BIAS, _t(tout), R)
    np.testing.assert_array_equal(B[0, 0], v)
    assert (B[1:] == 128).all()
    R2, tin2, tout2 = synthgen.planar_to_rgb_tilers(1, 256)
    C, _ = ln.linear_u8(B, _t(tin2), synthgen.YCC_TO_RGB_W, synthgen.YCC_TO_RGB_BIAS, _t(tout2), R2)
    np.testing.assert_array_equal(C, X)


@pytest.mark.parametrize("T", [3, 5])
def test_2d_filter_with_unit_ratio_is_circular_correlation(T):
    """p = q = 1: one output per pixel, a T x T window centred on it; equals scipy's circular
    correlation followed by the round-shift and clamp."""
    h, w = 9, 13
    X = synthgen.uniform_frame(4, h, w)
    R, tin, tout, starts, span = synthgen.polyphase2d_tilers(h, w, 1, 1, T)
    assert span == T
    K = synthgen.rng_for(5, 0).integers(-40, 90, size=(T, T))
    B, cnt = ln.linear_u8(X, _t(tin), K.reshape(1, -1), None, _t(tout), R)
    assert (cnt == 1).all()
    corr = scipy.ndimage.correlate(X.astype(np.int64), K.astype(np.int64), mode="wrap")
    np.testing.assert_array_equal(B, np.clip(np.floor_divide(corr + 128, 256), 0, 255))


def test_2d_box_filter_equals_block_sums():
    """p = 1, q = 2, a 2 x 2 window of weights 64: each output is the rounded mean of a
    2 x 2 block (the window of repetition (r, c) is rows 2r..2r+1, columns 2c..2c+1),
    i.e. a reshape-and-sum in numpy."""
    h, w = 12, 18
    X = synthgen.uniform_frame(6, h, w)
    R, tin, tout, starts, span = synthgen.polyphase2d_tilers(h, w, 1, 2, 2)
    assert starts == [0] and span == 2
    B, cnt = ln.linear_u8(X, _t(tin), np.full((1, 4), 64), None, _t(tout), R)
    assert (cnt == 1).all()
    s = X.astype(np.int64).reshape(h // 2, 2, w // 2, 2).sum(axis=(1, 3))
    np.testing.assert_array_equal(B, np.clip((64 * s + 128) // 256, 0, 255))


def _random_case(seed):
    g = synthgen.rng_for(seed, 9)
    h, w = int(g.integers(2, 7)), int(g.integers(2, 7))
    kind = seed % 3
    if kind == 0:
        R, tin, tout = synthgen.rgb_to_planar_tilers(h, w)
        A = synthgen.uniform_frame(seed, h, 3 * w)
    elif kind == 1:
        R, tin, tout = synthgen.planar_to_rgb_tilers(h, w)
        A = np.stack([synthgen.uniform_frame(seed, h, w, idx=k) for k in range(3)])
    else:
        p, q, T = [(2, 3, 4), (1, 2, 3), (3, 2, 2)][seed % 3]
        R, tin, tout, _, _ = synthgen.polyphase2d_tilers(h * q, w * q, p, q, T)
        A = synthgen.uniform_frame(seed, h * q, w * q)
    n_in = int(np.prod(tin.pat_shape))
    n_out = int(np.prod(tout.pat_shape))
    W = g.integers(-300, 400, size=(n_out, n_in))
    b = g.integers(-5000, 5000, size=n_out)
    return A, tin, tout, R, W, b


@pytest.mark.parametrize("seed", range(9))
def test_vectorised_equals_interpreter_with_exact_coverage(seed):
    A, tin, tout, R, W, b = _random_case(seed)
    B1, c1 = ln.linear_u8(A, _t(tin), W, b, _t(tout), R)
    B2, c2 = ln.linear_u8_interp(A, _t(tin), W, b, _t(tout), R)
    assert (c1 == 1).all() and (c2 == 1).all()
    np.testing.assert_array_equal(B1, B2)


# ---------------------------------------------------------------- planted mistakes

def _fails(fn, *a):
    try:
        fn(*a)
    except AssertionError:
        return True
    return False


def test_mutation_truncating_round_is_caught(monkeypatch):
    monkeypatch.setattr(ln, "_quantise", lambda acc: np.clip(acc // 256, 0, 255))
    assert _fails(test_2d_filter_with_unit_ratio_is_circular_correlation, 3)


def test_mutation_missing_clamp_is_caught(monkeypatch):
    monkeypatch.setattr(ln, "_quantise", lambda acc: np.floor_divide(acc + 128, 256) % 256)
    assert _fails(test_2d_filter_with_unit_ratio_is_circular_correlation, 5)


def test_mutation_fitting_sign_is_caught(monkeypatch):
    orig = ln._gather_index

    def flipped(t, r, i):
        return orig(t, r, tuple(-v for v in i))

    monkeypatch.setattr(ln, "_gather_index", flipped)
    assert _fails(test_identity_weights_deinterleave_equals_transpose)


def test_mutation_transposed_weights_are_caught(monkeypatch):
    orig = ln.linear_u8

    def transposed(A, tin, W, bias, tout, R):
        return orig(A, tin, np.asarray(W).reshape(3, 3).T, bias, tout, R)

    monkeypatch.setattr(ln, "linear_u8", transposed)
    assert _fails(test_channel_permutation_weights)
