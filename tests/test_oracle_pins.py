"""Pins for the CPU oracle: it is checked against things other than itself.

* sizes the paper prints (the CIF frame sizes and the [288, 44] multiplicity);
* special cases that reduce to library routines (identity, decimation via
  ``np.take(mode='wrap')``, integer shifts via ``np.roll``, circular
  correlation via ``scipy.ndimage.correlate(mode='wrap')``);
* closed forms (two-tap averages with round-half-up, clamped extrapolation);
* invariants (constant frames for every value 0..255, shift equivariance,
  exact coverage, linearity, H/V commutation of the float form);
* brute force through the literal Array-OL interpreter on tiny inputs.
"""

import json
import os

import numpy as np
import pytest
import scipy.ndimage

import synthgen
from oracle import polyphase as pp
from oracle import generic as gn
from oracle.arrayol import Tiler

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _flt(p, q, T, seed=0, kind="design"):
    if kind == "design":
        c = synthgen.design_taps(p, q, T)
    else:  # random integer taps with negative entries, each phase summing to 256
        g = synthgen.rng_for(seed, 99)
        c = g.integers(-300, 300, size=(p, T))
        c[:, 0] += 256 - c.sum(axis=1)
    return pp.Filter(p, q, c)


# ---------------------------------------------------------------- paper sizes

def test_paper_cif_shapes_through_interpreter():
    """Sec. III / III-A: 352 -> 132 per line in packets of 8, multiplicity [288, 44]."""
    with open(os.path.join(GOLDEN, "paper_cif.json")) as fh:
        g = json.load(fh)
    X = synthgen.uniform_frame(1, g["in_height"], g["in_width"])
    hf = _flt(3, g["packet"], 11)
    Z, counts, rep = pp.hfilter_task(X, hf)
    assert list(rep) == g["h_multiplicity"]
    assert Z.shape == (g["in_height"], g["out_width"])
    assert counts.min() == 1 and counts.max() == 1
    np.testing.assert_array_equal(Z, pp.polyphase_int_axis(X, hf, axis=-1))
    # the vertical 288 -> 128 the paper prints is reached at ratio 4/9 (see DESIGN readings)
    assert pp.output_length(g["in_height"], 4, 9) == g["out_height"]
    assert pp.repetitions(g["in_height"], 9) * 4 == g["out_height"]


def test_default_phase_starts_known_values():
    # 3/8 with 11 taps: output centres at 5/6, 7/2, 37/6 input pixels
    assert pp.default_phase_starts(3, 8, 11) == [-5, -2, 1]
    # no scaling: centres fall on input pixels, odd windows are symmetric
    assert pp.default_phase_starts(1, 1, 3) == [-1]
    assert pp.default_phase_starts(2, 2, 5) == [-2, -1]
    # 1/2 with two taps averages pixels 2r and 2r+1
    assert pp.default_phase_starts(1, 2, 2) == [0]


@pytest.mark.parametrize("p,q,T", [(3, 8, 11), (1, 2, 8), (2, 3, 16), (4, 9, 7), (5, 3, 6), (1, 1, 1)])
def test_default_window_contains_centre(p, q, T):
    s = pp.default_phase_starts(p, q, T)
    for phi in range(p):
        u = ((2 * phi + 1) * q - p) / (2 * p)  # geometric centre in input pixel index units
        assert s[phi] <= u < s[phi] + T
        # the window's middle tap is within one pixel of the centre
        assert abs(s[phi] + (T - 1) / 2 - u) <= 1.0


# ---------------------------------------------------------------- special cases

def test_identity_filter():
    X = synthgen.uniform_frame(3, 37, 53)
    f = pp.Filter(1, 1, [[256]])
    np.testing.assert_array_equal(pp.downscale_u8(X, f, f), X)
    g = pp.Filter(1, 1, [[0, 256, 0]])  # centred delta in a 3-tap window
    np.testing.assert_array_equal(pp.downscale_u8(X, g, g), X)
    h = pp.Filter(2, 2, [[0, 0, 256, 0, 0], [0, 0, 256, 0, 0]])
    # odd lengths: the last packet is completed by wrapping to the first pixel
    Y = pp.downscale_u8(X, h, h)
    assert Y.shape == (38, 54)
    np.testing.assert_array_equal(Y, np.take(np.take(X, np.arange(38), axis=0, mode="wrap"),
                                             np.arange(54), axis=1, mode="wrap"))


@pytest.mark.parametrize("q,T,k0", [(2, 1, 0), (3, 4, 2), (8, 11, 5), (5, 7, 0), (4, 3, 2)])
def test_decimation_equals_take_wrap(q, T, k0):
    X = synthgen.uniform_frame(4, 29, 41)
    c = np.zeros((1, T), np.int64)
    c[0, k0] = 256
    f = pp.Filter(1, q, c)
    s = f.s[0]
    rows = q * np.arange(pp.repetitions(X.shape[0], q)) + s + k0
    cols = q * np.arange(pp.repetitions(X.shape[1], q)) + s + k0
    ref = np.take(np.take(X, rows, axis=0, mode="wrap"), cols, axis=1, mode="wrap")
    np.testing.assert_array_equal(pp.downscale_u8(X, f, f), ref)


def test_shifted_delta_equals_roll():
    X = synthgen.uniform_frame(5, 24, 30)
    for shift in range(-3, 4):
        T = 7
        c = np.zeros((3, T), np.int64)
        s = pp.default_phase_starts(3, 3, T)
        for phi in range(3):
            c[phi, phi + shift - s[phi]] = 256  # output o reads input o + shift
        f = pp.Filter(3, 3, c)
        np.testing.assert_array_equal(pp.polyphase_int_axis(X, f, axis=-1), np.roll(X, -shift, axis=1))
        np.testing.assert_array_equal(pp.polyphase_int_axis(X, f, axis=-2), np.roll(X, -shift, axis=0))


# ---------------------------------------------------------------- closed forms

def test_two_tap_average_rounds_half_up():
    X = synthgen.uniform_frame(6, 16, 64).astype(np.int64)
    f = pp.Filter(1, 2, [[128, 128]])
    y = pp.polyphase_int_axis(X, f, axis=-1)
    a, b = X[:, 0::2], X[:, 1::2]
    np.testing.assert_array_equal(y, (a + b + 1) >> 1)


def test_extrapolating_taps_clamp():
    X = synthgen.uniform_frame(7, 8, 64).astype(np.int64)
    f = pp.Filter(1, 2, [[-256, 512]])  # 2*b - a, clamped
    y = pp.polyphase_int_axis(X, f, axis=-1)
    a, b = X[:, 0::2], X[:, 1::2]
    np.testing.assert_array_equal(y, np.clip(2 * b - a, 0, 255))
    f2 = pp.Filter(1, 2, [[-128, 384]])  # (3b - a)/2 rounded half up, clamped
    y2 = pp.polyphase_int_axis(X, f2, axis=-1)
    np.testing.assert_array_equal(y2, np.clip((3 * b - a + 1) >> 1, 0, 255))


# ---------------------------------------------------------------- invariants

@pytest.mark.parametrize("p,q,T,kind", [(3, 8, 11, "design"), (1, 2, 8, "design"), (2, 3, 16, "design"),
                                         (3, 8, 11, "random"), (4, 9, 5, "random"), (2, 3, 13, "random")])
def test_constant_frame_is_fixed_for_every_value(p, q, T, kind):
    f = _flt(p, q, T, seed=p * 100 + T, kind=kind)
    assert (f.c.sum(axis=1) == 256).all()
    X = np.broadcast_to(np.arange(256, dtype=np.uint8)[:, None, None], (256, 20, 27))
    Y = pp.downscale_u8(X, f, f)
    np.testing.assert_array_equal(Y, np.broadcast_to(np.arange(256, dtype=np.uint8)[:, None, None], Y.shape))
    # the float form keeps a constant too (weights sum to one)
    Yf = pp.downscale_f64(X[::51].astype(np.float64) / 255.0, f, f)
    np.testing.assert_allclose(Yf, np.broadcast_to(np.arange(0, 256, 51)[:, None, None] / 255.0, Yf.shape), atol=1e-12)


@pytest.mark.parametrize("p,q,T", [(3, 8, 11), (2, 3, 9), (1, 2, 4)])
def test_shift_equivariance(p, q, T):
    f = _flt(p, q, T)
    X = synthgen.uniform_frame(8, 4 * q, 6 * q)
    Y = pp.downscale_u8(X, f, f)
    for a in (1, 2):
        Xs = np.roll(np.roll(X, q * a, axis=1), -q, axis=0)
        Ys = np.roll(np.roll(Y, p * a, axis=1), -p, axis=0)
        np.testing.assert_array_equal(pp.downscale_u8(Xs, f, f), Ys)


def test_integer_pass_equals_rounded_float():
    for (p, q, T) in [(3, 8, 11), (2, 3, 16), (1, 2, 8)]:
        f = _flt(p, q, T, seed=T, kind="random")
        X = synthgen.uniform_frame(9, 13, 50)
        yi = pp.polyphase_int_axis(X, f, axis=-1)
        yf = pp.polyphase_f64_axis(X.astype(np.float64), f, axis=-1)
        np.testing.assert_array_equal(yi, np.clip(np.floor(yf + 0.5), 0, 255).astype(np.int64))


# ---------------------------------------------------------------- brute force

@pytest.mark.parametrize("seed", range(8))
def test_interpreter_matches_direct_definition(seed):
    g = synthgen.rng_for(seed, 7)
    p, q = [(3, 8), (1, 2), (2, 3), (4, 9), (1, 1), (3, 5), (5, 3)][seed % 7]
    T = int(g.integers(1, 17))
    H, W = int(g.integers(1, 30)), int(g.integers(1, 40))  # includes N < window span
    c = g.integers(-200, 400, size=(p, T))
    starts = None if seed % 2 == 0 else [int(v) for v in g.integers(-20, 20, size=p)]
    f = pp.Filter(p, q, c, starts)
    X = g.integers(0, 256, size=(H, W)).astype(np.uint8)
    Yi, ch, cv = pp.downscale_u8_interp(X, f, f)
    assert ch.min() == 1 and ch.max() == 1 and cv.min() == 1 and cv.max() == 1
    np.testing.assert_array_equal(Yi, pp.downscale_u8(X, f, f))
    # the per-output loop agrees as well, row by row
    Z = pp.polyphase_int_axis(X, f, axis=-1)
    for y in range(min(H, 3)):
        np.testing.assert_array_equal(pp.polyphase_int_1d(X[y], f), Z[y])


# ---------------------------------------------------------------- float form

@pytest.mark.parametrize("p,q,T", [(3, 8, 11), (2, 3, 16), (4, 9, 6)])
def test_float_dense_equals_gather(p, q, T):
    f = _flt(p, q, T)
    X = synthgen.rng_for(10, T).random((45, 61))
    np.testing.assert_allclose(pp.downscale_f64_dense(X, f, f), pp.downscale_f64(X, f, f), atol=1e-12, rtol=0)


def test_float_linear_and_commuting():
    f = _flt(3, 8, 11)
    v = _flt(2, 3, 10)
    g = synthgen.rng_for(11, 0)
    A, B = g.random((40, 56)), g.random((40, 56))
    Y = lambda X: pp.downscale_f64(X, f, v)  # noqa: E731
    np.testing.assert_allclose(Y(2.5 * A - B), 2.5 * Y(A) - Y(B), atol=1e-12)
    vh = pp.polyphase_f64_axis(pp.polyphase_f64_axis(A, v, axis=-2), f, axis=-1)
    np.testing.assert_allclose(vh, Y(A), atol=1e-12)


def test_dense_matrix_rows_sum_to_one_and_band():
    f = _flt(3, 8, 11)
    D = pp.dense_matrix(64, f)
    np.testing.assert_allclose(D.sum(axis=1), 1.0, atol=1e-15)
    assert ((D != 0).sum(axis=1) <= 11).all()


# ---------------------------------------------------------------- generic repetition

def _tiler(rt):
    return Tiler(rt.array_shape, rt.origin, rt.paving.tolist(), rt.fitting.tolist(), rt.pat_shape)


def _identity_out(rep_shape):
    d = len(rep_shape)
    return Tiler(tuple(rep_shape), (0,) * d, np.eye(d, dtype=np.int64).tolist(), [[] for _ in range(d)], ())


@pytest.mark.parametrize("seed", range(4))
def test_generic_interpreter_matches_vectorised(seed):
    rt = synthgen.random_tiler(seed, array_shape=(5, 7, 6), pat_shape=(3, 2))
    tin = _tiler(rt)
    A = synthgen.rng_for(seed, 1).uniform(-1, 1, size=rt.array_shape).astype(np.float32)
    w = synthgen.rng_for(seed, 2).uniform(-1, 1, size=rt.pat_shape).astype(np.float32)
    tout = _identity_out(rt.rep_shape)
    B, M, cnt = gn.weighted_sum_f64(A, tin, w, tout, rt.rep_shape)
    Bi, cnti = gn.weighted_sum_interp(A, tin, w, tout, rt.rep_shape)
    assert cnt.min() == 1 and cnt.max() == 1 and cnti.min() == 1
    np.testing.assert_allclose(B, Bi, rtol=0, atol=1e-12)


def test_generic_is_circular_correlation_for_identity_tilers():
    g = synthgen.rng_for(12, 0)
    A = g.uniform(-1, 1, size=(9, 11))
    w = g.uniform(-1, 1, size=(3, 5))
    tin = Tiler((9, 11), (0, 0), [[1, 0], [0, 1]], [[1, 0], [0, 1]], (3, 5))
    B, _, _ = gn.weighted_sum_f64(A, tin, w, _identity_out((9, 11)), (9, 11))
    # y[r] = sum_i w[i] A[r + i] (wrapped): correlate with the kernel anchored at its first element
    ref = scipy.ndimage.correlate(A, w, mode="wrap", origin=(-1, -2))
    np.testing.assert_allclose(B, ref, atol=1e-12)


def test_generic_single_tap_is_strided_permuted_gather():
    A = synthgen.rng_for(13, 0).uniform(-1, 1, size=(6, 10))
    # paving swaps axes with stride 2 on the column axis; origin (1, 3)
    tin = Tiler((6, 10), (1, 3), [[0, 1], [2, 0]], [[0], [0]], (1,))
    B, _, cnt = gn.weighted_sum_f64(A, tin, [1.0], _identity_out((5, 6)), (5, 6))
    ref = np.take(np.take(A, 1 + np.arange(6), axis=0, mode="wrap"), 3 + 2 * np.arange(5), axis=1, mode="wrap").T
    np.testing.assert_array_equal(B, ref)
