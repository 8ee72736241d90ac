"""The pins must catch plausible mistakes: each case plants one mistake in the
oracle (on the CPU, by patching) and checks that at least one pin fails."""

import numpy as np
import pytest

from oracle import polyphase as pp
from oracle import generic as gn
import tests.test_oracle_pins as pins


def _fails(fn, *args):
    try:
        fn(*args)
    except AssertionError:
        return True
    return False


def test_dropped_rounding_term_is_caught(monkeypatch):
    monkeypatch.setattr(pp, "_round_clamp", lambda acc: np.clip(np.asarray(acc, np.int64) // 256, 0, 255))
    assert _fails(pins.test_two_tap_average_rounds_half_up)


def test_missing_clamp_is_caught(monkeypatch):
    monkeypatch.setattr(pp, "_round_clamp", lambda acc: (np.asarray(acc, np.int64) + 128) // 256)
    assert _fails(pins.test_extrapolating_taps_clamp)


def test_window_start_off_by_one_is_caught(monkeypatch):
    orig = pp.default_phase_starts
    monkeypatch.setattr(pp, "default_phase_starts", lambda p, q, T: [s + 1 for s in orig(p, q, T)])
    assert _fails(pins.test_identity_filter) or _fails(pins.test_default_phase_starts_known_values)


def test_wrong_repetition_count_is_caught(monkeypatch):
    monkeypatch.setattr(pp, "repetitions", lambda n, q: n // q)  # floor instead of ceil
    assert _fails(pins.test_paper_cif_shapes_through_interpreter) or _fails(pins.test_identity_filter)


def test_reversed_taps_are_caught(monkeypatch):
    orig = pp._gather_tables

    def flipped(n, f):
        idx, w = orig(n, f)
        return idx, w[:, ::-1]

    monkeypatch.setattr(pp, "_gather_tables", flipped)
    assert _fails(pins.test_extrapolating_taps_clamp)


def test_truncating_modulus_is_caught(monkeypatch):
    orig = pp._gather_tables

    def trunc(n, f):
        m = pp.output_length(n, f.p, f.q)
        o = np.arange(m)
        r, phi = o // f.p, o % f.p
        start = f.q * r + np.asarray(f.s, dtype=np.int64)[phi]
        raw = start[:, None] + np.arange(f.T)[None, :]
        idx = np.fmod(raw, n)  # C-style remainder: negative for the left border
        idx = np.where(idx < 0, 0, idx)  # a typical "fix" that clamps instead of wrapping
        return idx, f.c[phi]

    monkeypatch.setattr(pp, "_gather_tables", trunc)
    assert _fails(pins.test_decimation_equals_take_wrap, 8, 11, 5) or _fails(pins.test_shifted_delta_equals_roll)


def test_transposed_dense_matrix_is_caught(monkeypatch):
    monkeypatch.setattr(pp, "downscale_f64_dense",
                        lambda X, hf, vf: pp.dense_matrix(X.shape[0], vf) @ np.asarray(X, np.float64) @ pp.dense_matrix(X.shape[1], hf).T[::-1])
    assert _fails(pins.test_float_dense_equals_gather, 3, 8, 11)


def test_generic_sign_error_is_caught(monkeypatch):
    orig = gn._gather_index

    def minus(t, r, i):
        out = list(orig(t, r, ()))
        # fitting applied with the wrong sign
        for d, S in enumerate(t.array_shape):
            off = sum(int(t.fitting[d][b]) * int(ib) for b, ib in enumerate(i))
            out[d] = np.mod(out[d] - off, S)
        return tuple(out)

    monkeypatch.setattr(gn, "_gather_index", minus)
    assert _fails(pins.test_generic_is_circular_correlation_for_identity_tilers)
