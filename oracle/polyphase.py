"""The downscaler as direct definitions (integer and float64).

Sec. III: the downscaler is a horizontal filter (352 -> 132 pixels per line
in the paper's CIF case) followed by a vertical filter (288 -> 128 lines),
each interpolating packets of 8 input pixels. Sec. III-A: the horizontal
task ``yhfk`` has multiplicity [288, 44], i.e. one elementary task per
(line, 8-pixel packet), each taking its pattern through a tiler.

Notation (one axis of length N):
  * ratio p/q: each repetition consumes a packet of q input pixels and
    emits p output pixels (the paper's 3 outputs per 8-pixel packet for
    352 -> 132 is p/q = 3/8);
  * R = ceil(N / q) repetitions, M = p * R outputs;
  * output o belongs to repetition r = o // p and phase phi = o % p;
  * taps c[phi][k], k < T, integer weights;
  * window start s_phi relative to q*r.

Readings where the paper is silent (it gives no coefficients, tap count,
border rule or rounding):
  * coefficients are caller data;
  * default window start: the output pixel of phase phi is centred at input
    coordinate u = ((2*phi+1)*q - p) / (2*p) (pixel centres at integers) and
    the T-tap window starts at floor(u) - floor((T-1)/2);
  * borders wrap modulo N (Array-OL tiler semantics);
  * integer output: floor((acc + 128) / 256), then clamp to 0..255;
  * the horizontal result is quantised to uint8 before the vertical filter
    (the two filters are separate components exchanging a frame array);
  * the float form uses weights c/256, no rounding and no clamp.
"""

from __future__ import annotations

import numpy as np

from .arrayol import Tiler, run_repetitive_task


# --------------------------------------------------------------------------
# geometry
# --------------------------------------------------------------------------

def default_phase_starts(p: int, q: int, taps: int) -> list:
    """Window start s_phi for each phase (exact integer arithmetic).

    The centre of output phase phi in input-index units is
    ((2*phi+1)*q - p) / (2*p); its floor minus floor((T-1)/2) starts a
    T-tap window around it.
    """
    return [((2 * phi + 1) * q - p) // (2 * p) - (taps - 1) // 2 for phi in range(p)]


def repetitions(n: int, q: int) -> int:
    """R = ceil(n / q): every repetition is a full packet, wrapping mod n."""
    return -(-n // q)


def output_length(n: int, p: int, q: int) -> int:
    return p * repetitions(n, q)


class Filter:
    """One axis' polyphase filter: ratio p/q, taps c[p][T], window starts s[p]."""

    def __init__(self, p, q, coeff, starts=None):
        self.p, self.q = int(p), int(q)
        self.c = np.asarray(coeff, dtype=np.int64).reshape(self.p, -1)
        self.T = self.c.shape[1]
        self.s = list(default_phase_starts(self.p, self.q, self.T) if starts is None else [int(v) for v in starts])


# --------------------------------------------------------------------------
# integer form
# --------------------------------------------------------------------------

def _round_clamp(acc):
    """floor((acc + 128) / 256) clamped to 0..255 (numpy int64 arrays or ints)."""
    return np.clip((np.asarray(acc, dtype=np.int64) + 128) // 256, 0, 255)


def polyphase_int_1d(x, f: Filter) -> np.ndarray:
    """One integer pass over a 1-D signal, with a Python loop per output."""
    x = [int(v) for v in x]
    n = len(x)
    m = output_length(n, f.p, f.q)
    y = np.zeros(m, np.int64)
    for o in range(m):
        r, phi = divmod(o, f.p)
        acc = 0
        for k in range(f.T):
            acc += int(f.c[phi, k]) * x[(f.q * r + f.s[phi] + k) % n]
        y[o] = min(255, max(0, (acc + 128) // 256))
    return y


def _gather_tables(n: int, f: Filter):
    """idx[o, k] = (q*r + s_phi + k) mod n and w[o, k] = c[phi][k] for every output o."""
    m = output_length(n, f.p, f.q)
    o = np.arange(m)
    r, phi = o // f.p, o % f.p
    start = f.q * r + np.asarray(f.s, dtype=np.int64)[phi]
    idx = np.mod(start[:, None] + np.arange(f.T)[None, :], n)
    w = f.c[phi]
    return idx, w


def polyphase_int_axis(x: np.ndarray, f: Filter, axis: int) -> np.ndarray:
    """Integer pass along ``axis`` of an integer array (vectorised gather, int64 accumulate)."""
    x = np.moveaxis(np.asarray(x, dtype=np.int64), axis, -1)
    idx, w = _gather_tables(x.shape[-1], f)
    acc = (x[..., idx] * w).sum(axis=-1)
    return np.moveaxis(_round_clamp(acc), -1, axis)


def downscale_u8(X: np.ndarray, hf: Filter, vf: Filter) -> np.ndarray:
    """Integer frame downscale: horizontal pass over every line, then vertical pass over every column.

    ``X`` is uint8 [..., H, W]; returns uint8 [..., M_h, M_w].
    """
    Z = polyphase_int_axis(X, hf, axis=-1).astype(np.uint8)  # uint8 intermediate frame
    Y = polyphase_int_axis(Z, vf, axis=-2)
    return Y.astype(np.uint8)


# --------------------------------------------------------------------------
# the same passes as Array-OL repetitive tasks (interpreter)
# --------------------------------------------------------------------------

def _span(f: Filter):
    lo = min(f.s)
    hi = max(s + f.T for s in f.s)
    return lo, hi - lo


def _elementary(f: Filter, lo: int):
    def task(pattern):
        out = []
        for phi in range(f.p):
            acc = 0
            for k in range(f.T):
                acc += int(f.c[phi, k]) * int(pattern[f.s[phi] - lo + k])
            out.append(min(255, max(0, (acc + 128) // 256)))
        return [out]
    return task


def hfilter_task(X: np.ndarray, f: Filter):
    """Horizontal filter as a repetitive task with multiplicity [H, ceil(W/q)].

    Input tiler: origin (0, s_min), paving [[1,0],[0,q]], fitting [[0],[1]],
    pattern [span]. Output tiler on the [H, p*R] array: paving [[1,0],[0,p]],
    fitting [[0],[1]], pattern [p]. Returns (Z, counts, repetition_space).
    """
    H, W = X.shape
    lo, span = _span(f)
    R = repetitions(W, f.q)
    tin = Tiler((H, W), (0, lo), [[1, 0], [0, f.q]], [[0], [1]], (span,))
    tout = Tiler((H, f.p * R), (0, 0), [[1, 0], [0, f.p]], [[0], [1]], (f.p,))
    (Z,), (cnt,) = run_repetitive_task((H, R), [tin], [X], _elementary(f, lo), [tout], [(H, f.p * R)])
    return Z.astype(np.int64), cnt, (H, R)


def vfilter_task(Z: np.ndarray, f: Filter):
    """Vertical filter as a repetitive task with multiplicity [ceil(H/q), W'].

    Input tiler: origin (s_min, 0), paving [[q,0],[0,1]], fitting [[1],[0]].
    Output tiler: paving [[p,0],[0,1]], fitting [[1],[0]], pattern [p].
    """
    H, W = Z.shape
    lo, span = _span(f)
    R = repetitions(H, f.q)
    tin = Tiler((H, W), (lo, 0), [[f.q, 0], [0, 1]], [[1], [0]], (span,))
    tout = Tiler((f.p * R, W), (0, 0), [[f.p, 0], [0, 1]], [[1], [0]], (f.p,))
    (Y,), (cnt,) = run_repetitive_task((R, W), [tin], [Z], _elementary(f, lo), [tout], [(f.p * R, W)])
    return Y.astype(np.int64), cnt, (R, W)


def downscale_u8_interp(X: np.ndarray, hf: Filter, vf: Filter):
    """The integer downscale through the interpreter; returns (Y, counts_h, counts_v)."""
    Z, ch, _ = hfilter_task(np.asarray(X), hf)
    Y, cv, _ = vfilter_task(Z, vf)
    return Y.astype(np.uint8), ch, cv


# --------------------------------------------------------------------------
# float64 form
# --------------------------------------------------------------------------

def polyphase_f64_axis(x: np.ndarray, f: Filter, axis: int) -> np.ndarray:
    """Float64 pass along ``axis``: sum_k (c[phi][k]/256) * x[(q r + s_phi + k) mod n]."""
    x = np.moveaxis(np.asarray(x, dtype=np.float64), axis, -1)
    idx, w = _gather_tables(x.shape[-1], f)
    y = (x[..., idx] * (w.astype(np.float64) / 256.0)).sum(axis=-1)
    return np.moveaxis(y, -1, axis)


def downscale_f64(X: np.ndarray, hf: Filter, vf: Filter) -> np.ndarray:
    """Float64 frame downscale (gather form): horizontal then vertical, no rounding, no clamp."""
    return polyphase_f64_axis(polyphase_f64_axis(X, hf, axis=-1), vf, axis=-2)


def dense_matrix(n: int, f: Filter) -> np.ndarray:
    """D[o, (q r + s_phi + k) mod n] += c[phi][k] / 256: the banded, circulant-wrapped filter matrix."""
    m = output_length(n, f.p, f.q)
    D = np.zeros((m, n), np.float64)
    for o in range(m):
        r, phi = divmod(o, f.p)
        for k in range(f.T):
            D[o, (f.q * r + f.s[phi] + k) % n] += f.c[phi, k] / 256.0
    return D


def downscale_f64_dense(X: np.ndarray, hf: Filter, vf: Filter) -> np.ndarray:
    """Float64 frame downscale as Y = D_v X D_h^T (one frame [H, W])."""
    H, W = X.shape
    return dense_matrix(H, vf) @ np.asarray(X, np.float64) @ dense_matrix(W, hf).T
