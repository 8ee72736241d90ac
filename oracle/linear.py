"""Array-OL repetition with a linear integer elementary task (uint8 arrays).

Sec. III: the application reads 24-bit RGB frames, filters colour
components and produces the output frame from the colour-space results;
Sec. III-A: every such step is a repetitive task whose elementary task takes
one pattern through an input tiler and gives one pattern through an output
tiler. Here the elementary task is linear with integer weights. For every
point r of the repetition space:

    x[i] = A[(o + P.r + F.i) mod S]                      i over the input pattern
    y[j] = clamp(floor((sum_i W[j][i] x[i] + bias[j] + 128) / 256), 0, 255)
    B[(o' + P'.r + F'.j) mod S'] = y[j]                  j over the output pattern

(patterns flattened row-major). With a pattern of three adjacent bytes this
is a conversion between interleaved RGB and planar colour components (and
back, with an interleaving output tiler); with a T x T input pattern and a
p x p output pattern it is a non-separable 2-D filter with several outputs
per repetition, e.g. a 2-D polyphase downscale. The rounding follows the
downscaler's reading (add 128, floor-divide by 256, then clamp); the weights
are caller data.

``linear_u8`` evaluates the definition for all repetition points at once,
one pattern element at a time, in exact integer arithmetic;
``linear_u8_interp`` runs the literal interpreter (tiny inputs only).
TEST INFRASTRUCTURE ONLY (see the package docstring).
"""

from __future__ import annotations

import itertools

import numpy as np

from .arrayol import Tiler, run_repetitive_task
from .generic import _gather_index, _rep_grid


def _pattern_points(pat_shape):
    return list(itertools.product(*[range(int(n)) for n in pat_shape]))


def _quantise(acc):
    """floor((acc + 128) / 256) clamped to 0..255 (acc: exact integers)."""
    return np.clip(np.floor_divide(acc + 128, 256), 0, 255)


def linear_u8(A: np.ndarray, tin: Tiler, W, bias, tout: Tiler, rep_shape):
    """All repetitions of the linear task. Returns (B, counts): the uint8 output array of
    shape ``tout.array_shape`` (elements never written stay 0) and the write count of
    every output element (a well-formed output tiler writes each exactly once)."""
    ins = _pattern_points(tin.pat_shape)
    outs = _pattern_points(tout.pat_shape)
    W = np.asarray(W, dtype=np.int64).reshape(len(outs), len(ins))
    bias = np.zeros(len(outs), np.int64) if bias is None else np.asarray(bias, dtype=np.int64).reshape(len(outs))
    r = _rep_grid(rep_shape)
    x = [A[_gather_index(tin, r, i)].astype(np.int64) for i in ins]  # one gather per pattern element
    B = np.zeros(tout.array_shape, np.uint8)
    cnt = np.zeros(tout.array_shape, np.int64)
    for j, jj in enumerate(outs):
        acc = np.full(r.shape[1], bias[j], np.int64)
        for i in range(len(ins)):
            if W[j, i]:
                acc += W[j, i] * x[i]
        idx = _gather_index(tout, r, jj)
        B[idx] = _quantise(acc).astype(np.uint8)
        np.add.at(cnt, idx, 1)
    return B, cnt


def linear_u8_interp(A: np.ndarray, tin: Tiler, W, bias, tout: Tiler, rep_shape):
    """The same repetition through the literal interpreter; returns (B, counts)."""
    n_in = len(_pattern_points(tin.pat_shape))
    n_out = len(_pattern_points(tout.pat_shape))
    Wl = [[int(v) for v in row] for row in np.asarray(W, dtype=np.int64).reshape(n_out, n_in)]
    bl = [0] * n_out if bias is None else [int(v) for v in np.asarray(bias).ravel()]

    def task(pattern):
        out = []
        for j in range(n_out):
            acc = bl[j]
            for i in range(n_in):
                acc += Wl[j][i] * int(pattern[i])
            out.append(min(255, max(0, (acc + 128) // 256)))
        return [out]

    (B,), (cnt,) = run_repetitive_task(rep_shape, [tin], [A], task, [tout], [tout.array_shape])
    return B.astype(np.uint8), cnt
