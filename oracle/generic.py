"""General Array-OL repetition with a weighted-sum elementary task (float64).

Sec. III-A and its tiler footnote: for every point r of the repetition
space the input tiler gathers the pattern elements

    A[(origin + paving . r + fitting . i) mod array_shape],  i in pattern space,

and the elementary task here is a weighted sum over the pattern,
``y = sum_i w[i] * pattern[i]``, written through an output tiler with a
single-element pattern at ``(origin' + paving' . r) mod shape'``.

``weighted_sum_f64`` evaluates the definition for every repetition point
(vectorised over r, one pattern element at a time, accumulating in float64
in pattern order). ``weighted_sum_at`` evaluates selected repetition
points only, for checking samples of very large runs.
"""

from __future__ import annotations

import itertools

import numpy as np

from .arrayol import Tiler, run_repetitive_task


def _rep_grid(rep_shape):
    grids = np.meshgrid(*[np.arange(n, dtype=np.int64) for n in rep_shape], indexing="ij")
    return np.stack([g.ravel() for g in grids], axis=0)  # [rep_rank, |R|]


def _gather_index(t: Tiler, r: np.ndarray, i) -> tuple:
    """Array index tuple for pattern element i at repetition points r ([rep_rank, n])."""
    out = []
    for d, S in enumerate(t.array_shape):
        v = np.full(r.shape[1], t.origin[d], dtype=np.int64)
        for a in range(r.shape[0]):
            if t.paving[d][a]:
                v = v + int(t.paving[d][a]) * r[a]
        for b, ib in enumerate(i):
            v = v + int(t.fitting[d][b]) * int(ib)
        out.append(np.mod(v, S))
    return tuple(out)


def weighted_sum_at(A: np.ndarray, tin: Tiler, w: np.ndarray, r: np.ndarray) -> np.ndarray:
    """y[r] = sum_i w[i] * A[index(r, i)] in float64, for the repetition points ``r`` ([rep_rank, n])."""
    w = np.asarray(w, dtype=np.float64).reshape(tin.pat_shape)
    acc = np.zeros(r.shape[1], np.float64)
    mag = np.zeros(r.shape[1], np.float64)
    for i in itertools.product(*[range(n) for n in tin.pat_shape]):
        v = A[_gather_index(tin, r, i)].astype(np.float64) * w[i]
        acc += v
        mag += np.abs(v)
    return acc, mag


def weighted_sum_f64(A: np.ndarray, tin: Tiler, w, tout: Tiler, rep_shape):
    """Full repetition: returns (B, B_mag, counts) with B the output array.

    ``B_mag[idx] = sum_i |w_i * x_i|`` is the magnitude a float result is
    compared against; ``counts`` is the number of writes per output element
    (a well-formed output tiler writes every element exactly once).
    """
    r = _rep_grid(rep_shape)
    acc, mag = weighted_sum_at(A, tin, w, r)
    B = np.zeros(tout.array_shape, np.float64)
    M = np.zeros(tout.array_shape, np.float64)
    cnt = np.zeros(tout.array_shape, np.int64)
    oidx = _gather_index(tout, r, ())
    B[oidx] = acc
    M[oidx] = mag
    np.add.at(cnt, oidx, 1)
    return B, M, cnt


def weighted_sum_interp(A: np.ndarray, tin: Tiler, w, tout: Tiler, rep_shape):
    """The same repetition through the literal interpreter (tiny inputs only)."""
    wf = [float(v) for v in np.asarray(w, dtype=np.float64).ravel()]

    def task(pattern):
        acc = 0.0
        for wi, xi in zip(wf, pattern):
            acc += wi * float(xi)
        return [[acc]]

    (B,), (cnt,) = run_repetitive_task(rep_shape, [tin], [A], task, [tout], [tout.array_shape])
    return B.astype(np.float64), cnt
