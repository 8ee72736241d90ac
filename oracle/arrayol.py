"""Literal Array-OL interpreter (pure Python loops; tiny inputs only).

Sec. III-A: a repetitive task has a multiplicity (its repetition space);
each point of that space runs one independent elementary task, which takes
a pattern from the input array through a tiler described by an origin, a
paving and a fitting. Array-OL (the tiler footnote) defines the element
``i`` of the pattern taken at repetition ``r`` as

    index(r, i) = (origin + paving . r + fitting . i)  mod  array_shape

component-wise, with a mathematical (non-negative) modulus so that patterns
wrap around the array borders. Output patterns are written back through an
output tiler in the same way.

Nothing here is vectorised or reordered: the loops follow the definition.
"""

from __future__ import annotations

import itertools
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Tiler:
    """An Array-OL tiler.

    ``paving`` is array_rank x rep_rank and ``fitting`` is array_rank x
    pat_rank, stored as nested lists of ints. A pattern of rank 0 (``pat_shape
    == ()``) is a single element.
    """

    array_shape: tuple
    origin: tuple
    paving: list
    fitting: list
    pat_shape: tuple = field(default=())

    def index(self, r, i):
        """Array index of pattern element ``i`` at repetition ``r``."""
        out = []
        for d, S in enumerate(self.array_shape):
            v = self.origin[d]
            for a, ra in enumerate(r):
                v += self.paving[d][a] * ra
            for b, ib in enumerate(i):
                v += self.fitting[d][b] * ib
            out.append(v % S)  # Python % is the non-negative modulus for S > 0
        return tuple(out)


def _points(shape):
    return itertools.product(*[range(int(n)) for n in shape])


def run_repetitive_task(rep_shape, in_tilers, in_arrays, task, out_tilers, out_shapes, out_dtype=object):
    """Run ``task`` once per repetition point.

    ``task`` receives one pattern per input (a nested list shaped like the
    tiler's pattern, flattened row-major into a Python list) and returns one
    flat list per output pattern. Returns ``(outputs, counts)`` where
    ``counts[j]`` holds how many times each element of output ``j`` was
    written; the repetition is well formed when every count is exactly 1.
    """
    outs = [np.zeros(s, dtype=out_dtype) for s in out_shapes]
    counts = [np.zeros(s, dtype=np.int64) for s in out_shapes]
    for r in _points(rep_shape):
        pats = []
        for t, arr in zip(in_tilers, in_arrays):
            pats.append([arr[t.index(r, i)] for i in _points(t.pat_shape)])
        results = task(*pats)
        for t, res, o, c in zip(out_tilers, results, outs, counts):
            elems = list(_points(t.pat_shape))
            assert len(res) == len(elems)
            for i, v in zip(elems, res):
                idx = t.index(r, i)
                o[idx] = v
                c[idx] += 1
    return outs, counts
