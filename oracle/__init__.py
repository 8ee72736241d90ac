"""CPU oracle for the Array-OL downscaler -- TEST INFRASTRUCTURE ONLY.

A plain, slow, obviously-correct CPU implementation of what the GPU path
computes, written from the paper (Rodrigues, Guyomarc'h, Dekeyser,
"Programming Massively Parallel Architectures using MARTE: a Case Study"):

* ``arrayol``   -- a literal Array-OL interpreter: tilers built from an
  origin, a paving matrix and a fitting matrix (Sec. III-A, the tiler
  footnote), a repetitive task that runs an elementary task once per point
  of its repetition space and counts the writes to every output element.
* ``polyphase`` -- the downscaler itself (Sec. III: a horizontal filter
  followed by a vertical filter, each interpolating packets of input pixels
  into fewer output pixels), as direct definitions: the integer form with
  uint8 frames, and the float form in float64, both by gather and by dense
  banded matrices.
* ``generic``   -- the general Array-OL repetition with a weighted-sum
  elementary task, in float64.
* ``linear``    -- the general Array-OL repetition on uint8 arrays with a
  linear integer elementary task and multi-element input and output patterns
  (colour conversion between interleaved RGB and planar components, the
  composition of the output frame, non-separable 2-D filters).

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg
may import this package. It shares no code with the GPU library and does
not import it; the GPU library never imports this package.

Readings of the paper where it is silent or garbled are listed in each
function's docstring (coefficients are user data; window placement, rounding,
clamping, the uint8 intermediate, modulo borders, ceil-repetition counts).
Parity status: the integer and float downscaler, the generic weighted sum
and the linear integer repetition are pinned by the not-gpu tests (special cases reducing to library routines,
closed forms, exhaustive invariants, brute force through the interpreter,
and the repetition space and frame sizes the paper prints).
"""

from . import arrayol, polyphase, generic, linear  # noqa: F401
