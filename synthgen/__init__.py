"""Seeded synthetic inputs for the Array-OL downscaler and the generic tiler.

This module is shared by the CPU oracle and the GPU path's tests and
benchmarks. It only *draws* inputs: frames, filter taps, stream mixes and
random tilers. It holds none of the downscaling or tiling arithmetic
itself; the taps it designs are ordinary user data that both sides receive
as input.

Every generator takes an integer seed and an index and draws from
``numpy.random.default_rng([seed, idx])`` so that any single frame, stream
or tiler can be regenerated on its own.

Workload recipes (the paper's CIF test video is not available, so these
stand in for it; shapes follow the paper's frames and the benchmark
configurations):

* ``uniform_frame``   -- uniform random uint8 grayscale frame.
* ``gradient_plane``  -- smooth random gradient plus uniform noise:
  ``clip(64 + 127*(0.5 + 0.5*sin(2*pi*(fx*x/W + fy*y/H) + theta)) + U{-16..16}, 0, 255)``
  with ``fx, fy ~ U[0.5, 3]`` and ``theta ~ U[0, 2*pi)`` per plane.
* ``yuv420_frames``   -- a sequence of planar I420 frames built from
  ``gradient_plane`` (luma H x W, two chroma planes H/2 x W/2).
* ``stream_mix``      -- per-stream draws of frame size, ratio and tap count.
* ``design_taps``     -- windowed-sinc interpolation taps quantised to
  integers summing to 256 per phase.
* ``random_tiler``    -- a random non-identity affine tiler (paving with a
  signed permutation, strides and a shear; fitting with strided and
  transposed axes) for the generic weighted-sum task.
"""

from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = [
    "rng_for",
    "uniform_frame",
    "gradient_plane",
    "yuv420_frames",
    "bf16_round",
    "fp16_round",
    "normalised",
    "design_taps",
    "StreamSpec",
    "stream_mix",
    "RandomTiler",
    "random_tiler",
    "SIZES",
    "RATIOS",
]


def rng_for(seed: int, idx: int = 0) -> np.random.Generator:
    """The generator every draw uses: ``default_rng([seed, idx])``."""
    return np.random.default_rng([int(seed), int(idx)])


# --------------------------------------------------------------------------
# frames
# --------------------------------------------------------------------------

def uniform_frame(seed: int, h: int, w: int, idx: int = 0) -> np.ndarray:
    """Uniform random uint8 frame of shape [h, w] (row-major)."""
    return rng_for(seed, idx).integers(0, 256, size=(h, w), dtype=np.uint8)


def gradient_plane(rng: np.random.Generator, h: int, w: int) -> np.ndarray:
    """Smooth random gradient plus uniform integer noise, uint8 [h, w]."""
    fx = rng.uniform(0.5, 3.0)
    fy = rng.uniform(0.5, 3.0)
    theta = rng.uniform(0.0, 2.0 * math.pi)
    x = np.arange(w, dtype=np.float32)[None, :] * np.float32(fx / w)
    y = np.arange(h, dtype=np.float32)[:, None] * np.float32(fy / h)
    base = 64.0 + 127.0 * (0.5 + 0.5 * np.sin(np.float32(2.0 * math.pi) * (x + y) + np.float32(theta)))
    noise = rng.integers(-16, 17, size=(h, w), dtype=np.int16)
    return np.clip(np.floor(base).astype(np.int16) + noise, 0, 255).astype(np.uint8)


def yuv420_frames(seed: int, n_frames: int, h: int = 1080, w: int = 1920, first: int = 0):
    """Planar I420 sequence: returns (Y[n,h,w], U[n,ch,cw], V[n,ch,cw]) uint8.

    Chroma planes are ceil(h/2) x ceil(w/2). Frame ``first + f`` draws from
    ``rng_for(seed, first + f)`` so any frame can be regenerated alone.
    """
    ch, cw = (h + 1) // 2, (w + 1) // 2
    Y = np.empty((n_frames, h, w), np.uint8)
    U = np.empty((n_frames, ch, cw), np.uint8)
    V = np.empty((n_frames, ch, cw), np.uint8)
    for f in range(n_frames):
        g = rng_for(seed, first + f)
        Y[f] = gradient_plane(g, h, w)
        U[f] = gradient_plane(g, ch, cw)
        V[f] = gradient_plane(g, ch, cw)
    return Y, U, V


def bf16_round(x: np.ndarray) -> np.ndarray:
    """Round float32 values to bfloat16 (nearest-even); returns the uint16 bit patterns."""
    b = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32)
    lsb = (b >> 16) & 1
    r = (b + np.uint32(0x7FFF) + lsb) >> 16
    return r.astype(np.uint16)


def fp16_round(x: np.ndarray) -> np.ndarray:
    """Round to IEEE half (nearest-even); returns the uint16 bit patterns."""
    return np.ascontiguousarray(x, dtype=np.float32).astype(np.float16).view(np.uint16)


def normalised(frames_u8: np.ndarray, fmt: str) -> np.ndarray:
    """Normalised pixels k/255 stored as bf16 or fp16 bit patterns (uint16)."""
    x = frames_u8.astype(np.float64) / 255.0
    if fmt == "bf16":
        return bf16_round(x.astype(np.float32))  # k/255 in f32 then RNE to bf16
    if fmt == "fp16":
        return x.astype(np.float16).view(np.uint16)
    raise ValueError(fmt)


# --------------------------------------------------------------------------
# filter taps
# --------------------------------------------------------------------------

def _sinc(t: np.ndarray) -> np.ndarray:
    return np.sinc(t)  # sin(pi t)/(pi t)


def design_taps(p: int, q: int, taps: int, starts=None) -> np.ndarray:
    """Integer interpolation taps ``c[p][taps]`` (int16), each phase summing to 256.

    Filter design for a p/q resampler: output pixel ``phi`` (of each group of
    p) is centred at input coordinate ``u = ((2*phi+1)*q - p) / (2*p)`` in
    pixel-index units. Its taps sit at ``start + k``; by default ``start`` is
    ``floor(u) - floor((taps-1)/2)`` unless the caller passes ``starts``.
    The prototype is a band-limited sinc with cut-off ``min(1, p/q)`` under a
    sinc (Lanczos-style) window of half-width ``taps/2``; each phase is
    normalised to sum 1 in float64, scaled by 256 and rounded, and the
    residual to 256 goes to the taps with the largest rounding remainders
    (ties to the lowest index).
    """
    fc = min(1.0, p / q)
    out = np.zeros((p, taps), np.int16)
    half = taps / 2.0
    for phi in range(p):
        num = (2 * phi + 1) * q - p
        u = num / (2.0 * p)
        s = (num // (2 * p)) - (taps - 1) // 2 if starts is None else int(starts[phi])
        t = (s + np.arange(taps, dtype=np.float64)) - u
        h = fc * _sinc(fc * t) * _sinc(t / half)
        h[np.abs(t) >= half] = 0.0
        if h.sum() == 0.0:
            h[np.argmin(np.abs(t))] = 1.0
        h = h / h.sum()
        scaled = 256.0 * h
        base = np.floor(scaled)
        rem = scaled - base
        c = base.astype(np.int64)
        deficit = 256 - int(c.sum())
        order = sorted(range(taps), key=lambda k: (-rem[k], k))
        for j in range(abs(deficit)):
            k = order[j % taps] if deficit > 0 else order[::-1][j % taps]
            c[k] += 1 if deficit > 0 else -1
        out[phi] = c
    return out


# --------------------------------------------------------------------------
# batched streams
# --------------------------------------------------------------------------

SIZES = [(480, 640), (720, 1280), (1080, 1920), (2160, 3840)]  # (h, w)
RATIOS = [(3, 8), (1, 2), (2, 3)]  # (p, q)


@dataclass
class StreamSpec:
    h: int
    w: int
    p: int
    q: int
    taps: int


def stream_mix(seed: int, n_streams: int = 64) -> list:
    """Per stream: size uniform over SIZES, ratio uniform over RATIOS, taps uniform over 8..16."""
    g = rng_for(seed, 0)
    out = []
    for _ in range(n_streams):
        h, w = SIZES[int(g.integers(0, len(SIZES)))]
        p, q = RATIOS[int(g.integers(0, len(RATIOS)))]
        t = int(g.integers(8, 17))
        out.append(StreamSpec(h, w, p, q, t))
    return out


# --------------------------------------------------------------------------
# random tilers for the generic weighted-sum repetition
# --------------------------------------------------------------------------

@dataclass
class RandomTiler:
    array_shape: tuple
    rep_shape: tuple
    pat_shape: tuple
    origin: tuple
    paving: np.ndarray   # [array_rank, rep_rank]
    fitting: np.ndarray  # [array_rank, pat_rank]


def random_tiler(seed: int, array_shape=(64, 1024, 1024), pat_shape=(5, 5), idx: int = 0) -> RandomTiler:
    """Random non-identity tiler.

    Paving ``= Pi * diag(s)`` plus one off-diagonal shear entry in {0, 1},
    where Pi is a signed permutation and ``s`` in {1, 2}^d. Fitting puts
    column b on a distinct array axis with signed step ``t`` in {1, 2, 3}
    (axis order drawn at random, so it is often transposed). The origin is
    uniform in the array. The repetition space is
    ``R_k = ceil(S[pi(k)] / s_k)`` so each paving column sweeps its axis.
    """
    g = rng_for(seed, idx)
    S = tuple(int(v) for v in array_shape)
    d = len(S)
    perm = g.permutation(d)
    signs = g.choice([-1, 1], size=d)
    strides = g.integers(1, 3, size=d)
    P = np.zeros((d, d), np.int64)
    for k in range(d):
        P[perm[k], k] = signs[k] * strides[k]
    if d > 1:
        a, b = g.choice(d, size=2, replace=False)
        k = int(b)
        row = int(perm[int(a)])
        if P[row, k] == 0:
            P[row, k] = int(g.integers(0, 2))
    pr = len(pat_shape)
    axes = g.choice(d, size=pr, replace=False)
    F = np.zeros((d, pr), np.int64)
    for b in range(pr):
        F[axes[b], b] = int(g.choice([-1, 1])) * int(g.integers(1, 4))
    origin = tuple(int(g.integers(0, S[a])) for a in range(d))
    R = tuple(int(-(-S[perm[k]] // int(strides[k]))) for k in range(d))
    return RandomTiler(S, R, tuple(int(v) for v in pat_shape), origin, P, F)


# --------------------------------------------------------------------------
# linear integer tasks: tiler specifications and caller weights
# --------------------------------------------------------------------------

@dataclass
class TilerSpec:
    array_shape: tuple
    origin: tuple
    paving: list      # [array dim][rep dim]
    fitting: list     # [array dim][pattern dim]
    pat_shape: tuple


def rgb_to_planar_tilers(h: int, w: int):
    """Interleaved RGB [h, 3w] to planar [3, h, w]: repetition space (h, w); the input pattern is
    the three adjacent bytes of a pixel (paving 3 along the row, fitting 1), the output pattern
    one byte in each plane. Returns (rep_shape, tin, tout)."""
    tin = TilerSpec((h, 3 * w), (0, 0), [[1, 0], [0, 3]], [[0], [1]], (3,))
    tout = TilerSpec((3, h, w), (0, 0, 0), [[0, 0], [1, 0], [0, 1]], [[1], [0], [0]], (3,))
    return (h, w), tin, tout


def planar_to_rgb_tilers(h: int, w: int):
    """Planar [3, h, w] back to interleaved RGB [h, 3w] (the composition of the frame)."""
    tin = TilerSpec((3, h, w), (0, 0, 0), [[0, 0], [1, 0], [0, 1]], [[1], [0], [0]], (3,))
    tout = TilerSpec((h, 3 * w), (0, 0), [[1, 0], [0, 3]], [[0], [1]], (3,))
    return (h, w), tin, tout


# Caller weights of the colour conversions, scaled by 256 (full-range BT.601
# approximations; rows of the RGB->YCbCr matrix sum to 256 for luma and 0 for
# chroma, the chroma offset 128 is the bias 128*256).
RGB_TO_YCC_W = np.array([[77, 150, 29], [-43, -85, 128], [128, -107, -21]], np.int16)
RGB_TO_YCC_BIAS = np.array([0, 128 * 256, 128 * 256], np.int32)
YCC_TO_RGB_W = np.array([[256, 0, 359], [256, -88, -183], [256, 454, 0]], np.int16)
YCC_TO_RGB_BIAS = np.array([-359 * 128, (88 + 183) * 128, -454 * 128], np.int32)


def polyphase2d_tilers(h: int, w: int, p: int, q: int, taps: int):
    """Non-separable 2-D polyphase filter as one repetition per q x q packet: the input
    pattern is the union window (span x span) of the p phases along each axis, the output
    pattern the p x p outputs of the packet. Window starts: the default pixel-centre
    placement. Returns (rep_shape, tin, tout, starts, span)."""
    starts = [((2 * phi + 1) * q - p) // (2 * p) - (taps - 1) // 2 for phi in range(p)]
    lo = min(starts)
    span = max(s + taps for s in starts) - lo
    ry, rx = -(-h // q), -(-w // q)
    tin = TilerSpec((h, w), (lo, lo), [[q, 0], [0, q]], [[1, 0], [0, 1]], (span, span))
    tout = TilerSpec((p * ry, p * rx), (0, 0), [[p, 0], [0, p]], [[1, 0], [0, 1]], (p, p))
    return (ry, rx), tin, tout, starts, span


def polyphase2d_weights(seed: int, p: int, q: int, taps: int):
    """Caller weights W[p*p][span*span] of a non-separable 2-D polyphase filter: for output
    phase (py, px) a taps x taps kernel (the outer product of the 1-D design plus a seeded
    random non-separable part, rounded so each kernel sums to 256) placed in the union window."""
    _, _, _, starts, span = polyphase2d_tilers(q, q, p, q, taps)
    lo = min(starts)
    c = design_taps(p, q, taps).astype(np.float64) / 256.0
    g = rng_for(seed, 7)
    W = np.zeros((p * p, span * span), np.int64)
    for py in range(p):
        for px in range(p):
            k = np.outer(c[py], c[px]) + 0.02 * g.standard_normal((taps, taps))
            k = 256.0 * k / k.sum()
            base = np.floor(k)
            rem = (k - base).ravel()
            ki = base.astype(np.int64).ravel()
            order = sorted(range(ki.size), key=lambda t: (-rem[t], t))
            for t in range(256 - int(ki.sum())):
                ki[order[t % ki.size]] += 1
            ki = ki.reshape(taps, taps)
            oy, ox = starts[py] - lo, starts[px] - lo
            full = np.zeros((span, span), np.int64)
            full[oy:oy + taps, ox:ox + taps] = ki
            W[py * p + px] = full.ravel()
    return W.astype(np.int16)
