"""Python binding of ``libaolmi.so``: Array-OL repetitive tasks on MI355X.

A thin ctypes layer over the C ABI declared in ``include/aolmi.h``. Functions
named ``aol_*`` mirror the C entry points one to one (argument marshalling
only); ``DownscalePlan`` and ``WeightedSumPlan`` wrap them for torch tensors.
PyTorch is used only for device memory and streams: tensors are passed as
``data_ptr()`` and ``torch.cuda.current_stream().cuda_stream``; every step
of the computation runs in the library's HIP kernels.

The library must be built (``python paper_1103_4881_amd/build.py``); when it
is missing, importing this package raises ``ImportError``. There is no CPU
fallback.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libaolmi.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run `python paper_1103_4881_amd/build.py`")

# torch carries its own HIP runtime under the same soname as ROCm's
# (libamdhip64.so.7). Loading torch first makes the library bind to that one
# runtime, so torch's streams and allocations are valid handles for it.
import torch  # noqa: E402,F401

_lib = ctypes.CDLL(LIB_PATH)

AOL_OK = 0
AOL_ERR_INVALID = -1
AOL_ERR_UNSUPPORTED = -2
AOL_ERR_NOMEM = -3
AOL_ERR_HIP = -4

AOL_PREC_U8 = 0
AOL_PREC_BF16 = 1
AOL_PREC_FP16 = 2
_PREC = {"u8": AOL_PREC_U8, "bf16": AOL_PREC_BF16, "fp16": AOL_PREC_FP16}

AOL_MAX_RANK = 4


class AolError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"aol status {status}: {msg}")
        self.status = status
        self.msg = msg


c_i32p = ctypes.POINTER(ctypes.c_int32)
c_i64p = ctypes.POINTER(ctypes.c_int64)
c_i16p = ctypes.POINTER(ctypes.c_int16)


class aol_polyphase(ctypes.Structure):
    _fields_ = [("p", ctypes.c_int32), ("q", ctypes.c_int32), ("taps", ctypes.c_int32),
                ("coeff", c_i16p), ("phase_start", c_i32p)]


class aol_plane_desc(ctypes.Structure):
    _fields_ = [("height", ctypes.c_int64), ("width", ctypes.c_int64),
                ("in_pitch", ctypes.c_int64), ("out_pitch", ctypes.c_int64)]


def _proto(name, restype, *args):
    f = getattr(_lib, name)
    f.restype = restype
    f.argtypes = list(args)
    return f


_lib.aol_last_error.restype = ctypes.c_char_p
_lib.aol_version.restype = ctypes.c_char_p
_proto("aol_default_phase_starts", ctypes.c_int, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, c_i32p)
_proto("aol_downscale_output_shape", ctypes.c_int, ctypes.c_int64, ctypes.c_int64,
       ctypes.POINTER(aol_polyphase), ctypes.POINTER(aol_polyphase), c_i64p, c_i64p)
_proto("aol_downscale_plan_create", ctypes.c_int, ctypes.POINTER(aol_plane_desc), ctypes.c_int32,
       ctypes.POINTER(aol_polyphase), ctypes.POINTER(aol_polyphase), ctypes.c_int, ctypes.POINTER(ctypes.c_void_p))
_proto("aol_plan_destroy", ctypes.c_int, ctypes.c_void_p)
_proto("aol_plan_set_tile", ctypes.c_int, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32)
_proto("aol_plan_set_walk", ctypes.c_int, ctypes.c_void_p, ctypes.c_int32)
_proto("aol_plan_set_band", ctypes.c_int, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32)
_proto("aol_plan_schedule", ctypes.c_char_p, ctypes.c_void_p, ctypes.c_int32)
_proto("aol_downscale_u8", ctypes.c_int, ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_void_p), c_i64p,
       ctypes.POINTER(ctypes.c_void_p), c_i64p, ctypes.c_void_p)
_proto("aol_downscale_f", ctypes.c_int, ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_void_p), c_i64p,
       ctypes.POINTER(ctypes.c_void_p), c_i64p, ctypes.c_void_p)

_proto("aol_unfused_workspace_bytes", ctypes.c_int, ctypes.c_void_p, c_i64p)
_proto("aol_downscale_u8_unfused", ctypes.c_int, ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_void_p), c_i64p,
       ctypes.POINTER(ctypes.c_void_p), c_i64p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p)

_proto("aol_downscale_u8_unfused_static", ctypes.c_int, ctypes.c_void_p, ctypes.c_int32,
       ctypes.POINTER(ctypes.c_void_p), c_i64p, ctypes.POINTER(ctypes.c_void_p), c_i64p, ctypes.c_void_p)


class aol_pipeline_stats(ctypes.Structure):
    _fields_ = [("groups", ctypes.c_int32), ("frames", ctypes.c_int32), ("wall_ms", ctypes.c_double),
                ("span_ms", ctypes.c_double), ("h2d_ms", ctypes.c_double), ("kernel_ms", ctypes.c_double),
                ("d2h_ms", ctypes.c_double), ("h2d_bytes", ctypes.c_int64), ("d2h_bytes", ctypes.c_int64)]


_proto("aol_pipeline_create", ctypes.c_int, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
       ctypes.POINTER(ctypes.c_void_p))
_proto("aol_pipeline_destroy", ctypes.c_int, ctypes.c_void_p)
_proto("aol_pipeline_run_u8", ctypes.c_int, ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_void_p), c_i64p,
       ctypes.POINTER(ctypes.c_void_p), c_i64p, ctypes.c_void_p, ctypes.POINTER(aol_pipeline_stats))


class aol_stream_desc(ctypes.Structure):
    _fields_ = [("height", ctypes.c_int64), ("width", ctypes.c_int64), ("in_pitch", ctypes.c_int64),
                ("out_pitch", ctypes.c_int64), ("hf", aol_polyphase), ("vf", aol_polyphase)]


_proto("aol_batch_plan_create", ctypes.c_int, ctypes.c_int32, ctypes.POINTER(aol_stream_desc), ctypes.c_int,
       ctypes.c_char_p, ctypes.POINTER(ctypes.c_void_p))
_proto("aol_batch_plan_destroy", ctypes.c_int, ctypes.c_void_p)
_proto("aol_batch_set_pointers", ctypes.c_int, ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p),
       ctypes.POINTER(ctypes.c_void_p), ctypes.c_void_p)
_proto("aol_batch_run", ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p)
_proto("aol_batch_graph_create", ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p))
_proto("aol_batch_graph_create_pointers", ctypes.c_int, ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p),
       ctypes.POINTER(ctypes.c_void_p), ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p))
_proto("aol_graph_launch", ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p)
_proto("aol_batch_buffers_create", ctypes.c_int, ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p),
       ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_void_p))
_proto("aol_batch_run_buffers", ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)
_proto("aol_batch_buffers_destroy", ctypes.c_int, ctypes.c_void_p)
_proto("aol_graph_destroy", ctypes.c_int, ctypes.c_void_p)
_proto("aol_autotune", ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p)
_proto("aol_batch_schedule", ctypes.c_char_p, ctypes.c_void_p)
_proto("aol_batch_set_schedule", ctypes.c_int, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32)
_proto("aol_batch_set_part_weight", ctypes.c_int, ctypes.c_void_p, ctypes.c_int32)


class aol_tiler(ctypes.Structure):
    _fields_ = [("array_rank", ctypes.c_int32), ("rep_rank", ctypes.c_int32), ("pat_rank", ctypes.c_int32),
                ("reserved", ctypes.c_int32),
                ("array_shape", ctypes.c_int64 * 4), ("rep_shape", ctypes.c_int64 * 4),
                ("pat_shape", ctypes.c_int64 * 4), ("origin", ctypes.c_int64 * 4),
                ("paving", (ctypes.c_int64 * 4) * 4), ("fitting", (ctypes.c_int64 * 4) * 4)]


_proto("aol_wsum_plan_create", ctypes.c_int, ctypes.POINTER(aol_tiler), ctypes.POINTER(aol_tiler),
       ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_void_p))
_proto("aol_wsum_run", ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)
_proto("aol_wsum_plan_destroy", ctypes.c_int, ctypes.c_void_p)
_proto("aol_weighted_sum_f32", ctypes.c_int, ctypes.POINTER(aol_tiler), ctypes.POINTER(aol_tiler),
       ctypes.POINTER(ctypes.c_float), ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)

_proto("aol_linear_plan_create", ctypes.c_int, ctypes.POINTER(aol_tiler), ctypes.POINTER(aol_tiler), c_i16p,
       c_i32p, ctypes.POINTER(ctypes.c_void_p))
_proto("aol_linear_run", ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)
_proto("aol_linear_plan_destroy", ctypes.c_int, ctypes.c_void_p)


def _check(status: int):
    if status != AOL_OK:
        raise AolError(status, _lib.aol_last_error().decode())


def aol_last_error() -> str:
    return _lib.aol_last_error().decode()


def aol_version() -> str:
    return _lib.aol_version().decode()


def _stream_handle(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


# --------------------------------------------------------------------------
# filters
# --------------------------------------------------------------------------

class Polyphase:
    """One axis' filter: ratio p/q, integer taps ``coeff[p][taps]``, optional window starts."""

    def __init__(self, p: int, q: int, coeff, phase_start=None):
        self.coeff = np.ascontiguousarray(np.asarray(coeff, dtype=np.int16).reshape(int(p), -1))
        self.p, self.q, self.taps = int(p), int(q), int(self.coeff.shape[1])
        self.phase_start = None if phase_start is None else np.ascontiguousarray(np.asarray(phase_start, np.int32))
        self._c = aol_polyphase(self.p, self.q, self.taps, self.coeff.ctypes.data_as(c_i16p),
                                None if self.phase_start is None else self.phase_start.ctypes.data_as(c_i32p))

    @property
    def c_struct(self) -> aol_polyphase:
        return self._c


def aol_default_phase_starts(p: int, q: int, taps: int) -> list:
    out = (ctypes.c_int32 * int(p))()
    _check(_lib.aol_default_phase_starts(p, q, taps, out))
    return list(out)


def aol_downscale_output_shape(h: int, w: int, hf: Polyphase, vf: Polyphase):
    oh, ow = ctypes.c_int64(), ctypes.c_int64()
    _check(_lib.aol_downscale_output_shape(h, w, ctypes.byref(hf.c_struct), ctypes.byref(vf.c_struct),
                                           ctypes.byref(oh), ctypes.byref(ow)))
    return oh.value, ow.value


# --------------------------------------------------------------------------
# frame downscaler
# --------------------------------------------------------------------------

def aol_downscale_plan_create(planes, hf: Polyphase, vf: Polyphase, precision="u8"):
    """``planes``: list of (height, width[, in_pitch, out_pitch]). Returns an opaque handle."""
    arr = (aol_plane_desc * len(planes))()
    for i, d in enumerate(planes):
        d = [int(v) for v in d] + [0] * (4 - len(d))
        arr[i] = aol_plane_desc(*d[:4])
    h = ctypes.c_void_p()
    prec = _PREC[precision] if isinstance(precision, str) else int(precision)
    _check(_lib.aol_downscale_plan_create(arr, len(planes), ctypes.byref(hf.c_struct), ctypes.byref(vf.c_struct),
                                          prec, ctypes.byref(h)))
    return h


def aol_plan_destroy(plan):
    _check(_lib.aol_plan_destroy(plan))


def aol_plan_set_tile(plan, tile_rx: int, tile_ry: int):
    _check(_lib.aol_plan_set_tile(plan, tile_rx, tile_ry))


def aol_plan_set_band(plan, band_reps: int, seg_reps: int):
    _check(_lib.aol_plan_set_band(plan, band_reps, seg_reps))


def aol_plan_set_walk(plan, order: int):
    _check(_lib.aol_plan_set_walk(plan, order))


def aol_plan_schedule(plan, n_frames: int) -> str:
    return _lib.aol_plan_schedule(plan, int(n_frames)).decode()


def _ptrs(vals):
    return (ctypes.c_void_p * len(vals))(*[int(v) for v in vals])


def _i64s(vals):
    return (ctypes.c_int64 * len(vals))(*[int(v) for v in vals])


def aol_downscale_u8(plan, n_frames, d_in, in_frame_stride, d_out, out_frame_stride, stream=None):
    _check(_lib.aol_downscale_u8(plan, int(n_frames), _ptrs(d_in), _i64s(in_frame_stride), _ptrs(d_out),
                                 _i64s(out_frame_stride), _stream_handle(stream)))


def aol_downscale_f(plan, n_frames, d_in, in_frame_stride, d_out, out_frame_stride, stream=None):
    _check(_lib.aol_downscale_f(plan, int(n_frames), _ptrs(d_in), _i64s(in_frame_stride), _ptrs(d_out),
                                _i64s(out_frame_stride), _stream_handle(stream)))


def aol_unfused_workspace_bytes(plan) -> int:
    n = ctypes.c_int64()
    _check(_lib.aol_unfused_workspace_bytes(plan, ctypes.byref(n)))
    return n.value


def aol_downscale_u8_unfused(plan, n_frames, d_in, in_frame_stride, d_out, out_frame_stride, d_work, work_bytes,
                             stream=None):
    _check(_lib.aol_downscale_u8_unfused(plan, int(n_frames), _ptrs(d_in), _i64s(in_frame_stride), _ptrs(d_out),
                                         _i64s(out_frame_stride), ctypes.c_void_p(int(d_work)), int(work_bytes),
                                         _stream_handle(stream)))


def aol_downscale_u8_unfused_static(plan, n_frames, d_in, in_frame_stride, d_out, out_frame_stride, stream=None):
    _check(_lib.aol_downscale_u8_unfused_static(plan, int(n_frames), _ptrs(d_in), _i64s(in_frame_stride),
                                                _ptrs(d_out), _i64s(out_frame_stride), _stream_handle(stream)))


class DownscalePlan:
    """Plan for a set of planes filtered by (hf, vf); runs on torch device tensors.

    Each plane's frames are a tensor ``[n_frames, h, w]`` (uint8 for ``"u8"``;
    int16/uint16/bfloat16/float16 bit patterns for ``"bf16"``/``"fp16"``) with
    unit stride along rows; outputs are ``[n_frames, out_h, out_w]`` uint8 or
    float32 tensors with unit stride along rows.
    """

    def __init__(self, shapes, hf: Polyphase, vf: Polyphase, precision="u8", in_pitches=None, out_pitches=None):
        self.hf, self.vf, self.precision = hf, vf, precision
        self.shapes = [tuple(int(v) for v in s) for s in shapes]
        self.out_shapes = [aol_downscale_output_shape(h, w, hf, vf) for (h, w) in self.shapes]
        self.in_pitches = list(in_pitches or [w for (h, w) in self.shapes])
        self.out_pitches = list(out_pitches or [ow for (oh, ow) in self.out_shapes])
        self._h = aol_downscale_plan_create(
            [(h, w, self.in_pitches[i], self.out_pitches[i]) for i, (h, w) in enumerate(self.shapes)],
            hf, vf, precision)

    def set_tile(self, tile_rx: int, tile_ry: int):
        aol_plan_set_tile(self._h, tile_rx, tile_ry)

    def set_band(self, band_reps: int = 0, seg_reps: int = 0):
        aol_plan_set_band(self._h, band_reps, seg_reps)

    def set_walk(self, order: int):
        aol_plan_set_walk(self._h, order)

    def schedule(self, n_frames: int) -> dict:
        """The schedule a launch over ``n_frames`` frames uses."""
        import json
        return json.loads(aol_plan_schedule(self._h, n_frames))

    def close(self):
        if getattr(self, "_h", None):
            aol_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check_tensors(self, ins, outs):
        import torch
        if len(ins) != len(self.shapes) or len(outs) != len(self.shapes):
            raise ValueError("one input and one output tensor per plane")
        n = ins[0].shape[0]
        for i, (t, (h, w), o, (oh, ow)) in enumerate(zip(ins, self.shapes, outs, self.out_shapes)):
            if not (t.is_cuda and o.is_cuda):
                raise ValueError("tensors must be on the GPU")
            if t.stride(1) != self.in_pitches[i] or o.stride(1) != self.out_pitches[i]:
                raise ValueError("row strides must equal the plan's pitches")
            if t.dim() != 3 or t.shape[0] != n or t.shape[1] != h or t.shape[2] != w or t.stride(2) != 1:
                raise ValueError(f"input must be [n_frames, {h}, {w}] with unit column stride")
            if o.dim() != 3 or o.shape[0] != n or o.shape[1] != oh or o.shape[2] != ow or o.stride(2) != 1:
                raise ValueError(f"output must be [n_frames, {oh}, {ow}] with unit column stride")
            if self.precision == "u8":
                if t.dtype != torch.uint8 or o.dtype != torch.uint8:
                    raise ValueError("u8 plans take uint8 tensors")
            else:
                if t.element_size() != 2 or o.dtype != torch.float32:
                    raise ValueError("float plans take 16-bit inputs and float32 outputs")
        return n

    def workspace_bytes(self) -> int:
        """Workspace bytes per frame of the unfused form (integer plans)."""
        return aol_unfused_workspace_bytes(self._h)

    def run_unfused(self, ins, outs, work, stream=None):
        """The two-kernel form: the intermediate goes through ``work`` (a uint8 device
        tensor, 256-byte aligned); frames run in groups that fit it."""
        import torch
        n = self._check_tensors(ins, outs)
        if not work.is_cuda or work.dtype != torch.uint8 or not work.is_contiguous():
            raise ValueError("workspace must be a contiguous uint8 device tensor")
        aol_downscale_u8_unfused(self._h, n, [t.data_ptr() for t in ins], [t.stride(0) for t in ins],
                                 [o.data_ptr() for o in outs], [o.stride(0) for o in outs], work.data_ptr(),
                                 work.numel(), stream)

    def run(self, ins, outs, stream=None):
        n = self._check_tensors(ins, outs)
        fn = aol_downscale_u8 if self.precision == "u8" else aol_downscale_f
        fn(self._h, n, [t.data_ptr() for t in ins], [t.stride(0) for t in ins],
           [o.data_ptr() for o in outs], [o.stride(0) for o in outs], stream)


# --------------------------------------------------------------------------
# host-to-host frame pipeline
# --------------------------------------------------------------------------

def aol_pipeline_create(plan, batch_frames: int, depth: int):
    h = ctypes.c_void_p()
    _check(_lib.aol_pipeline_create(plan, int(batch_frames), int(depth), ctypes.byref(h)))
    return h


def aol_pipeline_destroy(pipe):
    _check(_lib.aol_pipeline_destroy(pipe))


def aol_pipeline_run_u8(pipe, n_frames, h_in, in_frame_stride, h_out, out_frame_stride, stream=None) -> dict:
    st = aol_pipeline_stats()
    _check(_lib.aol_pipeline_run_u8(pipe, int(n_frames), _ptrs(h_in), _i64s(in_frame_stride), _ptrs(h_out),
                                    _i64s(out_frame_stride), _stream_handle(stream), ctypes.byref(st)))
    return {f: getattr(st, f) for f, _ in aol_pipeline_stats._fields_}


class Pipeline:
    """Host-to-host downscale of frames in host memory (CPU tensors ``[n_frames, h, w]``, uint8,
    ideally pinned): groups of ``batch_frames`` frames, ``depth`` groups in flight."""

    def __init__(self, plan: "DownscalePlan", batch_frames: int = 1, depth: int = 3):
        if plan.precision != "u8":
            raise ValueError("pipelines run integer plans")
        self.plan = plan  # kept alive: the pipeline refers to it
        self._h = aol_pipeline_create(plan._h, batch_frames, depth)

    def run(self, ins, outs, stream=None) -> dict:
        """Blocks until every output frame is in host memory; returns the stage times."""
        import torch
        n = ins[0].shape[0]
        for t, (h, w), o, (oh, ow), ip, op in zip(ins, self.plan.shapes, outs, self.plan.out_shapes,
                                                  self.plan.in_pitches, self.plan.out_pitches):
            if t.is_cuda or o.is_cuda or t.dtype != torch.uint8 or o.dtype != torch.uint8:
                raise ValueError("host uint8 tensors expected")
            if tuple(t.shape) != (n, h, w) or tuple(o.shape) != (n, oh, ow):
                raise ValueError(f"shapes must be [{n}, {h}, {w}] -> [{n}, {oh}, {ow}]")
            if t.stride(1) != ip or o.stride(1) != op or t.stride(2) != 1 or o.stride(2) != 1:
                raise ValueError("row strides must equal the plan's pitches")
        return aol_pipeline_run_u8(self._h, n, [t.data_ptr() for t in ins], [t.stride(0) for t in ins],
                                   [o.data_ptr() for o in outs], [o.stride(0) for o in outs], stream)

    def close(self):
        if getattr(self, "_h", None):
            aol_pipeline_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# --------------------------------------------------------------------------
# generic weighted-sum repetition
# --------------------------------------------------------------------------

def make_tiler(array_shape, rep_shape, pat_shape, origin, paving, fitting) -> aol_tiler:
    """Build an ``aol_tiler``; ``paving`` is [array dim][rep dim], ``fitting`` [array dim][pattern dim]."""
    t = aol_tiler()
    t.array_rank, t.rep_rank, t.pat_rank = len(array_shape), len(rep_shape), len(pat_shape)
    for d, v in enumerate(array_shape):
        t.array_shape[d] = int(v)
    for k, v in enumerate(rep_shape):
        t.rep_shape[k] = int(v)
    for b, v in enumerate(pat_shape):
        t.pat_shape[b] = int(v)
    for d, v in enumerate(origin):
        t.origin[d] = int(v)
    P = np.asarray(paving, dtype=np.int64).reshape(len(array_shape), len(rep_shape))
    F = np.asarray(fitting, dtype=np.int64).reshape(len(array_shape), len(pat_shape))
    for d in range(len(array_shape)):
        for k in range(len(rep_shape)):
            t.paving[d][k] = int(P[d, k])
        for b in range(len(pat_shape)):
            t.fitting[d][b] = int(F[d, b])
    return t


def identity_out_tiler(rep_shape) -> aol_tiler:
    d = len(rep_shape)
    return make_tiler(rep_shape, rep_shape, (), (0,) * d, np.eye(d, dtype=np.int64), np.zeros((d, 0), np.int64))


def aol_wsum_plan_create(tin: aol_tiler, tout: aol_tiler, weights):
    w = np.ascontiguousarray(np.asarray(weights, dtype=np.float32).ravel())
    h = ctypes.c_void_p()
    _check(_lib.aol_wsum_plan_create(ctypes.byref(tin), ctypes.byref(tout),
                                     w.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), ctypes.byref(h)))
    return h


def aol_wsum_run(plan, d_in, d_out, stream=None):
    _check(_lib.aol_wsum_run(plan, ctypes.c_void_p(int(d_in)), ctypes.c_void_p(int(d_out)), _stream_handle(stream)))


def aol_wsum_plan_destroy(plan):
    _check(_lib.aol_wsum_plan_destroy(plan))


def aol_weighted_sum_f32(tin: aol_tiler, tout: aol_tiler, weights, d_in, d_out, stream=None):
    """One-shot weighted-sum repetition (no plan; the weights go in the kernel arguments)."""
    w = np.ascontiguousarray(np.asarray(weights, dtype=np.float32).ravel())
    _check(_lib.aol_weighted_sum_f32(ctypes.byref(tin), ctypes.byref(tout),
                                     w.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                     ctypes.c_void_p(int(d_in)), ctypes.c_void_p(int(d_out)), _stream_handle(stream)))


class WeightedSumPlan:
    """``out[(o' + P'.r) mod S'] = sum_i w[i] * in[(o + P.r + F.i) mod S]`` on float32 device tensors."""

    def __init__(self, tin: aol_tiler, tout: aol_tiler, weights):
        self.tin, self.tout = tin, tout
        self.in_shape = tuple(tin.array_shape[d] for d in range(tin.array_rank))
        self.out_shape = tuple(tout.array_shape[d] for d in range(tout.array_rank))
        self._h = aol_wsum_plan_create(tin, tout, weights)

    def run(self, x, y, stream=None):
        import torch
        if x.dtype != torch.float32 or y.dtype != torch.float32 or not (x.is_cuda and y.is_cuda):
            raise ValueError("float32 device tensors expected")
        if tuple(x.shape) != self.in_shape or tuple(y.shape) != self.out_shape:
            raise ValueError(f"shapes must be {self.in_shape} -> {self.out_shape}")
        if not (x.is_contiguous() and y.is_contiguous()):
            raise ValueError("contiguous tensors expected")
        aol_wsum_run(self._h, x.data_ptr(), y.data_ptr(), stream)

    def close(self):
        if getattr(self, "_h", None):
            aol_wsum_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# --------------------------------------------------------------------------
# linear integer repetition (uint8)
# --------------------------------------------------------------------------

def aol_linear_plan_create(tin: aol_tiler, tout: aol_tiler, weights, bias=None):
    w = np.ascontiguousarray(np.asarray(weights, dtype=np.int16).ravel())
    b = None if bias is None else np.ascontiguousarray(np.asarray(bias, dtype=np.int32).ravel())
    h = ctypes.c_void_p()
    _check(_lib.aol_linear_plan_create(ctypes.byref(tin), ctypes.byref(tout), w.ctypes.data_as(c_i16p),
                                       None if b is None else b.ctypes.data_as(c_i32p), ctypes.byref(h)))
    return h


def aol_linear_run(plan, d_in, d_out, stream=None):
    _check(_lib.aol_linear_run(plan, ctypes.c_void_p(int(d_in)), ctypes.c_void_p(int(d_out)), _stream_handle(stream)))


def aol_linear_plan_destroy(plan):
    _check(_lib.aol_linear_plan_destroy(plan))


class LinearPlan:
    """``out[(o' + P'.r + F'.j) mod S'] = clamp(floor((sum_i W[j][i] in[(o + P.r + F.i) mod S]
    + bias[j] + 128) / 256), 0, 255)`` on uint8 device tensors."""

    def __init__(self, tin: aol_tiler, tout: aol_tiler, weights, bias=None):
        self.in_shape = tuple(tin.array_shape[d] for d in range(tin.array_rank))
        self.out_shape = tuple(tout.array_shape[d] for d in range(tout.array_rank))
        self._h = aol_linear_plan_create(tin, tout, weights, bias)

    def run(self, x, y, stream=None):
        import torch
        if x.dtype != torch.uint8 or y.dtype != torch.uint8 or not (x.is_cuda and y.is_cuda):
            raise ValueError("uint8 device tensors expected")
        if tuple(x.shape) != self.in_shape or tuple(y.shape) != self.out_shape:
            raise ValueError(f"shapes must be {self.in_shape} -> {self.out_shape}")
        if not (x.is_contiguous() and y.is_contiguous()):
            raise ValueError("contiguous tensors expected")
        aol_linear_run(self._h, x.data_ptr(), y.data_ptr(), stream)

    def close(self):
        if getattr(self, "_h", None):
            aol_linear_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# --------------------------------------------------------------------------
# batches of streams
# --------------------------------------------------------------------------

def aol_batch_plan_create(streams, precision="u8", tune_cache=None):
    """``streams``: list of (height, width, hf, vf[, in_pitch, out_pitch]) with Polyphase filters."""
    arr = (aol_stream_desc * len(streams))()
    for i, st in enumerate(streams):
        h, w, hf, vf = st[:4]
        ip, op = (st[4], st[5]) if len(st) >= 6 else (0, 0)
        arr[i] = aol_stream_desc(int(h), int(w), int(ip), int(op), hf.c_struct, vf.c_struct)
    hnd = ctypes.c_void_p()
    prec = _PREC[precision] if isinstance(precision, str) else int(precision)
    _check(_lib.aol_batch_plan_create(len(streams), arr, prec, None if tune_cache is None else tune_cache.encode(),
                                      ctypes.byref(hnd)))
    return hnd


def aol_batch_plan_destroy(plan):
    _check(_lib.aol_batch_plan_destroy(plan))


def aol_batch_set_pointers(plan, d_in, d_out, stream=None):
    _check(_lib.aol_batch_set_pointers(plan, _ptrs(d_in), _ptrs(d_out), _stream_handle(stream)))


def aol_batch_run(plan, stream=None):
    _check(_lib.aol_batch_run(plan, _stream_handle(stream)))


def aol_batch_graph_create(plan, stream):
    g = ctypes.c_void_p()
    _check(_lib.aol_batch_graph_create(plan, _stream_handle(stream), ctypes.byref(g)))
    return g


def aol_batch_graph_create_pointers(plan, d_in, d_out, stream):
    g = ctypes.c_void_p()
    _check(_lib.aol_batch_graph_create_pointers(plan, d_in, d_out, _stream_handle(stream), ctypes.byref(g)))
    return g


def aol_graph_launch(graph, stream=None):
    _check(_lib.aol_graph_launch(graph, _stream_handle(stream)))


def aol_batch_buffers_create(plan, d_in, d_out):
    b = ctypes.c_void_p()
    _check(_lib.aol_batch_buffers_create(plan, d_in, d_out, ctypes.byref(b)))
    return b


def aol_batch_run_buffers(plan, buffers, stream=None):
    _check(_lib.aol_batch_run_buffers(plan, buffers, _stream_handle(stream)))


def aol_batch_buffers_destroy(buffers):
    _check(_lib.aol_batch_buffers_destroy(buffers))


def aol_graph_destroy(graph):
    _check(_lib.aol_graph_destroy(graph))


def aol_autotune(plan, stream=None):
    _check(_lib.aol_autotune(plan, _stream_handle(stream)))


def aol_batch_schedule(plan) -> str:
    return _lib.aol_batch_schedule(plan).decode()


def aol_batch_set_schedule(plan, seg_reps: int, lds_budget: int):
    _check(_lib.aol_batch_set_schedule(plan, int(seg_reps), int(lds_budget)))


def aol_batch_set_part_weight(plan, permille: int):
    _check(_lib.aol_batch_set_part_weight(plan, int(permille)))


class BatchPlan:
    """Many streams, one frame each per step, one persistent launch (optionally a graph)."""

    def __init__(self, streams, precision="u8", tune_cache=None):
        self.precision = precision
        self.filters = [(s[2], s[3]) for s in streams]  # keep the coefficient arrays alive
        self.shapes = [(int(s[0]), int(s[1])) for s in streams]
        self.out_shapes = [aol_downscale_output_shape(h, w, hf, vf) for (h, w), (hf, vf) in zip(self.shapes, self.filters)]
        self._h = aol_batch_plan_create(streams, precision, tune_cache)
        self._graphs = []
        self._buffer_sets = []

    def set_pointers(self, ins, outs, stream=None):
        self.set_pointer_arrays(self.pointer_arrays(ins, outs), stream)

    def pointer_arrays(self, ins, outs):
        """Checks one frame's tensors and returns their device addresses as the two
        pointer arrays `set_pointer_arrays` takes (build them once per set of buffers)."""
        import torch
        if len(ins) != len(self.shapes) or len(outs) != len(self.shapes):
            raise ValueError("one input and one output per stream")
        for t, (h, w), o, (oh, ow) in zip(ins, self.shapes, outs, self.out_shapes):
            if not (t.is_cuda and o.is_cuda) or t.shape[-2:] != (h, w) or o.shape[-2:] != (oh, ow):
                raise ValueError("one [h, w] input and one [out_h, out_w] output device tensor per stream")
            if not (t.is_contiguous() and o.is_contiguous()):
                raise ValueError("contiguous tensors expected")
            if self.precision == "u8" and (t.dtype != torch.uint8 or o.dtype != torch.uint8):
                raise ValueError("u8 batches take uint8 tensors")
            if self.precision != "u8" and (t.element_size() != 2 or o.dtype != torch.float32):
                raise ValueError("float batches take 16-bit inputs and float32 outputs")
        return _ptrs([t.data_ptr() for t in ins]), _ptrs([o.data_ptr() for o in outs])

    def set_pointer_arrays(self, arrays, stream=None):
        """Points the next launches at the buffers of `pointer_arrays` (a stream-ordered
        update of the device pointer table; the tensors must stay alive)."""
        _check(_lib.aol_batch_set_pointers(self._h, arrays[0], arrays[1], _stream_handle(stream)))

    def run(self, stream=None):
        aol_batch_run(self._h, stream)

    def graph(self, stream):
        g = aol_batch_graph_create(self._h, stream)
        self._graphs.append(g)
        return g

    def graph_with_pointers(self, arrays, stream):
        """A graph that runs one step on the buffers of `pointer_arrays`, with its own pointer
        table (one graph per buffer set; the tensors must stay alive)."""
        g = aol_batch_graph_create_pointers(self._h, arrays[0], arrays[1], stream)
        self._graphs.append(g)
        return g

    def buffers(self, arrays):
        """A buffer set: the buffers of `pointer_arrays` in a pointer table of its own (one
        per frame slot of a serving loop; the tensors must stay alive)."""
        b = aol_batch_buffers_create(self._h, arrays[0], arrays[1])
        self._buffer_sets.append(b)
        return b

    def run_buffers(self, buffers, stream=None):
        """One step over a buffer set: one launch, the plan's own pointer table untouched."""
        aol_batch_run_buffers(self._h, buffers, stream)

    def autotune(self, stream=None):
        aol_autotune(self._h, stream)

    def schedule(self) -> str:
        return aol_batch_schedule(self._h)

    def set_schedule(self, seg_reps: int, lds_budget: int):
        aol_batch_set_schedule(self._h, seg_reps, lds_budget)

    def set_part_weight(self, permille: int):
        aol_batch_set_part_weight(self._h, permille)

    def close(self):
        for g in self._graphs:
            aol_graph_destroy(g)
        self._graphs = []
        for b in getattr(self, "_buffer_sets", []):
            aol_batch_buffers_destroy(b)
        self._buffer_sets = []
        if getattr(self, "_h", None):
            aol_batch_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
