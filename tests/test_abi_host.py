"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every symbol the public header declares, and validates arguments on the
host before touching the device."""

import ctypes
import os
import re

import numpy as np
import pytest

import synthgen
import paper_1103_4881_amd as aol
from oracle import polyphase as pp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names.update(re.findall(r"\b(aol_[a-z0-9_]+)\s*\(", text))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    names = _declared_symbols()
    assert "aol_downscale_u8" in names and "aol_downscale_f" in names
    lib = ctypes.CDLL(aol.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.parametrize("p,q,T", [(3, 8, 11), (1, 2, 8), (2, 3, 16), (4, 9, 7), (5, 3, 6), (16, 64, 32), (1, 1, 1)])
def test_default_phase_starts_match_oracle(p, q, T):
    assert aol.aol_default_phase_starts(p, q, T) == pp.default_phase_starts(p, q, T)


@pytest.mark.parametrize("h,w", [(480, 640), (1080, 1920), (540, 960), (1, 1), (17, 9), (288, 352)])
def test_output_shape_matches_oracle(h, w):
    hf = aol.Polyphase(3, 8, synthgen.design_taps(3, 8, 11))
    vf = aol.Polyphase(2, 3, synthgen.design_taps(2, 3, 10))
    oh, ow = aol.aol_downscale_output_shape(h, w, hf, vf)
    assert (oh, ow) == (pp.output_length(h, 2, 3), pp.output_length(w, 3, 8))


def test_paper_cif_output_shape():
    hf = aol.Polyphase(3, 8, synthgen.design_taps(3, 8, 11))
    vf = aol.Polyphase(4, 9, synthgen.design_taps(4, 9, 11))
    assert aol.aol_downscale_output_shape(288, 352, hf, vf) == (128, 132)


def _expect(status, fn, *args):
    with pytest.raises(aol.AolError) as ei:
        fn(*args)
    assert ei.value.status == status, ei.value.msg
    assert aol.aol_last_error()


def test_invalid_arguments_are_rejected_on_host():
    good = aol.Polyphase(3, 8, synthgen.design_taps(3, 8, 11))
    _expect(aol.AOL_ERR_INVALID, aol.aol_default_phase_starts, 0, 8, 11)
    _expect(aol.AOL_ERR_INVALID, aol.aol_downscale_output_shape, 0, 10, good, good)
    bad_p = aol.Polyphase(17, 8, np.full((17, 4), 64))
    _expect(aol.AOL_ERR_UNSUPPORTED, aol.aol_downscale_plan_create, [(64, 64)], bad_p, good, "u8")
    big_taps = aol.Polyphase(1, 2, np.full((1, 33), 8))
    _expect(aol.AOL_ERR_UNSUPPORTED, aol.aol_downscale_plan_create, [(64, 64)], good, big_taps, "u8")
    _expect(aol.AOL_ERR_INVALID, aol.aol_downscale_plan_create, [(0, 64)], good, good, "u8")
    _expect(aol.AOL_ERR_UNSUPPORTED, aol.aol_downscale_plan_create, [(64, 64)] * 5, good, good, "u8")
    _expect(aol.AOL_ERR_INVALID, aol.aol_downscale_plan_create, [(64, 64, 10, 0)], good, good, "u8")
    huge = aol.Polyphase(1, 2, [[4000, -3744]])
    _expect(aol.AOL_ERR_UNSUPPORTED, aol.aol_downscale_plan_create, [(64, 64)], huge, good, "u8")
    # 3/256 needs more significant bits than bf16 holds (taps 257 -> 257/256)
    odd = aol.Polyphase(1, 2, [[257, -1]])
    _expect(aol.AOL_ERR_UNSUPPORTED, aol.aol_downscale_plan_create, [(64, 64)], odd, good, "bf16")
    _expect(aol.AOL_ERR_INVALID, aol.aol_downscale_plan_create, [(64, 64)], good, good, 7)


def test_single_hip_runtime_in_process():
    """The library must bind to torch's HIP runtime, not load a second one."""
    with open("/proc/self/maps") as fh:
        paths = {line.split()[-1] for line in fh if "libamdhip64" in line}
    assert len(paths) == 1, paths


def test_wsum_validation_on_host():
    w = np.ones(9, np.float32)
    good = aol.make_tiler((8, 8), (8, 8), (3, 3), (0, 0), [[1, 0], [0, 1]], [[1, 0], [0, 1]])
    ident = aol.identity_out_tiler((8, 8))
    # output tiler that is not a bijection: every repetition writes row 0
    clash = aol.make_tiler((8, 8), (8, 8), (), (0, 0), [[0, 0], [0, 1]], np.zeros((2, 0), np.int64))
    _expect(aol.AOL_ERR_INVALID, aol.aol_wsum_plan_create, good, clash, w)
    # output array of the wrong size
    small = aol.identity_out_tiler((8, 7))
    _expect(aol.AOL_ERR_INVALID, aol.aol_wsum_plan_create, good, small, w)
    # pattern too large
    big = aol.make_tiler((8, 8), (8, 8), (9, 9), (0, 0), [[1, 0], [0, 1]], [[1, 0], [0, 1]])
    _expect(aol.AOL_ERR_UNSUPPORTED, aol.aol_wsum_plan_create, big, ident, np.ones(81, np.float32))
    # rank 5
    t5 = aol.make_tiler((2, 2, 2, 2), (2, 2, 2, 2), (1,), (0, 0, 0, 0), np.eye(4, dtype=np.int64),
                        np.zeros((4, 1), np.int64))
    t5.array_rank = 5
    _expect(aol.AOL_ERR_UNSUPPORTED, aol.aol_wsum_plan_create, t5, aol.identity_out_tiler((2, 2, 2, 2)), w)
    # a valid plan needs no device: creation succeeds and destroys cleanly
    h = aol.aol_wsum_plan_create(good, ident, w)
    aol.aol_wsum_plan_destroy(h)


def test_batch_validation_on_host():
    good = aol.Polyphase(3, 8, synthgen.design_taps(3, 8, 11))
    bad = aol.Polyphase(17, 8, np.full((17, 4), 64))
    _expect(aol.AOL_ERR_INVALID, aol.aol_batch_plan_create, [(0, 64, good, good)], "u8")
    _expect(aol.AOL_ERR_UNSUPPORTED, aol.aol_batch_plan_create, [(64, 64, good, good), (64, 64, bad, good)], "u8")
    _expect(aol.AOL_ERR_INVALID, aol.aol_batch_plan_create, [(64, 64, good, good, 10, 0)], "u8")
    _expect(aol.AOL_ERR_INVALID, aol.aol_batch_run, None, 0)


def test_one_shot_weighted_sum_validation_on_host():
    """aol_weighted_sum_f32 validates both tilers and the buffers before any launch (stream 0:
    no device is touched)."""
    w = np.ones(9, np.float32)
    good = aol.make_tiler((8, 8), (8, 8), (3, 3), (0, 0), [[1, 0], [0, 1]], [[1, 0], [0, 1]])
    ident = aol.identity_out_tiler((8, 8))
    clash = aol.make_tiler((8, 8), (8, 8), (), (0, 0), [[0, 0], [0, 1]], np.zeros((2, 0), np.int64))
    _expect(aol.AOL_ERR_INVALID, aol.aol_weighted_sum_f32, good, clash, w, 16, 16, 0)
    _expect(aol.AOL_ERR_INVALID, aol.aol_weighted_sum_f32, good, aol.identity_out_tiler((8, 7)), w, 16, 16, 0)
    big = aol.make_tiler((8, 8), (8, 8), (9, 9), (0, 0), [[1, 0], [0, 1]], [[1, 0], [0, 1]])
    _expect(aol.AOL_ERR_UNSUPPORTED, aol.aol_weighted_sum_f32, big, ident, np.ones(81, np.float32), 16, 16, 0)
    _expect(aol.AOL_ERR_INVALID, aol.aol_weighted_sum_f32, good, ident, w, 0, 16, 0)  # NULL input
    _expect(aol.AOL_ERR_INVALID, aol.aol_weighted_sum_f32, good, ident, w, 18, 16, 0)  # misaligned input


def test_schedule_calls_reject_null_plans():
    _expect(aol.AOL_ERR_INVALID, aol.aol_batch_set_schedule, None, 0, 150 * 1024)
    _expect(aol.AOL_ERR_INVALID, aol.aol_batch_set_part_weight, None, 1000)
    _expect(aol.AOL_ERR_INVALID, aol.aol_batch_run_buffers, None, None, 0)
    _expect(aol.AOL_ERR_INVALID, aol.aol_batch_buffers_create, None, None, None)
    assert aol.aol_plan_schedule(None, 1) == ""
