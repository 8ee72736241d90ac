"""Guards on the gfx950 code the library's kernels compile to (CPU only).

* The integer epilogue must not use v_ashr_pk_u8_i32: the compiler ORs the
  whole destination register afterwards while the instruction leaves the
  upper half holding the sign bits of a negative sum, which corrupts the
  neighbouring bytes (seen as saturated pixels after negative-lobe sums).
* No kernel may use scratch (private segment) memory.
"""

import glob
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1103_4881_amd", "csrc")
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


@pytest.fixture(scope="module")
def device_asm(tmp_path_factory):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    out = {}
    for src in sorted(glob.glob(os.path.join(CSRC, "*.hip"))):
        dst = tmp_path_factory.mktemp("asm") / (os.path.basename(src) + ".s")
        cmd = [HIPCC, "-x", "hip", "--offload-arch=gfx950", "--cuda-device-only", "-S", "-O3", "-std=c++17",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
               "-I", os.path.join(ROOT, "include"), "-I", CSRC, src, "-o", str(dst)]
        subprocess.run(cmd, check=True, capture_output=True)
        out[os.path.basename(src)] = dst.read_text()
    return out


def test_no_packed_shift_saturate(device_asm):
    for name, text in device_asm.items():
        assert "v_ashr_pk_u8_i32" not in text, name


def test_no_scratch(device_asm):
    for name, text in device_asm.items():
        sizes = [int(v) for v in re.findall(r"\.private_segment_fixed_size:\s+(\d+)", text)]
        assert sizes and max(sizes) == 0, (name, sizes)
