"""Guards on the gfx950 code the library's kernels compile to (CPU only).

* The integer epilogue must not use v_ashr_pk_u8_i32: the compiler ORs the
  whole destination register afterwards while the instruction leaves the
  upper half holding the sign bits of a negative sum, which corrupts the
  neighbouring bytes (seen as saturated pixels after negative-lobe sums).
* No kernel may use scratch (private segment) memory.
* No matrix-core instruction may sit under a narrowed EXEC mask: MFMA
  ignores EXEC, so a product that control flow meant to skip (a K-step a
  block does not have) would still be accumulated. Seen when a block loop's
  bound lived in a vector register and the loop became divergent.
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


def _masked_mfma(text):
    """MFMAs whose basic block narrowed EXEC before them without restoring it."""
    found = []
    lines = text.split("\n")
    for i, line in enumerate(lines):
        if "v_mfma" not in line:
            continue
        j = i - 1
        while j >= 0:
            t = lines[j].strip()
            if re.match(r"^[.\w$]+:", t):  # a block label (maybe followed by a comment)
                break
            if t.startswith("s_or_b64 exec") or t.startswith("s_mov_b64 exec, -1"):
                break
            if t.startswith(("s_and_saveexec", "s_and_b64 exec", "s_andn2_b64 exec", "s_andn2_saveexec")):
                found.append((i, t, line.strip()))
                break
            j -= 1
    return found


def test_no_mfma_under_exec_mask(device_asm):
    for name, text in device_asm.items():
        assert not _masked_mfma(text), (name, _masked_mfma(text)[:4])


def test_mask_scan_finds_a_masked_mfma():
    # the scan itself, on a hand-made block
    block = "\n".join(["BB0_1:", "\ts_and_saveexec_b64 s[6:7], s[12:13]",
                       "\tv_mfma_i32_16x16x64_i8 v[26:29], v[18:21], v[2:5], v[26:29]", "\ts_or_b64 exec, exec, s[6:7]",
                       "\tv_mfma_i32_16x16x64_i8 v[26:29], v[18:21], v[2:5], v[26:29]"])
    assert len(_masked_mfma(block)) == 1
