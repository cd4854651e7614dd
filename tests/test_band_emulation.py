"""Host stepping of the row-band sweep kernel's per-thread code.

tests/band_emu.cpp includes the kernel's own per-thread code
(paper_0904_4887_amd/csrc/band_sweep.h), compiles it for the host with the
ROCm clang, and steps every thread of every block: each global and LDS access
is bounds-checked, the output must equal two in-place colour passes of the same
point update bit for bit, with both colour orders, float32 (4- and 2-wide
vectors) and float64, the zero-input variant, several band heights, chunk
lengths that do and do not divide the slab, and threads of a step run forwards
and backwards (one barrier per step means no thread may read what another
writes in the same step).
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_0904_4887_amd", "csrc")


def _clang():
    for c in ("/opt/rocm/llvm/bin/clang++", shutil.which("clang++")):
        if c and os.path.exists(c):
            return c
    return None


def test_band_sweep_steps_match_colour_passes(tmp_path):
    cxx = _clang()
    if cxx is None:
        pytest.skip("no clang++ (the per-thread code uses clang vector types)")
    exe = str(tmp_path / "band_emu")
    r = subprocess.run([cxx, "-O1", "-std=c++17", "-I", CSRC, os.path.join(HERE, "band_emu.cpp"), "-o", exe],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-2000:]
    assert r.stdout.rstrip().endswith("OK (0 failing cases)"), r.stdout[-2000:]
