"""Host-side checks of the index maps the kernels share (CPU only): the
propagator table's slots with the (lx, ly) <-> (ly, lx) sharing when 4 | N
(every class reaches a slot, shared slots are read through the reflection
exactly when lx > ly, the slot-to-class inverse round-trips) and the
row-blocked spectrum layout (a bijection).  The program includes the
library's internal header and is compiled for the host only."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.mark.skipif(shutil.which(HIPCC) is None and not os.path.exists(HIPCC), reason="hipcc not available")
def test_table_slots_and_row_blocks(tmp_path):
    exe = tmp_path / "slots"
    src = os.path.join(ROOT, "tests", "host_index", "slots.cpp")
    r = subprocess.run([HIPCC, "-std=c++17", "-O1", "-x", "hip", "--offload-host-only",
                        "-I", os.path.join(ROOT, "paper_1304_2062_amd", "csrc"), "-I", os.path.join(ROOT, "include"),
                        src, "-o", str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "bad 0" in r.stdout
