"""CPU check of the persistent step kernel's device-wide barrier logic.

The barrier (paper_1602_02694_amd/csrc/grid_sync.hpp) is one template used by
the kernel with device atomics; tests/grid_sync_check.cpp instantiates it with
host atomics and runs it on threads: ordering across 3000 epochs, and that a
participant that never arrives makes every other one leave within its poll
bound with the failure flag set (so a kernel can never wait forever).
"""

import os
import subprocess

from conftest import ROOT


def test_grid_barrier_logic_on_host_threads(tmp_path):
    src = os.path.join(ROOT, "tests", "grid_sync_check.cpp")
    inc = os.path.join(ROOT, "paper_1602_02694_amd", "csrc")
    exe = str(tmp_path / "grid_sync_check")
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-pthread", "-I" + inc, src, "-o", exe])
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
