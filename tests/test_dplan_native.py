"""The device planner's program (paper_2608_01332_amd/csrc/dplan.hpp) run on
the CPU by its sequential executor (tests/native/dplan_emul.cpp), plain and
under AddressSanitizer + UndefinedBehaviorSanitizer (host code only): every
statistic and schedule equals the host planner's with the list-rank
selection, for 1024 threads (the GPU's), 37 and 1, each in three orders of the
threads within a phase, with sibling groups built by one thread each and by
the whole workgroup, and invalid trees get the host's status."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
SRC = [os.path.join(ROOT, "tests", "native", "dplan_emul.cpp"),
       os.path.join(ROOT, "paper_2608_01332_amd", "csrc", "plan.cpp")]


@pytest.mark.parametrize("mode", ["plain", "asan"])
def test_device_planner_program_on_cpu(mode, tmp_path):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc is not available")
    flags = {"plain": ["-O2"],
             "asan": ["-O1", "-g", "-Xarch_host", "-fsanitize=address,undefined", "-fno-omit-frame-pointer"]}[mode]
    exe = str(tmp_path / f"dplan_emul_{mode}")
    b = subprocess.run([HIPCC, "-x", "hip", "-std=c++17", "--offload-arch=gfx950", "-pthread"] + flags + SRC
                       + ["-o", exe], capture_output=True, text=True)
    assert b.returncode == 0, b.stderr[-4000:]
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=1:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=900)
    assert r.returncode == 0, (r.stdout + r.stderr)[-4000:]
    assert "device planner emulation OK" in r.stdout
