"""The host planner's own self-check (tests/native/plan_selfcheck.cpp), built
with g++ and run plain, under AddressSanitizer (+ UndefinedBehaviorSanitizer)
and under ThreadSanitizer: plans built on four threads at once equal plans
built alone, every pass schedule passes the CREW check, and each schedule
corrupted in one place fails it."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = [os.path.join(ROOT, "tests", "native", "plan_selfcheck.cpp"),
       os.path.join(ROOT, "paper_2608_01332_amd", "csrc", "plan.cpp")]


@pytest.mark.parametrize("mode", ["plain", "asan", "tsan"])
def test_planner_selfcheck(mode, tmp_path):
    if shutil.which("g++") is None:
        pytest.skip("g++ is not available")
    flags = {"plain": ["-O2"], "asan": ["-O1", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer"],
             "tsan": ["-O1", "-g", "-fsanitize=thread"]}[mode]
    exe = str(tmp_path / f"plan_selfcheck_{mode}")
    b = subprocess.run(["g++", "-std=c++17", "-pthread"] + flags + SRC + ["-o", exe], capture_output=True, text=True)
    assert b.returncode == 0, b.stderr[-4000:]
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=1:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    env["TSAN_OPTIONS"] = "halt_on_error=1"
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "plan self-check OK" in r.stdout
