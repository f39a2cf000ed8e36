"""The serving scheduler (continuous batching, memory-based admission) built
for the host alone with AddressSanitizer and UndefinedBehaviorSanitizer and
driven by a mock executor on a fake clock (tests/sched_fake_clock.cpp)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def test_scheduler_fake_clock_under_sanitizers(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path / "sched_fake_clock")
    src = [os.path.join(HERE, "sched_fake_clock.cpp"), os.path.join(ROOT, "paper_2306_08792_amd", "csrc", "scheduler.cpp")]
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", *src, "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    # verify_asan_link_order=0: the sanitizer runtime need not be the first
    # library loaded when the environment preloads another one
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "scheduler ok" in r.stdout
    print(r.stdout)
