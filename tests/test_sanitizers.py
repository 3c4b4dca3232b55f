"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (no GPU).

The CPU oracle (driven by tests/oracle_driver.c through every function it
exports) and the serving layer's host-side scheduling core (driven by
tests/sched_driver.cpp, with a fake executor in place of the device) are
built with -fsanitize=address,undefined and run; any finding aborts the run.
"""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]
# the sanitizer runtime must not insist on being first in the preload list of
# whatever environment runs the test
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0", UBSAN_OPTIONS="print_stacktrace=1")


def _run(exe, marker):
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300, env=ENV)
    assert out.returncode == 0, out.stdout + out.stderr
    assert marker in out.stdout
    assert "runtime error" not in out.stderr, out.stderr


def test_oracle_under_sanitizers(tmp_path):
    exe = tmp_path / "oracle_driver"
    subprocess.run(["gcc", "-std=c11", *SAN, "-fopenmp", "-Wall", "-Wextra",
                    os.path.join(ROOT, "oracle", "ensei_oracle.c"), os.path.join(ROOT, "tests", "oracle_driver.c"),
                    "-o", str(exe)], check=True)
    _run(exe, "oracle driver ok")


def test_scheduler_under_sanitizers(tmp_path):
    exe = tmp_path / "sched_driver_san"
    subprocess.run(["g++", "-std=c++17", *SAN, "-pthread", "-Wall", "-Wextra", "-Werror",
                    "-I", os.path.join(ROOT, "paper_2003_05328_amd", "csrc"), "-I", os.path.join(ROOT, "include"),
                    os.path.join(ROOT, "tests", "sched_driver.cpp"), "-o", str(exe)], check=True)
    _run(exe, "sched checks ok")
