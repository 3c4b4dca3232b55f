"""The serving layer's admission logic (first-fit arena over the ciphertext
budget, in-order batch formation) on the CPU: tests/sched_driver.cpp is built
with g++ against the same header the server uses and run."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_scheduler_logic(tmp_path):
    exe = tmp_path / "sched_driver"
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-Wextra", "-Werror",
                    "-I", os.path.join(ROOT, "paper_2003_05328_amd", "csrc"), "-I", os.path.join(ROOT, "include"),
                    os.path.join(ROOT, "tests", "sched_driver.cpp"), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "sched checks ok" in out.stdout
