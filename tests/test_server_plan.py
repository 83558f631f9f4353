"""The serving loop's scheduling on the CPU (no GPU): the range sets, the arena
free list and the batch choice of paper_1605_00561_amd/csrc/server_plan.h,
driven by tests/server_plan_check.cpp (built here with g++, with ASan and
UBSan).  The GPU tests check the same loop end to end."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_server_plan(tmp_path):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path / "server_plan_check")
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-Wall", "-Wextra", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=all", "-I", os.path.join(ROOT, "paper_1605_00561_amd", "csrc"),
                    os.path.join(ROOT, "tests", "server_plan_check.cpp"), "-o", exe],
                   check=True, capture_output=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120,
                       env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1"))
    assert r.returncode == 0, r.stderr
    assert r.stdout.startswith("ok "), r.stdout
    assert int(r.stdout.split()[1]) > 100
