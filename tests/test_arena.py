"""The serving loop's shadow arena allocator (host code) on the CPU: random
allocate / release sequences against a bitmap of the arena (first fit,
failure exactly when no free run fits, no overlap, maximal free runs)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2401_04701_amd", "csrc")


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path_factory.mktemp("arena") / "arena_check")
    subprocess.run([gxx, "-O2", "-std=c++17", "-I", CSRC, os.path.join(HERE, "arena_check.cpp"),
                    "-o", exe], check=True)
    return exe


@pytest.mark.parametrize("size,steps,seed", [(64, 20000, 1), (512, 20000, 2), (4096, 5000, 3),
                                             (3, 2000, 4)])
def test_arena_against_bitmap(checker, size, steps, seed):
    r = subprocess.run([checker, str(size), str(steps), str(seed)], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 0 and r.stdout.startswith("ok"), r.stdout + r.stderr
