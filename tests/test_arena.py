"""The serving loop's output-arena allocator (csrc/arena.h), exercised by a
randomized C++ self-check built with g++: no overlap, in range, and the
free space coalesces back into one block."""
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2407_19396_amd", "csrc")


@pytest.fixture(scope="module")
def binary(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("arena") / "arena_check")
    subprocess.run(["g++", "-O2", "-std=c++17", "-I", CSRC, os.path.join(HERE, "arena_check.cpp"),
                    "-o", out], check=True)
    return out


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_arena_random_alloc_free(binary, seed):
    r = subprocess.run([binary, str(seed)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.strip() == "ok"
