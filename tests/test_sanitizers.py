"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer.

The CPU oracle is rebuilt with -fsanitize=address,undefined (every report
fatal) and driven through every entry point (all families, all six
observation modes, external actions and the random policy, layouts,
exhaustive short action sequences from the 5x5 starts) in a child process
that preloads the sanitizer runtime; its outputs must equal the ordinary
build's bit for bit.  The serving loop's output-arena allocator runs its
randomized self-check under the same sanitizers."""
import os
import subprocess
import sys

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2407_19396_amd", "csrc")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g"]


def _libasan():
    p = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


def _run_driver(path, env_extra):
    env = dict(os.environ, **env_extra)
    r = subprocess.run([sys.executable, os.path.join(HERE, "sanitize_driver.py"), path], env=env,
                       capture_output=True, text=True, timeout=900)
    assert r.returncode == 0, r.stdout[-4000:] + r.stderr[-4000:]
    return np.load(path)


@pytest.mark.skipif(_libasan() is None, reason="gcc's AddressSanitizer runtime is not installed")
def test_oracle_under_asan_ubsan_equals_plain_build(tmp_path):
    import oracle
    san = oracle.build(force=True, sanitize=True)
    plain = oracle.build(force=False)
    a = _run_driver(str(tmp_path / "san.npz"),
                    {"OX_ORACLE_LIB": san, "LD_PRELOAD": _libasan(),
                     "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1",
                     "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1", "OMP_NUM_THREADS": "2"})
    b = _run_driver(str(tmp_path / "plain.npz"), {"OX_ORACLE_LIB": plain, "OMP_NUM_THREADS": "2"})
    assert sorted(a.files) == sorted(b.files) and len(a.files) > 50
    for k in a.files:
        assert np.array_equal(a[k], b[k]), k


@pytest.mark.parametrize("seed", [1, 2])
def test_arena_under_asan_ubsan(tmp_path, seed):
    out = str(tmp_path / "arena_check_san")
    subprocess.run(["g++", "-O1", "-std=c++17", *SAN, "-I", CSRC, os.path.join(HERE, "arena_check.cpp"),
                    "-o", out], check=True)
    r = subprocess.run([out, str(seed)], capture_output=True, text=True, timeout=300,
                       env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1"))
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.strip() == "ok"
