"""CPU code built with AddressSanitizer and UndefinedBehaviorSanitizer (gcc /
g++, host code only): the oracle's C interface on random small inputs, the
serving scheduler with its stand-in device, and the serving arena.  Any
out-of-bounds access, use after free, leak or undefined arithmetic aborts
the program and fails the test."""
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
FLAGS = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]

PROGRAMS = [
    ("oracle_sanitize.c", ["gcc", "-std=c11", "-pthread"]),
    ("serve_sched_check.cpp", ["g++", "-std=c++17"]),
    ("arena_check.cpp", ["g++", "-std=c++17"]),
]


@pytest.mark.parametrize("src,cc", PROGRAMS, ids=[p[0] for p in PROGRAMS])
def test_sanitized(tmp_path, src, cc):
    exe = str(tmp_path / "prog")
    subprocess.run(cc + FLAGS + [os.path.join(HERE, "host", src), "-o", exe], check=True, capture_output=True)
    env = dict(os.environ, ASAN_OPTIONS="abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, (r.stdout + r.stderr)[-4000:]
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-4000:]
