"""Host-only checks of the GPU library's index arithmetic (no GPU needed)."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))


def test_fastdiv_and_key_permutation(tmp_path):
    exe = str(tmp_path / "layout_check")
    subprocess.run(["/opt/rocm/bin/hipcc", "-O2", "-std=c++17", "-x", "hip", "--offload-arch=gfx950",
                    os.path.join(HERE, "host", "layout_check.cpp"), "-o", exe],
                   check=True, capture_output=True)
    r = subprocess.run([exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr


def test_serving_arena(tmp_path):
    exe = str(tmp_path / "arena_check")
    subprocess.run(["g++", "-O2", "-std=c++17", os.path.join(HERE, "host", "arena_check.cpp"), "-o", exe],
                   check=True, capture_output=True)
    r = subprocess.run([exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr


def test_serving_scheduler(tmp_path):
    """Admission, batch formation and per-stream ordering of the serving
    runtime, driven by a stand-in device that finishes batches in random order
    and flags any two batches in flight that touch the same ring slot or leaf
    set with a write."""
    exe = str(tmp_path / "serve_sched_check")
    subprocess.run(["g++", "-O2", "-std=c++17", os.path.join(HERE, "host", "serve_sched_check.cpp"), "-o", exe],
                   check=True, capture_output=True)
    r = subprocess.run([exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
