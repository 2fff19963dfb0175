"""The shot server's arena allocator (csrc/fd_arena.h), built on the host with gcc under
AddressSanitizer and UndefinedBehaviorSanitizer and checked against a brute-force
first-fit model (tests/cpp/test_arena.cpp): same offsets, no overlap, holes equal to the
free runs, everything merged back after the last release."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_arena_against_first_fit_model(tmp_path):
    exe = tmp_path / "test_arena"
    cmd = ["g++", "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
           "-I", os.path.join(ROOT, "paper_2506_02486_amd", "csrc"),
           os.path.join(ROOT, "tests", "cpp", "test_arena.cpp"), "-o", str(exe)]
    subprocess.run(cmd, check=True, capture_output=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.strip() == "ok"


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_buddy_allocator_and_stream_pool_against_models(tmp_path):
    """The shot server's buddy allocator and bounded admission stream pool
    (csrc/fd_arena.h, csrc/fd_stream_pool.h) under ASan/UBSan against brute-force
    models (tests/cpp/test_buddy_pool.cpp): free blocks always the maximal free aligned
    blocks, each allocation the lowest block of the smallest fitting order, everything
    merged back; the pool reuses idle streams, creates lazily up to its bound, and at
    the bound releases the older half of the completed streams or waits for the
    oldest."""
    exe = tmp_path / "test_buddy_pool"
    cmd = ["g++", "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
           "-I", os.path.join(ROOT, "paper_2506_02486_amd", "csrc"),
           os.path.join(ROOT, "tests", "cpp", "test_buddy_pool.cpp"), "-o", str(exe)]
    subprocess.run(cmd, check=True, capture_output=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-2000:]
    assert r.stdout.strip() == "ok"
