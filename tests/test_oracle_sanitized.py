"""Run every oracle entry point under AddressSanitizer and UndefinedBehaviorSanitizer
(host build with gcc, small grids including 1x1x1 and halos wider than the grid)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_sanitizers(tmp_path):
    exe = tmp_path / "ora_san"
    cmd = ["gcc", "-O1", "-g", "-std=c99", "-fopenmp", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
           os.path.join(ROOT, "oracle", "fd_oracle.c"),
           os.path.join(ROOT, "oracle", "sanitize_driver.c"), "-o", str(exe), "-lm"]
    subprocess.run(cmd, check=True, capture_output=True)
    env = dict(os.environ, OMP_NUM_THREADS="2", ASAN_OPTIONS="detect_leaks=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "ok" in r.stdout
