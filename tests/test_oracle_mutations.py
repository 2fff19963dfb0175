"""The oracle's pins catch plausible mistakes in the oracle itself.

Each case plants one mistake (a wrong weight, a wrong neighbour, a sign, a dropped
factor, a wrong wrap, ...) in a copy of ``oracle/fd_oracle.c``, builds the copy in a
temporary directory and runs the CPU pin suites against it (``ORACLE_LIB``); every
mutant must fail at least one pin.  The unmutated copy, built the same way, must pass.
Nothing here touches the GPU or the repository's own oracle build.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "fd_oracle.c")
PINS = ["tests/test_oracle_pins.py", "tests/test_oracle_adjoint.py", "tests/test_oracle_gemm.py"]

# (what the mistake is, exact text in the oracle, replacement)
MUTATIONS = [
    ("c4 weight", "-1.0 / 560.0", "-1.0 / 561.0"),
    ("wrong -m neighbour",
     "s += CM[m] * (u[c + m * st[a]] + u[c - m * st[a]]);",
     "s += CM[m] * (u[c + m * st[a]] + u[c - (m > 1 ? m - 1 : m) * st[a]]);"),
    ("sign of eta on u^{n-1}", "(1.0 - eta) * up[c]", "(1.0 + eta) * up[c]"),
    ("adjoint: dropped D on a^{n+2}", "old[q] = -(1.0 - eta) * c[q] / (1.0 + eta);",
     "old[q] = -(1.0 - eta) * c[q];"),
    ("adjoint: dropped D inside L", "p[q] = vdt2[q] * c[q] / (1.0 + eta_at(ex, ey, ez, i, j, k));",
     "p[q] = vdt2[q] * c[q];"),
    ("gradient: dropped source term", "if (i == si && j == sj && k == sk) lu += w;",
     "if (0) lu += w;"),
    ("periodic wrap off by one",
     "u[at(&b, nx - 1 + h, j, k)] = u[at(&b, wrap(nx - 1 + h, nx), j, k)];",
     "u[at(&b, nx - 1 + h, j, k)] = u[at(&b, wrap(nx - 2 + h, nx), j, k)];"),
    ("source without 1/(1+eta)",
     "un[c] += vdt2[c] * w / (1.0 + eta_at(ex, ey, ez, si, sj, sk));", "un[c] += vdt2[c] * w;"),
    ("linear sponge", "e = 0.5 * dt * sigma_max * r * r;", "e = 0.5 * dt * sigma_max * r;"),
    ("receivers sample u^n", "traces[(int64_t)n * nrec + r] = un", "traces[(int64_t)n * nrec + r] = u"),
    ("y spacing used for z", "b.iz2 = 1.0 / (dz * dz);", "b.iz2 = 1.0 / (dy * dy);"),
    ("Ricker without the factor 2", "w[n] = (1.0 - 2.0 * a) * exp(-a);",
     "w[n] = (1.0 - a) * exp(-a);"),
    ("gradient sign", "grad_m_out[o] = -g[q] * vdt2[q] * vdt2[q] / (dt * dt);",
     "grad_m_out[o] = g[q] * vdt2[q] * vdt2[q] / (dt * dt);"),
    ("gemm: inner index from 1",
     "for (int64_t p = 0; p < k; ++p) s += a[i * lda + p] * b[p * ldb + j];",
     "for (int64_t p = 1; p < k; ++p) s += a[i * lda + p] * b[p * ldb + j];"),
    ("gemm: B transposed", "s += a[i * lda + p] * b[p * ldb + j];",
     "s += a[i * lda + p] * b[j * ldb + p];"),
    ("gemm: accumulate ignored", "double s = accumulate ? c[i * ldc + j] : 0.0;",
     "double s = 0.0;"),
    ("gemm: row stride of A taken as k", "s += a[i * lda + p] * b[p * ldb + j];",
     "s += a[i * k + p] * b[p * ldb + j];"),
    ("point step: x and z spacing swapped",
     "const double id2[3] = {1.0 / (dx * dx), 1.0 / (dy * dy), 1.0 / (dz * dz)};",
     "const double id2[3] = {1.0 / (dz * dz), 1.0 / (dy * dy), 1.0 / (dx * dx)};"),
]


def _build(src_text: str, out_dir: str) -> str:
    c = os.path.join(out_dir, "fd_oracle.c")
    with open(c, "w") as f:
        f.write(src_text)
    so = os.path.join(out_dir, "liboracle.so")
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c99", "-o", so, c,
                           "-lm"])
    return so


def _pins_pass(so: str) -> bool:
    env = dict(os.environ, ORACLE_LIB=so, OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, "-m", "pytest", *PINS, "-x", "-q", "-p", "no:cacheprovider"],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    return r.returncode == 0


def test_every_planted_mistake_fails_a_pin(tmp_path):
    text = open(SRC).read()
    jobs = [("unmutated", text)]
    for name, old, new in MUTATIONS:
        assert text.count(old) == 1, f"mutation site not found once: {name}"
        jobs.append((name, text.replace(old, new)))
    dirs = []
    for i, (name, t) in enumerate(jobs):
        d = tmp_path / f"m{i}"
        d.mkdir()
        dirs.append(_build(t, str(d)))
    with ThreadPoolExecutor(max_workers=4) as ex:
        passed = list(ex.map(_pins_pass, dirs))
    assert passed[0], "the unmutated oracle copy must pass its pins"
    survivors = [name for (name, _), ok in zip(jobs[1:], passed[1:]) if ok]
    assert not survivors, f"mutations no pin catches: {survivors}"
