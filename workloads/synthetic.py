"""Seeded synthetic workloads for the acoustic isotropic finite-difference hot path.

The paper runs its acoustic isotropic kernel on a 1200^3 grid for 1000 steps
(Sec. 4.5, Minimod) and publishes no velocity model, geometry or data, so every
input here is synthetic.  All arrays are C-ordered ``(nz, ny, nx)`` with x fastest,
float32 unless noted.  Nothing in this module computes any part of the method.
"""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import scipy.ndimage as ndi

__all__ = [
    "layered_velocity",
    "smooth_velocity",
    "blob_perturbed",
    "center_source",
    "receivers_plane",
    "receivers_xline",
    "serving_shots",
    "poisson_arrivals",
    "random_field",
    "fd_voxels",
]


def layered_velocity(nx: int, ny: int, nz: int, seed: int = 1, nlayers: int = 4,
                     v_top: float = 1500.0, v_step: float = 1000.0,
                     noise: float = 50.0) -> np.ndarray:
    """Layered model: layer ``l = floor(nlayers*k/nz)`` has ``v_top + v_step*l`` m/s,
    plus iid ``U(-noise, noise)`` drawn in float64 from ``default_rng(seed)`` in C order
    ``(nz, ny, nx)``, then cast to float32.  With the defaults the layers are
    1500/2500/3500/4500 m/s."""
    k = np.arange(nz)
    layer = (nlayers * k) // nz
    base = v_top + v_step * layer.astype(np.float64)
    rng = np.random.default_rng(seed)
    jitter = rng.uniform(-noise, noise, size=(nz, ny, nx))
    return (base[:, None, None] + jitter).astype(np.float32)


def _filter_axis(a: np.ndarray, axis: int, sigma: float, truncate: float,
                 workers: int) -> np.ndarray:
    """1-D Gaussian filter along ``axis`` with periodic wrap, split into independent
    slabs along another axis so several threads can work at once (scipy releases the
    GIL inside its line filters).  The result does not depend on ``workers``."""
    out = np.empty_like(a)
    split = 0 if axis != 0 else 1
    n = a.shape[split]
    bounds = np.linspace(0, n, max(1, min(workers, n)) + 1).astype(int)

    def run(lo_hi):
        lo, hi = lo_hi
        sl = [slice(None)] * 3
        sl[split] = slice(lo, hi)
        sl = tuple(sl)
        ndi.gaussian_filter1d(a[sl], sigma=sigma, axis=axis, mode="wrap",
                              truncate=truncate, output=out[sl])

    with ThreadPoolExecutor(max_workers=len(bounds) - 1) as ex:
        list(ex.map(run, zip(bounds[:-1], bounds[1:])))
    return out


def smooth_velocity(nx: int, ny: int, nz: int, seed: int = 2, sigma: float = 8.0,
                    vmin: float = 1500.0, vmax: float = 4500.0,
                    truncate: float = 4.0, workers: int | None = None) -> np.ndarray:
    """Smooth random model: float32 standard normal field from ``default_rng(seed)``
    (C order ``(nz, ny, nx)``), Gaussian-filtered with standard deviation ``sigma``
    cells along z, then y, then x (periodic wrap, kernel truncated at
    ``truncate*sigma``), then min-max scaled in float64 to exactly ``[vmin, vmax]``
    and cast to float32."""
    if workers is None:
        workers = min(16, os.cpu_count() or 1)
    rng = np.random.default_rng(seed)
    a = rng.standard_normal((nz, ny, nx), dtype=np.float32)
    for axis in (0, 1, 2):
        a = _filter_axis(a, axis, sigma, truncate, workers)
    lo = float(a.min())
    hi = float(a.max())
    scaled = vmin + (vmax - vmin) * ((a.astype(np.float64) - lo) / (hi - lo))
    out = scaled.astype(np.float32)
    # the endpoints are exact by construction; pin them against float rounding
    out[np.unravel_index(np.argmin(a), a.shape)] = np.float32(vmin)
    out[np.unravel_index(np.argmax(a), a.shape)] = np.float32(vmax)
    return out


def blob_perturbed(v: np.ndarray, center: tuple[int, int, int] | None = None,
                   radius: float = 16.0, amp: float = 0.05) -> np.ndarray:
    """``v * (1 + amp*exp(-|x-c|^2/(2 radius^2)))`` in float64, cast to float32;
    ``center`` is ``(i, j, k)`` in cells, the grid centre by default."""
    nz, ny, nx = v.shape
    if center is None:
        center = (nx // 2, ny // 2, nz // 2)
    ci, cj, ck = center
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    r2 = (i - ci) ** 2 + (j - cj) ** 2 + (k - ck) ** 2
    return (v.astype(np.float64) * (1.0 + amp * np.exp(-r2 / (2.0 * radius ** 2)))).astype(np.float32)


def center_source(nx: int, ny: int, nz: int) -> tuple[int, int, int]:
    """0-based interior index of the grid centre ``(nx//2, ny//2, nz//2)``."""
    return (nx // 2, ny // 2, nz // 2)


def receivers_plane(nx: int, ny: int, k: int) -> np.ndarray:
    """Every point of the plane ``z = k``: int32 ``(nx*ny, 3)`` rows ``(i, j, k)``,
    x fastest."""
    j, i = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    return np.stack([i.ravel(), j.ravel(), np.full(nx * ny, k)], axis=1).astype(np.int32)


def receivers_xline(nx: int, j: int, k: int) -> np.ndarray:
    """The x-line ``(0..nx-1, j, k)``: int32 ``(nx, 3)``."""
    i = np.arange(nx)
    return np.stack([i, np.full(nx, j), np.full(nx, k)], axis=1).astype(np.int32)


def serving_shots(n: int = 256, seed: int = 3, lo: int = 128, hi: int = 384,
                  margin: int = 16) -> list[dict]:
    """Shot geometries for the serving stream: ``nx, ny, nz`` iid uniform integers in
    ``[lo, hi]`` and a source uniform in ``[margin, n_a - margin)`` per axis, all from
    ``default_rng(seed)`` drawn shot by shot."""
    rng = np.random.default_rng(seed)
    shots = []
    for s in range(n):
        nx, ny, nz = (int(x) for x in rng.integers(lo, hi + 1, size=3))
        src = tuple(int(rng.integers(margin, m - margin)) for m in (nx, ny, nz))
        shots.append({"id": s, "nx": nx, "ny": ny, "nz": nz, "src": src})
    return shots


def poisson_arrivals(n: int, rate: float, seed: int = 4) -> np.ndarray:
    """Arrival times (seconds, float64, starting at 0) of a Poisson process of
    ``rate`` per second: cumulative sums of exponential gaps from ``default_rng(seed)``,
    shifted so the first arrival is at 0."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=n)
    t = np.cumsum(gaps)
    return t - t[0]


def random_field(shape: tuple[int, ...], seed: int, scale: float = 1.0,
                 dtype=np.float32) -> np.ndarray:
    """iid standard normal field times ``scale`` from ``default_rng(seed)``."""
    rng = np.random.default_rng(seed)
    return (scale * rng.standard_normal(shape)).astype(dtype)


def fd_voxels(weights: np.ndarray, count: int = 16, seed: int = 5,
              rel: float = 1e-2) -> np.ndarray:
    """Draw ``count`` distinct voxels (flat C-order indices) uniformly among those with
    ``|weights| >= rel * max|weights|``, from ``default_rng(seed)``."""
    w = np.abs(np.asarray(weights)).ravel()
    cand = np.flatnonzero(w >= rel * w.max())
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(cand, size=min(count, cand.size), replace=False))
