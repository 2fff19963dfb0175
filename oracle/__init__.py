"""FP64 CPU oracle of the acoustic isotropic finite-difference hot path.

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
benchmark's CPU-baseline leg, never by the product package.  It shares no code with
the HIP path; the only thing both sides consume is the seeded input data of
``workloads``.

The compiled part is ``fd_oracle.c`` (plain loops, FP64, OpenMP over z planes),
loaded with ctypes.  This module adds the composition the paper's method implies
(Sec. 4.5, Minimod acoustic isotropic kernel): a Courant-number time step, a Ricker
source, a quadratic damping sponge, and the forward / adjoint sweeps.  Interior
arrays are C-ordered ``(nz, ny, nx)``; padded FP64 boxes carry a 4-cell halo.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fd_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

H = 4
COURANT = 0.4
F0 = 15.0
SPONGE_R = 1e-3

_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_fp = np.ctypeslib.ndpointer(dtype=np.float32, flags="C_CONTIGUOUS")
_ip = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")


def build(force: bool = True) -> str:
    """Compile ``fd_oracle.c`` into ``liboracle.so`` with gcc (no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c99",
                               "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _nullable(ptype):
    """ctypes argtype accepting either an ndarray or None (NULL)."""
    class _T(ptype):
        @classmethod
        def from_param(cls, obj):
            if obj is None:
                return None
            return ptype.from_param(obj)
    return _T


_dpn = _nullable(_dp)
_ipn = _nullable(_ip)


def lib():
    """The compiled oracle.  ``ORACLE_LIB`` in the environment names another build
    of it to load instead (the mutation test loads deliberately broken copies)."""
    global _lib
    if _lib is None:
        alt = os.environ.get("ORACLE_LIB")
        if alt:
            L = C.CDLL(alt)
        else:
            build(force=False)
            L = C.CDLL(_LIB)
        i32, i64, f64 = C.c_int, C.c_int64, C.c_double
        L.ora_elems.restype = i64
        L.ora_elems.argtypes = [i32, i32, i32]
        L.ora_cfl_dt.restype = f64
        L.ora_cfl_dt.argtypes = [_fp, i64, f64, f64]
        L.ora_ricker.restype = None
        L.ora_ricker.argtypes = [_dp, i32, i32, f64, f64, f64]
        L.ora_sponge_sigma_max.restype = f64
        L.ora_sponge_sigma_max.argtypes = [f64, f64, i32, f64]
        L.ora_sponge_eta.restype = None
        L.ora_sponge_eta.argtypes = [_dp, i32, i32, f64, f64]
        L.ora_fill_halo_periodic.restype = None
        L.ora_fill_halo_periodic.argtypes = [i32, i32, i32, _dp]
        L.ora_laplacian.restype = None
        L.ora_laplacian.argtypes = [i32, i32, i32, f64, f64, f64, _dp, _dp]
        L.ora_step.restype = None
        L.ora_step.argtypes = [i32, i32, i32, f64, f64, f64, _dp, _dp, _dp, _dp,
                               _dpn, _dpn, _dpn]
        L.ora_vdt2.restype = None
        L.ora_vdt2.argtypes = [i32, i32, i32, _fp, f64, _dp]
        L.ora_forward.restype = i32
        L.ora_forward.argtypes = [i32, i32, i32, f64, f64, f64, _dp, i32, _dpn,
                                  i32, i32, i32, _dpn, _dpn, _dpn, i32, i32, _ipn,
                                  _dpn, _dpn, _dpn]
        L.ora_step_points.restype = None
        L.ora_step_points.argtypes = [i32, i32, i32, f64, f64, f64, _fp, _fp, _dp,
                                      _dpn, _dpn, _dpn, i32, f64, i32, i32, i32, i32,
                                      _ip, _dp]
        L.ora_adjoint_step.restype = None
        L.ora_adjoint_step.argtypes = [i32, i32, i32, f64, f64, f64, _dpn, _dp, _dp, _dp,
                                       _dpn, _dpn, _dpn, i32, _dpn, _dpn, f64, i32, i32,
                                       i32]
        L.ora_fwi_gradient.restype = f64
        L.ora_fwi_gradient.argtypes = [i32, i32, i32, f64, f64, f64, _dp, f64, i32, _dpn,
                                       i32, i32, i32, _dpn, _dpn, _dpn, i32, i32, _ipn,
                                       _dp, _dpn, _dpn, _dpn, _dpn]
        vp = C.c_void_p
        L.ora_block_gemm.restype = None
        L.ora_block_gemm.argtypes = [i64, i64, i64, vp, i64, vp, i64, vp, i64, i32]
        L.ora_threads.restype = i32
        L.ora_threads.argtypes = []
        L.ora_set_threads.restype = None
        L.ora_set_threads.argtypes = [i32]
        _lib = L
    return _lib


def threads() -> int:
    """OpenMP threads the oracle's parallel loops use."""
    return lib().ora_threads()


def set_threads(n: int) -> None:
    """Use ``n`` OpenMP threads in later oracle calls."""
    lib().ora_set_threads(int(n))


# ------------------------------------------------------------------ layout helpers

def padded_shape(nx, ny, nz):
    return (nz + 2 * H, ny + 2 * H, nx + 2 * H)


def to_box(a: np.ndarray) -> np.ndarray:
    """Interior (nz,ny,nx) -> zero-halo FP64 box (nz+8,ny+8,nx+8)."""
    nz, ny, nx = a.shape
    b = np.zeros(padded_shape(nx, ny, nz), dtype=np.float64)
    b[H:-H, H:-H, H:-H] = a
    return b


def interior(b: np.ndarray) -> np.ndarray:
    return b[H:-H, H:-H, H:-H]


# ------------------------------------------------------------------ setup steps

def cfl_dt(v: np.ndarray, dmin: float, courant: float = COURANT) -> float:
    """dt = courant * min(d) / max(v)."""
    v = np.ascontiguousarray(v, dtype=np.float32)
    return lib().ora_cfl_dt(v, v.size, dmin, courant)


def ricker(nt: int, dt: float, f0: float = F0, t0: float | None = None,
           n0: int = 0) -> np.ndarray:
    """Ricker wavelet at t = (n0+n) dt, n < nt; the delay t0 defaults to 1/f0."""
    if t0 is None:
        t0 = 1.0 / f0
    w = np.empty(nt, dtype=np.float64)
    lib().ora_ricker(w, nt, n0, dt, f0, t0)
    return w


def sponge_eta(n: int, width: int, vmax: float, d: float, dt: float,
               R: float = SPONGE_R) -> np.ndarray:
    """eta = (dt/2) sigma for one axis; sigma quadratic over the ``width`` outer cells."""
    smax = lib().ora_sponge_sigma_max(vmax, d, width, R)
    eta = np.empty(n, dtype=np.float64)
    lib().ora_sponge_eta(eta, n, width, smax, dt)
    return eta


def sponge_tables(nx, ny, nz, width, vmax, d, dt, R=SPONGE_R):
    """(eta_x, eta_y, eta_z) or (None, None, None) when width == 0."""
    if width <= 0:
        return None, None, None
    dx, dy, dz = d
    return (sponge_eta(nx, width, vmax, dx, dt, R), sponge_eta(ny, width, vmax, dy, dt, R),
            sponge_eta(nz, width, vmax, dz, dt, R))


# ------------------------------------------------------------------ operators

def laplacian(box: np.ndarray, d=(10.0, 10.0, 10.0)) -> np.ndarray:
    """L applied to a padded FP64 box (halo used as given); returns the interior."""
    box = np.ascontiguousarray(box, dtype=np.float64)
    nz, ny, nx = (s - 2 * H for s in box.shape)
    out = np.zeros_like(box)
    lib().ora_laplacian(nx, ny, nz, *d, box, out)
    return interior(out).copy()


def fill_halo_periodic(box: np.ndarray) -> np.ndarray:
    box = np.ascontiguousarray(box, dtype=np.float64)
    nz, ny, nx = (s - 2 * H for s in box.shape)
    lib().ora_fill_halo_periodic(nx, ny, nz, box)
    return box


def step_box(up, u, vdt2, d=(10.0, 10.0, 10.0), eta=(None, None, None)):
    """One update on padded FP64 boxes (halo of u as given); returns the new box."""
    nz, ny, nx = (s - 2 * H for s in u.shape)
    un = np.zeros_like(u)
    lib().ora_step(nx, ny, nz, *d, np.ascontiguousarray(up), np.ascontiguousarray(u), un,
                   np.ascontiguousarray(vdt2), *eta)
    return un


def vdt2(v: np.ndarray, dt: float) -> np.ndarray:
    v = np.ascontiguousarray(v, dtype=np.float32)
    nz, ny, nx = v.shape
    out = np.empty(v.shape, dtype=np.float64)
    lib().ora_vdt2(nx, ny, nz, v, dt, out)
    return out


# ------------------------------------------------------------------ full runs

def forward(v: np.ndarray | None, nt: int, dt: float, d=(10.0, 10.0, 10.0), src=None,
            w: np.ndarray | None = None, eta=(None, None, None), periodic=False,
            rec: np.ndarray | None = None, state=None, q: np.ndarray | None = None):
    """Run ``nt`` steps.  ``src`` = (i,j,k) with wavelet ``w`` (len nt), ``rec`` an
    int32 (nrec,3) array, ``state`` = (u_prev, u) interior float64 arrays or None.
    ``q`` (FP64 interior vdt2) overrides ``v``/``dt`` when given.
    Returns (traces (nt,nrec) float64, u_prev, u) after the last step."""
    if q is None:
        q = vdt2(v, dt)
    q = np.ascontiguousarray(q, dtype=np.float64)
    nz, ny, nx = q.shape
    if rec is None:
        rec = np.zeros((0, 3), dtype=np.int32)
    rec = np.ascontiguousarray(rec, dtype=np.int32)
    nrec = rec.shape[0]
    traces = np.zeros((nt, max(nrec, 1)), dtype=np.float64)
    if state is None:
        up = np.zeros((nz, ny, nx))
        u = np.zeros((nz, ny, nx))
    else:
        up = np.array(state[0], dtype=np.float64, order="C", copy=True)
        u = np.array(state[1], dtype=np.float64, order="C", copy=True)
    if src is None or w is None:
        si = sj = sk = -1
        wa = None
    else:
        si, sj, sk = (int(x) for x in src)
        wa = np.ascontiguousarray(w[:nt], dtype=np.float64)
    rc = lib().ora_forward(nx, ny, nz, *d, q, nt, wa, si, sj, sk, *eta,
                           1 if periodic else 0, nrec, rec if nrec else None,
                           traces if nrec else None, up, u)
    if rc != 0:
        raise MemoryError("oracle forward: out of memory")
    return traces[:, :nrec], up, u


def step_points(up: np.ndarray, u: np.ndarray, q: np.ndarray,
                pts: np.ndarray, d=(10.0, 10.0, 10.0), eta=(None, None, None),
                periodic=False, src=None, w_src: float = 0.0) -> np.ndarray:
    """u^{n+1} at selected points from float32 interior arrays of u^{n-1}, u^n and
    the FP64 interior vdt2 ``q``."""
    up = np.ascontiguousarray(up, dtype=np.float32)
    u = np.ascontiguousarray(u, dtype=np.float32)
    q = np.ascontiguousarray(q, dtype=np.float64)
    pts = np.ascontiguousarray(pts, dtype=np.int32)
    nz, ny, nx = u.shape
    out = np.empty(pts.shape[0], dtype=np.float64)
    si, sj, sk = src if src is not None else (-1, -1, -1)
    lib().ora_step_points(nx, ny, nz, *d, up, u, q, *eta, 1 if periodic else 0,
                          float(w_src), si, sj, sk, pts.shape[0], pts, out)
    return out


def adjoint_step(c2, c, vdt2_int, d=(10.0, 10.0, 10.0), eta=(None, None, None),
                 periodic=False, u_n=None, g=None, w=0.0, src=None):
    """Transpose of one forward step (interior arrays in, interior out):
    a = 2Dc + L(QDc) - E D c2; optionally g += D c (L u_n + f).  ``u_n`` is an
    interior array; its halo is zero or periodic per ``periodic``.  Returns (a, g)."""
    nz, ny, nx = c.shape
    cb = to_box(c)
    c2b = to_box(c2) if c2 is not None else None
    qb = to_box(vdt2_int)
    out = np.zeros_like(cb)
    ub = None
    gb = None
    if u_n is not None:
        ub = to_box(u_n)
        if periodic:
            lib().ora_fill_halo_periodic(nx, ny, nz, ub)
        gb = to_box(g) if g is not None else np.zeros_like(cb)
    si, sj, sk = src if src is not None else (-1, -1, -1)
    lib().ora_adjoint_step(nx, ny, nz, *d, c2b, cb, out, qb, *eta, 1 if periodic else 0,
                           ub, gb, float(w), si, sj, sk)
    return interior(out).copy(), (interior(gb).copy() if gb is not None else None)


def fwi_gradient(v: np.ndarray | None, nt: int, dt: float, obs: np.ndarray, src, w,
                 rec: np.ndarray, d=(10.0, 10.0, 10.0), eta=(None, None, None),
                 periodic=False, q: np.ndarray | None = None):
    """Adjoint-state gradient with full storage.  ``q`` (FP64 interior vdt2)
    overrides ``v`` when given.  Returns a dict with J, traces, g_vdt2, grad_m
    (interior arrays) and grad_w (dJ/dw per step)."""
    if q is None:
        q = vdt2(v, dt)
    q = np.ascontiguousarray(q, dtype=np.float64)
    nz, ny, nx = q.shape
    rec = np.ascontiguousarray(rec, dtype=np.int32)
    nrec = rec.shape[0]
    obs = np.ascontiguousarray(obs, dtype=np.float64).reshape(nt, nrec)
    traces = np.zeros((nt, nrec))
    g = np.zeros((nz, ny, nx))
    gm = np.zeros((nz, ny, nx))
    gw = np.zeros(nt)
    si, sj, sk = src
    J = lib().ora_fwi_gradient(nx, ny, nz, *d, q, dt, nt,
                               np.ascontiguousarray(w[:nt], dtype=np.float64), si, sj, sk,
                               *eta, 1 if periodic else 0, nrec, rec, obs, traces, g, gm, gw)
    if J < 0:
        raise MemoryError("oracle gradient: out of memory")
    return {"J": J, "traces": traces, "g_vdt2": g, "grad_m": gm, "grad_w": gw}


# ------------------------------------------------- Cannon's matrix multiply (Sec. 4.4)

def _rows(x: np.ndarray, name: str) -> int:
    """Leading dimension (elements) of a 2-D FP64 array with unit column stride."""
    if x.dtype != np.float64 or x.ndim != 2:
        raise ValueError(f"{name}: a 2-D float64 array is needed")
    if x.size == 0:
        return max(x.shape[1], 1)
    if x.shape[1] > 1 and x.strides[1] != 8:
        raise ValueError(f"{name}: unit column stride is needed")
    return x.strides[0] // 8 if x.shape[0] > 1 else max(x.shape[1], 1)


def block_gemm(a: np.ndarray, b: np.ndarray, c: np.ndarray | None = None,
               accumulate: bool = False) -> np.ndarray:
    """The local block product of one Cannon step, by its definition (ora_block_gemm):
    c = (c if accumulate else 0) + a @ b in FP64, each element summed over the inner
    index in increasing order.  ``a`` (m, k), ``b`` (k, n), ``c`` (m, n) may be row
    views of larger arrays; ``c`` is written in place and returned."""
    m, k = a.shape
    k2, n = b.shape
    if k != k2:
        raise ValueError("block_gemm: inner dimensions differ")
    if c is None:
        c = np.zeros((m, n))
        accumulate = False
    if c.shape != (m, n):
        raise ValueError("block_gemm: c has the wrong shape")
    lib().ora_block_gemm(m, n, k, a.ctypes.data, _rows(a, "a"), b.ctypes.data, _rows(b, "b"),
                         c.ctypes.data, _rows(c, "c"), 1 if accumulate else 0)
    return c


def cannon_order(rank: int, P: int) -> list:
    """The B row stripes rank ``rank`` multiplies with, in step order: it starts with
    its own stripe and receives its neighbour's after every step (a ring)."""
    return [(rank + s) % P for s in range(P)]


def cannon(A: np.ndarray, B: np.ndarray, P: int) -> np.ndarray:
    """C = A @ B by Cannon's algorithm on P simulated ranks (Sec. 4.4): with Ns = N/P,
    rank r holds the row stripes A_r, B_r and C_r (Ns x N); at each of its P steps it
    adds A_r[:, q*Ns:(q+1)*Ns] @ B_q (a product of N * Ns * Ns multiply-adds) to C_r,
    where B_q is the stripe it holds, then passes that stripe around the ring."""
    N = A.shape[0]
    if A.shape != (N, N) or B.shape != (N, N) or P < 1 or N % P:
        raise ValueError("cannon: square N x N operands with N divisible by P are needed")
    ns = N // P
    A = np.ascontiguousarray(A, dtype=np.float64)
    B = np.ascontiguousarray(B, dtype=np.float64)
    C = np.zeros((N, N))
    held = list(range(P))  # the B stripe each rank holds
    for _ in range(P):
        for r in range(P):
            q = held[r]
            block_gemm(A[r * ns:(r + 1) * ns, q * ns:(q + 1) * ns], B[q * ns:(q + 1) * ns, :],
                       C[r * ns:(r + 1) * ns, :], accumulate=True)
        held = [held[(r + 1) % P] for r in range(P)]  # each rank receives from r + 1
    return C

