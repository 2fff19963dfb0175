"""Continuous-batching shot server (binding of the libfd shot-server C ABI).

``ShotServer`` owns a device arena (a torch byte tensor) and two HIP streams at the
default priority; the C++ server admits shots in submission order by footprint and
slot count and advances all admitted shots one step per batched launch.  ``PlainLoop``
is the comparison: the same kernels, one shot at a time in arrival order.
"""
from __future__ import annotations

import ctypes as C
import time

import numpy as np
import torch

from . import api
from ._lib import FD_ARENA_BUDDY, FD_EAGAIN, FD_ENOTFOUND, FD_OK, check, fd_shot_desc, lib


class Shot:
    """One forward-modelling shot: a device velocity view (nz, ny, nx) plus geometry."""

    def __init__(self, v: torch.Tensor, nt: int, dt: float, src, rec: np.ndarray | None = None,
                 d=(10.0, 10.0, 10.0), f0: float = api.RICKER_F0, t0: float | None = None,
                 sponge_width: int = 16, sponge_vmax: float = 0.0):
        if v.dtype != torch.float32 or not v.is_cuda or v.dim() != 3 or v.stride(2) != 1:
            raise TypeError("v must be a float32 ROCm view (nz, ny, nx) with unit x stride")
        self.v = v
        self.nt = int(nt)
        self.dt = float(dt)
        self.src = tuple(int(x) for x in src)
        self.rec = (np.zeros((0, 3), np.int32) if rec is None
                    else np.ascontiguousarray(rec, dtype=np.int32).reshape(-1, 3))
        self.d = tuple(float(x) for x in d)
        self.f0 = float(f0)
        self.t0 = 1.0 / self.f0 if t0 is None else float(t0)
        self.sponge_width = int(sponge_width)
        self.sponge_vmax = float(sponge_vmax)

    @property
    def shape(self):
        nz, ny, nx = self.v.shape
        return nx, ny, nz

    @property
    def nrec(self) -> int:
        return self.rec.shape[0]

    def desc(self) -> fd_shot_desc:
        nx, ny, nz = self.shape
        d = fd_shot_desc()
        d.nx, d.ny, d.nz, d.nt = nx, ny, nz, self.nt
        d.dx, d.dy, d.dz = self.d
        d.dt, d.f0, d.t0 = self.dt, self.f0, self.t0
        d.src[0], d.src[1], d.src[2] = self.src
        d.sponge_width = self.sponge_width
        d.sponge_vmax = self.sponge_vmax
        d.v_dev = self.v.data_ptr()
        d.v_zstride, d.v_ystride = self.v.stride(0), self.v.stride(1)
        d.nrec = self.nrec
        d.rec_ijk_host = self.rec.ctypes.data if self.nrec else None
        return d

    def footprint(self) -> int:
        return check(lib().fd_shot_footprint(C.byref(self.desc())), "fd_shot_footprint")


class ShotServer:
    """Submit shots from any thread; poll for (code, traces (nt, nrec), t_ns)."""

    def __init__(self, arena_bytes: int, max_slots: int = 32, device="cuda",
                 max_active_points: int = 0, allocator: str = "first_fit"):
        if allocator not in ("first_fit", "buddy"):
            raise ValueError("allocator must be 'first_fit' or 'buddy'")
        self.arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device=device)
        self.cs = torch.cuda.Stream(device=device)
        self.xs = torch.cuda.Stream(device=device)
        h = C.c_void_p()
        check(lib().fd_server_create(C.byref(h), self.arena.data_ptr(), self.arena.numel(),
                                     int(max_slots), self.cs.cuda_stream, self.xs.cuda_stream),
              "fd_server_create")
        self.h = h
        self._shots: dict[int, Shot] = {}
        if allocator == "buddy":
            check(lib().fd_server_set_allocator(self.h, FD_ARENA_BUDDY), "fd_server_set_allocator")
        if max_active_points:
            self.set_admission(max_active_points)

    def set_admission(self, max_active_points: int):
        """Activation policy (fd_server_set_admission): 0 (default) a shot joins the
        running ones when their interior points and its own stay within 8,388,608
        (one 128 x 32 tile of 8 planes per CU), or within twice that while more
        shots wait behind it; > 0 when they stay within this many.  A shot always
        joins when none runs."""
        check(lib().fd_server_set_admission(self.h, int(max_active_points)),
              "fd_server_set_admission")

    def submit(self, shot: Shot) -> int:
        # the server reads the velocity on its own stream: finish writes to it first
        torch.cuda.current_stream(shot.v.device).synchronize()
        sid = C.c_int64()
        check(lib().shot_submit(self.h, C.byref(shot.desc()), C.byref(sid)), "shot_submit")
        self._shots[sid.value] = shot
        return sid.value

    def poll(self, sid: int):
        """None while the shot runs; else (code, traces or None, (submit, admit, done) ns)."""
        shot = self._shots.get(sid)
        n = 0 if shot is None else shot.nt * shot.nrec
        buf = np.empty(max(n, 1), dtype=np.float32)
        t = (C.c_int64 * 3)()
        rc = lib().shot_poll(self.h, int(sid), buf.ctypes.data, n, t)
        if rc == FD_EAGAIN:
            return None
        if rc == FD_ENOTFOUND:
            check(rc, "shot_poll")
        self._shots.pop(sid, None)
        traces = buf[:n].reshape(shot.nt, shot.nrec) if (rc == FD_OK and shot) else None
        return rc, traces, (t[0], t[1], t[2])

    def wait(self, sid: int, timeout: float = 600.0, interval: float = 1e-4):
        t_end = time.monotonic() + timeout
        while True:
            r = self.poll(sid)
            if r is not None:
                return r
            if time.monotonic() > t_end:
                raise TimeoutError(f"shot {sid} not done after {timeout} s")
            time.sleep(interval)

    def stats(self):
        out = (C.c_int64 * 4)()
        check(lib().fd_server_stats(self.h, out), "fd_server_stats")
        return {"queued": out[0], "running": out[1], "finished": out[2], "steps": out[3]}

    def shutdown(self):
        check(lib().fd_server_shutdown(self.h), "fd_server_shutdown")

    def close(self):
        if self.h:
            check(lib().fd_server_destroy(self.h), "fd_server_destroy")
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class PlainLoop:
    """The comparison loop: each shot alone, in order, with the same kernels in the
    library's native step loop (fd_forward_run: the fused update, the receiver row
    taken by the stencil launch when the receivers share one plane) on buffers sized
    for the largest grid."""

    def __init__(self, max_shape, d=(10.0, 10.0, 10.0), device="cuda"):
        nx, ny, nz = max_shape
        self.device = device
        self.cap = api.Grid(nx, ny, nz, d).elems
        self.buf = [torch.zeros(self.cap, dtype=torch.float32, device=device) for _ in range(5)]

    def run(self, shot: Shot) -> np.ndarray:
        nx, ny, nz = shot.shape
        g = api.Grid(nx, ny, nz, shot.d)
        up, u, un, q, v = self.buf
        for t in (up, u, un):
            t[:g.elems].zero_()
        g.interior(v).copy_(shot.v)
        api.prepare_vdt2(g, v, q, shot.dt)
        sp = None
        if shot.sponge_width > 0:
            vmax = shot.sponge_vmax if shot.sponge_vmax > 0 else float(shot.v.max().item())
            sp = api.Sponge(g, shot.sponge_width, vmax, shot.dt, device=self.device)
        w = api.ricker(shot.nt, shot.dt, shot.f0, shot.t0)
        off = plane = None
        if shot.nrec:
            off = torch.from_numpy(g.offsets(shot.rec)).to(self.device)
            plane = api.receiver_plane(g, shot.rec, self.device)
        tr = torch.zeros((shot.nt, max(shot.nrec, 1)), dtype=torch.float32, device=self.device)
        api.forward_run(g, up, u, un, q, sp, shot.nt, src=shot.src, wavelet=w, rec_off=off,
                        traces=tr if off is not None else None, rec_plane=plane)
        return tr[:, :shot.nrec].cpu().numpy()
