"""Torch-facing wrappers of the libfd C ABI.

Torch only allocates device memory and supplies the current HIP stream; every step of
the computation runs in the library's HIP kernels.  All tensors are float32 on a ROCm
device.  Volume tensors are flat buffers of ``Grid.elems`` floats in the library's
padded layout (x fastest, 4-point halo); ``Grid.interior`` / ``Grid.padded`` give
strided views of them.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib
from ._lib import FDError, check, fd_grid, fd_source, fd_sponge, lib  # noqa: F401

COURANT = 0.4
RICKER_F0 = 15.0
SPONGE_R = 1e-3


def _stream(stream=None) -> int:
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, torch.cuda.Stream):
        return stream.cuda_stream
    return int(stream)


def _ptr(t) -> int | None:
    if t is None:
        return None
    return t.data_ptr()


class Grid:
    """One subdomain geometry (``fd_grid``): interior ``nx*ny*nz``, spacing ``d``."""

    def __init__(self, nx: int, ny: int, nz: int, d=(10.0, 10.0, 10.0)):
        self.c = fd_grid()
        check(lib().fd_grid_init(C.byref(self.c), nx, ny, nz, *map(float, d)), "fd_grid_init")
        self.nx, self.ny, self.nz = nx, ny, nz
        self.d = tuple(float(x) for x in d)
        self.elems = check(lib().fd_grid_elems(C.byref(self.c)), "fd_grid_elems")
        self.ref = C.byref(self.c)

    @property
    def origin(self) -> int:
        return self.c.origin

    @property
    def strides(self) -> tuple[int, int]:
        return self.c.ystride, self.c.zstride

    def face_elems(self, face: int) -> int:
        return check(lib().fd_face_elems(self.ref, face), "fd_face_elems")

    def zeros(self, device="cuda") -> torch.Tensor:
        return torch.zeros(self.elems, dtype=torch.float32, device=device)

    def interior(self, t: torch.Tensor) -> torch.Tensor:
        ys, zs = self.strides
        return t.as_strided((self.nz, self.ny, self.nx), (zs, ys, 1), self.origin)

    def padded(self, t: torch.Tensor) -> torch.Tensor:
        ys, zs = self.strides
        return t.as_strided((self.nz + 8, self.ny + 8, self.nx + 8), (zs, ys, 1),
                            self.origin - 4 * zs - 4 * ys - 4)

    def check(self, t: torch.Tensor, name: str):
        if t is None:
            return
        if not isinstance(t, torch.Tensor) or t.dtype != torch.float32 or not t.is_cuda:
            raise TypeError(f"{name}: expected a float32 ROCm tensor")
        if not t.is_contiguous() or t.numel() < self.elems:
            raise ValueError(f"{name}: expected a contiguous buffer of >= {self.elems} floats")

    def offsets(self, ijk: np.ndarray) -> np.ndarray:
        ijk = np.ascontiguousarray(ijk, dtype=np.int32).reshape(-1, 3)
        out = np.empty(ijk.shape[0], dtype=np.int64)
        check(lib().fd_receiver_offsets(self.ref, ijk.ctypes.data, ijk.shape[0],
                                        out.ctypes.data), "fd_receiver_offsets")
        return out


class Sponge:
    """Damping tables eta_x, eta_y, eta_z on the device (``fd_sponge``)."""

    def __init__(self, grid: Grid, width: int, vmax: float, dt: float, R: float = SPONGE_R,
                 device="cuda"):
        self.width = width
        tabs = []
        for n, d in zip((grid.nx, grid.ny, grid.nz), grid.d):
            emax = lib().fd_sponge_eta_max(vmax, d, dt, width, R)
            if emax < 0:
                check(int(emax), "fd_sponge_eta_max")
            h = np.empty(n, dtype=np.float32)
            check(lib().fd_sponge_profile(h.ctypes.data, n, width, emax), "fd_sponge_profile")
            tabs.append(torch.from_numpy(h).to(device))
        self.eta_x, self.eta_y, self.eta_z = tabs
        self.c = fd_sponge(self.eta_x.data_ptr(), self.eta_y.data_ptr(), self.eta_z.data_ptr())
        self.ref = C.byref(self.c)


def sponge_ref(sp: Sponge | None):
    return None if sp is None else sp.ref


# ----------------------------------------------------------------- set-up (S0)

def cfl_dt(grid: Grid, v: torch.Tensor, courant: float = COURANT, stream=None):
    """(dt, vmax) from a device reduction of max(v); synchronises the stream."""
    grid.check(v, "v")
    scratch = torch.empty(2, dtype=torch.int32, device=v.device)
    vmax = C.c_double()
    dt = C.c_double()
    check(lib().fd_cfl_dt(grid.ref, v.data_ptr(), courant, scratch.data_ptr(), C.byref(vmax),
                          C.byref(dt), _stream(stream)), "fd_cfl_dt")
    return dt.value, vmax.value


def cfl_dt_static(grid: Grid, v: torch.Tensor, courant: float = COURANT, stream=None):
    """cfl_dt through fd_cfl_dt_static: no workspace, nothing allocated (the library's
    static result slots; calls overlapping on one device race)."""
    grid.check(v, "v")
    vmax = C.c_double()
    dt = C.c_double()
    check(lib().fd_cfl_dt_static(grid.ref, v.data_ptr(), courant, C.byref(vmax), C.byref(dt),
                                 _stream(stream)), "fd_cfl_dt_static")
    return dt.value, vmax.value


def prepare_vdt2(grid: Grid, v: torch.Tensor, vdt2: torch.Tensor, dt: float, stream=None):
    grid.check(v, "v")
    grid.check(vdt2, "vdt2")
    check(lib().fd_prepare_vdt2(grid.ref, v.data_ptr(), vdt2.data_ptr(), dt, _stream(stream)),
          "fd_prepare_vdt2")


def prepare_vdt2_m(grid: Grid, m: torch.Tensor, vdt2: torch.Tensor, dt: float, stream=None):
    """vdt2 = dt^2 / m from squared slowness m (same layout and halo treatment)."""
    grid.check(m, "m")
    grid.check(vdt2, "vdt2")
    check(lib().fd_prepare_vdt2_m(grid.ref, m.data_ptr(), vdt2.data_ptr(), dt, _stream(stream)),
          "fd_prepare_vdt2_m")


def ricker(nt: int, dt: float, f0: float = RICKER_F0, t0: float | None = None,
           n0: int = 0) -> np.ndarray:
    if t0 is None:
        t0 = 1.0 / f0
    w = np.empty(max(nt, 1), dtype=np.float32)
    check(lib().fd_ricker(w.ctypes.data, nt, n0, dt, f0, t0), "fd_ricker")
    return w[:nt]


# ----------------------------------------------------------------- per-step path

def step(grid: Grid, u_prev, u, u_next, vdt2, sponge: Sponge | None = None, stream=None):
    for n, t in (("u_prev", u_prev), ("u", u), ("u_next", u_next), ("vdt2", vdt2)):
        grid.check(t, n)
    check(lib().fd_step(grid.ref, u_prev.data_ptr(), u.data_ptr(), u_next.data_ptr(),
                        vdt2.data_ptr(), sponge_ref(sponge), _stream(stream)), "fd_step")


def step_fused(grid: Grid, u_prev, u, u_next, vdt2, sponge: Sponge | None = None, src=None,
               faces=None, stream=None):
    """fd_step + inject_source (``src`` = ((i,j,k), w)) + halo_pack of u_next into
    ``faces`` (six buffers or None entries), in one kernel."""
    for n, t in (("u_prev", u_prev), ("u", u), ("u_next", u_next), ("vdt2", vdt2)):
        grid.check(t, n)
    sref = None
    if src is not None:
        (i, j, k), w = src
        sref = C.byref(fd_source(int(i), int(j), int(k), float(w)))
    check(lib().fd_step_fused(grid.ref, u_prev.data_ptr(), u.data_ptr(), u_next.data_ptr(),
                              vdt2.data_ptr(), sponge_ref(sponge), sref,
                              None if faces is None else _faces(faces, grid), _stream(stream)),
          "fd_step_fused")


def step_exchange(grid: Grid, u_prev, u, u_next, vdt2, sponge: Sponge | None = None, src=None,
                  face_in=None, face_out=None, stream=None):
    """The per-step exchange path as one kernel: u's face halos read from the receive
    buffers ``face_in``, fd_step + source ``src`` = ((i,j,k), w), the faces of u_next
    written to ``face_out`` (fd_step_exchange)."""
    for n, t in (("u_prev", u_prev), ("u", u), ("u_next", u_next), ("vdt2", vdt2)):
        grid.check(t, n)
    sref = None
    if src is not None:
        (i, j, k), w = src
        sref = C.byref(fd_source(int(i), int(j), int(k), float(w)))
    check(lib().fd_step_exchange(grid.ref, u_prev.data_ptr(), u.data_ptr(), u_next.data_ptr(),
                                 vdt2.data_ptr(), sponge_ref(sponge), sref,
                                 None if face_in is None else _faces(face_in, grid),
                                 None if face_out is None else _faces(face_out, grid),
                                 _stream(stream)),
          "fd_step_exchange")


def inject_source(grid: Grid, u_next, vdt2, sponge, ijk, w: float, stream=None):
    grid.check(u_next, "u_next")
    grid.check(vdt2, "vdt2")
    i, j, k = (int(x) for x in ijk)
    check(lib().inject_source(grid.ref, u_next.data_ptr(), vdt2.data_ptr(), sponge_ref(sponge),
                              i, j, k, float(w), _stream(stream)), "inject_source")


def record_receivers(grid: Grid, u, rec_off: torch.Tensor, trace_row: torch.Tensor,
                     stream=None):
    """trace_row[r] = u[rec_off[r]]: rec_off from ``Grid.offsets`` (interior points)."""
    grid.check(u, "u")
    n = rec_off.numel()
    _check_points("record_receivers", rec_off, trace_row)
    check(lib().record_receivers(grid.ref, u.data_ptr(), rec_off.data_ptr(), n,
                                 trace_row.data_ptr(), _stream(stream)), "record_receivers")


def _faces(faces, grid: Grid):
    """ctypes array of six face pointers; each given face must be a contiguous
    float32 device tensor of at least that face's element count."""
    if len(faces) != 6:
        raise ValueError("expected six face buffers (-x, +x, -y, +y, -z, +z)")
    arr = _lib._FACES()
    for i in range(6):
        f = faces[i]
        if f is not None:
            if (not isinstance(f, torch.Tensor) or f.dtype != torch.float32 or not f.is_cuda
                    or not f.is_contiguous() or f.numel() < grid.face_elems(i)):
                raise TypeError(f"face {i}: expected a contiguous float32 ROCm tensor of "
                                f">= {grid.face_elems(i)} elements")
        arr[i] = None if f is None else f.data_ptr()
    return arr


def halo_pack(grid: Grid, u, faces, stream=None):
    grid.check(u, "u")
    check(lib().halo_pack(grid.ref, u.data_ptr(), _faces(faces, grid), _stream(stream)),
          "halo_pack")


def halo_pack_record(grid: Grid, u, faces, rec_off: torch.Tensor | None = None,
                     trace_row: torch.Tensor | None = None, stream=None):
    """halo_pack and record_receivers of the same u in one launch
    (fd_halo_pack_record); without receivers it only packs."""
    grid.check(u, "u")
    n = 0
    if rec_off is not None and rec_off.numel():
        _check_points("halo_pack_record", rec_off, trace_row)
        n = rec_off.numel()
    check(lib().fd_halo_pack_record(grid.ref, u.data_ptr(), _faces(faces, grid),
                                    rec_off.data_ptr() if n else None, n,
                                    trace_row.data_ptr() if n else None, _stream(stream)),
          "fd_halo_pack_record")


def halo_unpack(grid: Grid, u, faces, stream=None):
    grid.check(u, "u")
    check(lib().halo_unpack(grid.ref, u.data_ptr(), _faces(faces, grid), _stream(stream)),
          "halo_unpack")


def face_buffers(grid: Grid, device="cuda"):
    return [torch.zeros(grid.face_elems(f), dtype=torch.float32, device=device)
            for f in range(6)]


def loopback(faces):
    """Receive buffers of a single-device exchange: each face receives what the
    opposite face sent, which makes the subdomain periodic."""
    return [faces[1], faces[0], faces[3], faces[2], faces[5], faces[4]]


# ----------------------------------------------------------------- adjoint

def adjoint_step(grid: Grid, a_nn, a_n1, a_out, vdt2, sponge=None, u_n=None, g_vdt2=None,
                 src=None, stream=None):
    for n, t in (("a_nn", a_nn), ("a_n1", a_n1), ("a_out", a_out), ("vdt2", vdt2),
                 ("u_n", u_n), ("g_vdt2", g_vdt2)):
        grid.check(t, n)
    sref = None
    if src is not None:
        (i, j, k), w = src
        sref = C.byref(fd_source(int(i), int(j), int(k), float(w)))
    check(lib().fd_adjoint_step(grid.ref, _ptr(a_nn), a_n1.data_ptr(), a_out.data_ptr(),
                                vdt2.data_ptr(), sponge_ref(sponge), _ptr(u_n), _ptr(g_vdt2),
                                sref, _stream(stream)), "fd_adjoint_step")


def _check_points(where: str, off: torch.Tensor, vals: torch.Tensor):
    if (off.dtype != torch.int64 or vals.dtype != torch.float32 or not off.is_contiguous()
            or not vals.is_contiguous() or vals.numel() < off.numel()
            or off.device.type != "cuda" or vals.device.type != "cuda"):
        raise TypeError(f"{where}: device int64 offsets and float32 values (>= as many)")


def scatter_add(grid: Grid, a, off: torch.Tensor, vals: torch.Tensor, stream=None):
    grid.check(a, "a")
    _check_points("scatter_add", off, vals)
    check(lib().fd_scatter_add(grid.ref, a.data_ptr(), off.data_ptr(), vals.data_ptr(),
                               off.numel(), _stream(stream)), "fd_scatter_add")


def grad_finalize(grid: Grid, g_vdt2, vdt2, dt: float, grad_m, stream=None):
    for n, t in (("g_vdt2", g_vdt2), ("vdt2", vdt2), ("grad_m", grad_m)):
        grid.check(t, n)
    check(lib().fd_grad_finalize(grid.ref, g_vdt2.data_ptr(), vdt2.data_ptr(), dt,
                                 grad_m.data_ptr(), _stream(stream)), "fd_grad_finalize")


def adjoint_step_scaled(grid: Grid, b_nn, b_n1, b_out, vdt2, sponge=None, u_n=None, g_b=None,
                        src=None, stream=None, res=None):
    """b_out = D (2 b_n1 - E b_nn + Q L b_n1) (the adjoint in b = Q D lambda), and
    optionally g_b += b_n1 (L u_n + f).  ``res = (plane, row)`` (a ReceiverPlane and
    a device row of its receivers' values) also adds the row at the receivers as
    scatter_add_scaled would, in the same launch (fd_adjoint_step_scaled_res)."""
    if b_nn is None or b_n1 is None or b_out is None:
        raise ValueError("adjoint_step_scaled: b_nn, b_n1 and b_out are required")
    for n, t in (("b_nn", b_nn), ("b_n1", b_n1), ("b_out", b_out), ("vdt2", vdt2),
                 ("u_n", u_n), ("g_b", g_b)):
        grid.check(t, n)
    sref = None
    if src is not None:
        (i, j, k), w = src
        sref = C.byref(fd_source(int(i), int(j), int(k), float(w)))
    if res is not None:
        plane, row = res
        m = plane.map
        if (m.dtype != torch.int32 or not m.is_cuda or not m.is_contiguous()
                or m.numel() != grid.nx * grid.ny):
            raise TypeError("adjoint_step_scaled: the plane map must be a device int32 nx*ny array")
        if (row.dtype != torch.float32 or not row.is_cuda or not row.is_contiguous()
                or row.numel() < plane.nrec):
            raise TypeError("adjoint_step_scaled: the row must be a contiguous device float32 "
                            "array covering every receiver of the plane")
        check(lib().fd_adjoint_step_scaled_res(
            grid.ref, b_nn.data_ptr(), b_n1.data_ptr(), b_out.data_ptr(), vdt2.data_ptr(),
            sponge_ref(sponge), _ptr(u_n), _ptr(g_b), sref, m.data_ptr(), plane.k,
            row.data_ptr(), _stream(stream)), "fd_adjoint_step_scaled_res")
        return
    check(lib().fd_adjoint_step_scaled(grid.ref, b_nn.data_ptr(), b_n1.data_ptr(),
                                       b_out.data_ptr(), vdt2.data_ptr(), sponge_ref(sponge),
                                       _ptr(u_n), _ptr(g_b), sref, _stream(stream)),
          "fd_adjoint_step_scaled")


def scatter_add_scaled(grid: Grid, b, off: torch.Tensor, vals: torch.Tensor, vdt2,
                       sponge=None, stream=None):
    """b[off] += vals * vdt2 / (1 + eta) at each offset."""
    grid.check(b, "b")
    grid.check(vdt2, "vdt2")
    _check_points("scatter_add_scaled", off, vals)
    check(lib().fd_scatter_add_scaled(grid.ref, b.data_ptr(), off.data_ptr(), vals.data_ptr(),
                                      vdt2.data_ptr(), sponge_ref(sponge), off.numel(),
                                      _stream(stream)), "fd_scatter_add_scaled")


def grad_finalize_scaled(grid: Grid, g_b, vdt2, dt: float, grad_m, stream=None):
    for n, t in (("g_b", g_b), ("vdt2", vdt2), ("grad_m", grad_m)):
        grid.check(t, n)
    check(lib().fd_grad_finalize_scaled(grid.ref, g_b.data_ptr(), vdt2.data_ptr(), dt,
                                        grad_m.data_ptr(), _stream(stream)),
          "fd_grad_finalize_scaled")


def set_kchunk(kchunk: int):
    check(lib().fd_set_kchunk(int(kchunk)), "fd_set_kchunk")


def set_tiles(mode: int):
    """Forward kernel shape (fd_set_tiles): 0 automatic, 1 = 64 x 32 tiles, 2 = 64 x 16
    tiles, 3 = one thread per point wherever the update takes no faces inside."""
    check(lib().fd_set_tiles(int(mode)), "fd_set_tiles")


def step_launch(grid: Grid) -> dict:
    """Launch shape of the z-marching forward kernel over ``grid`` (fd_step_launch); grids
    of at most 2^22 points run fd_step and the fused forms one thread per point."""
    out = (C.c_int32 * 4)()
    check(lib().fd_step_launch(grid.ref, out), "fd_step_launch")
    tx, ty, kc, zc = out
    return {"tiles_x": tx, "tiles_y": ty, "kchunk": kc, "zchunks": zc, "blocks": tx * ty * zc}


KERNEL_NAMES = {0: "point", 1: "march_64x32", 2: "march_64x16", 3: "wide_128x32",
                4: "wide_64x64"}


def step_kernel(grid: Grid, faces: bool = False) -> dict:
    """The forward kernel a step over ``grid`` takes (fd_step_kernel): ``faces`` for the
    exchange step with all twelve face buffers, else the update without faces."""
    out = (C.c_int32 * 6)()
    check(lib().fd_step_kernel(grid.ref, int(bool(faces)), out), "fd_step_kernel")
    kind, tx, ty, kc, zc, nb = out
    return {"kernel": KERNEL_NAMES[kind], "tile": (tx, ty), "kchunk": kc, "zchunks": zc,
            "blocks": nb}


# ----------------------------------------------------------------- forward model

class ReceiverPlane:
    """Receivers on one z plane as the forward kernel samples them itself
    (fd_receiver_plane_map): ``map`` (device int32, nx*ny) and the plane ``k``."""

    def __init__(self, map_: torch.Tensor, k: int, nrec: int):
        self.map = map_
        self.k = int(k)
        self.nrec = int(nrec)


def receiver_plane(grid: Grid, rec_ijk: np.ndarray, device="cuda") -> ReceiverPlane | None:
    """The plane map of receivers that all lie on one z plane at distinct points, or
    None (they are then sampled by a separate launch)."""
    ijk = np.ascontiguousarray(rec_ijk, dtype=np.int32).reshape(-1, 3)
    if ijk.shape[0] == 0:
        return None
    m = np.empty(grid.nx * grid.ny, dtype=np.int32)
    k = C.c_int32()
    rc = lib().fd_receiver_plane_map(grid.ref, ijk.ctypes.data, ijk.shape[0], m.ctypes.data,
                                     C.byref(k))
    if rc == _lib.FD_EINVAL:
        return None
    check(rc, "fd_receiver_plane_map")
    return ReceiverPlane(torch.from_numpy(m).to(device), k.value, ijk.shape[0])


def _run_struct(grid, u_prev, u, u_next, vdt2, sponge, nt, src, wavelet, rec_off, traces,
                send, send2, rec_plane, who):
    """The fd_run of forward_run / forward_graph, the arrays by address, and the host
    objects that must outlive the call."""
    for n, t in (("u_prev", u_prev), ("u", u), ("u_next", u_next), ("vdt2", vdt2)):
        grid.check(t, n)
    r = _lib.fd_run()
    if rec_plane is not None:
        m = rec_plane.map
        if (m.dtype != torch.int32 or not m.is_cuda or not m.is_contiguous()
                or m.numel() != grid.nx * grid.ny):
            raise TypeError(f"{who}: rec_plane map must be a device int32 nx*ny array")
        r.rec_map = m.data_ptr()
        r.rec_k = rec_plane.k
    bufs = {t.data_ptr(): t for t in (u_prev, u, u_next)}
    r.u_prev, r.u, r.u_next = u_prev.data_ptr(), u.data_ptr(), u_next.data_ptr()
    r.vdt2 = vdt2.data_ptr()
    if sponge is not None:
        r.sponge = sponge.c
    r.nt = int(nt)
    wa = None
    if src is not None:
        wa = np.ascontiguousarray(wavelet, dtype=np.float32)
        if wa.size < nt:
            raise ValueError(f"{who}: wavelet shorter than nt")
        r.wavelet = wa.ctypes.data
        r.src[0], r.src[1], r.src[2] = (int(x) for x in src)
    if rec_off is not None and rec_off.numel():
        if (rec_off.dtype != torch.int64 or traces is None or traces.dtype != torch.float32
                or not traces.is_contiguous() or traces.dim() != 2
                or traces.shape[0] < nt or traces.shape[1] != rec_off.numel()):
            raise TypeError(f"{who}: rec_off int64 and contiguous float32 traces "
                            "(>= nt, nrec)")
        r.nrec = rec_off.numel()
        r.rec_off = rec_off.data_ptr()
        r.traces = traces.data_ptr()
    if send is not None:
        fs = _faces(send, grid)
        for f in range(6):
            r.send[f] = fs[f]
    if send2 is not None:
        if send is None:
            raise ValueError(f"{who}: send2 needs send")
        fs = _faces(send2, grid)
        for f in range(6):
            r.send2[f] = fs[f]
    return r, bufs, wa


def forward_run(grid: Grid, u_prev, u, u_next, vdt2, sponge: Sponge | None, nt: int, src=None,
                wavelet=None, rec_off: torch.Tensor | None = None,
                traces: torch.Tensor | None = None, send=None, send2=None, stream=None,
                rec_plane: ReceiverPlane | None = None):
    """``nt`` steps in the library's native loop (fd_forward_run): per step unpack of
    ``send`` into the opposite halos (loopback; skipped when ``send`` is None), the
    fused update with the source ``src`` at amplitude ``wavelet[s]``, pack into
    ``send``, and the receiver row ``traces[s]``; with ``send2`` (a second face set)
    each step is one fd_step_exchange and the sets alternate.  Returns the rotated
    ``(u_prev, u, u_next)``: u^{n+nt-1}, u^{n+nt} and the spare array; with
    ``send2`` it returns ``(u_prev, u, u_next, send, send2)``, ``send`` holding the
    faces of the new u.  ``rec_plane`` (from ``receiver_plane`` of the same receivers
    as ``rec_off``) lets the stencil launch take the receiver row where no faces are
    packed."""
    r, bufs, keep = _run_struct(grid, u_prev, u, u_next, vdt2, sponge, nt, src, wavelet, rec_off,
                                traces, send, send2, rec_plane, "forward_run")
    check(lib().fd_forward_run(grid.ref, C.byref(r), _stream(stream)), "fd_forward_run")
    if send2 is None:
        return bufs[r.u_prev], bufs[r.u], bufs[r.u_next]
    swapped = r.send[0] != send[0].data_ptr()
    if swapped:
        send, send2 = send2, send
    return bufs[r.u_prev], bufs[r.u], bufs[r.u_next], send, send2


class ForwardGraph:
    """A forward run recorded once as a HIP graph (fd_forward_graph) and launched as
    often as wanted: each ``launch`` re-runs the ``nt`` steps from a zero state with
    the fixed source wavelet, reading the current contents of ``vdt2`` (a new model
    written into it is picked up) and writing ``traces``.  After a launch the final
    state is in ``u_prev``, ``u`` (and, with faces, the faces of ``u`` in ``send``)."""

    def __init__(self, grid: Grid, u_prev, u, u_next, vdt2, sponge: Sponge | None, nt: int,
                 src=None, wavelet=None, rec_off=None, traces=None, send=None, send2=None,
                 rec_plane: ReceiverPlane | None = None):
        r, bufs, _ = _run_struct(grid, u_prev, u, u_next, vdt2, sponge, nt, src, wavelet, rec_off,
                                 traces, send, send2, rec_plane, "ForwardGraph")
        h = C.c_void_p()
        check(lib().fd_forward_graph(grid.ref, C.byref(r), C.byref(h)), "fd_forward_graph")
        self._h = h
        # every array the graph touches stays referenced while it lives
        self._keep = (grid, vdt2, sponge, rec_off, traces, send, send2, rec_plane, u_prev, u, u_next)
        self.u_prev, self.u, self.u_next = bufs[r.u_prev], bufs[r.u], bufs[r.u_next]
        self.send = self.send2 = None
        if send2 is not None:
            swapped = r.send[0] != send[0].data_ptr()
            self.send, self.send2 = (send2, send) if swapped else (send, send2)
        elif send is not None:
            self.send = send

    def launch(self, stream=None):
        if self._h is None:
            raise RuntimeError("ForwardGraph: closed")
        check(lib().fd_graph_launch(self._h, _stream(stream)), "fd_graph_launch")

    def close(self):
        if self._h is not None:
            check(lib().fd_graph_destroy(self._h), "fd_graph_destroy")
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclass
class Geometry:
    """Source and receivers of one shot (0-based interior indices)."""
    src: tuple[int, int, int] | None = None
    rec: np.ndarray | None = None  # int32 (nrec, 3)
    f0: float = RICKER_F0
    t0: float | None = None


class Simulation:
    """Forward model of one subdomain: S0 set-up once, then S1-S7 per step.

    ``exchange="loopback"`` packs the six faces of u^n each step and unpacks each
    into the opposite halo (periodic subdomain); ``None`` keeps zero (Dirichlet)
    halos.  The wavefields stay on the device; ``run`` returns device traces."""

    def __init__(self, v: np.ndarray | torch.Tensor, d=(10.0, 10.0, 10.0),
                 courant: float = COURANT, sponge_width: int = 0, geom: Geometry | None = None,
                 exchange: str | None = None, dt: float | None = None, device="cuda",
                 sponge_vmax: float | None = None):
        nz, ny, nx = v.shape
        self.grid = g = Grid(nx, ny, nz, d)
        self.device = device
        vt = g.zeros(device)
        g.interior(vt).copy_(torch.as_tensor(v, dtype=torch.float32))
        self.v = vt
        dt_cfl, vmax = cfl_dt(g, vt, courant)
        self.vmax = vmax
        self.dt = dt_cfl if dt is None else float(dt)
        self.vdt2 = g.zeros(device)
        prepare_vdt2(g, vt, self.vdt2, self.dt)
        self.sponge = (Sponge(g, sponge_width, vmax if sponge_vmax is None else sponge_vmax,
                              self.dt, device=device) if sponge_width > 0 else None)
        self.geom = geom or Geometry()
        self.u_prev = g.zeros(device)
        self.u = g.zeros(device)
        self.u_next = g.zeros(device)
        self.n = 0
        self.exchange = exchange
        if exchange not in (None, "loopback"):
            raise ValueError("exchange must be None or 'loopback'")
        # two face sets: ``send`` holds the faces of u, ``send2`` receives those of
        # u_next in the one-kernel step (a real exchange double-buffers likewise)
        self.send = face_buffers(g, device) if exchange else None
        self.send2 = face_buffers(g, device) if exchange else None
        self._faces_current = True  # zero state, zero face buffers
        rec = self.geom.rec
        if rec is not None and len(rec):
            self.rec_off = torch.from_numpy(g.offsets(rec)).to(device)
            # receivers on one plane: the native loops sample them in the stencil launch
            self.rec_plane = receiver_plane(g, rec, device)
        else:
            self.rec_off = None
            self.rec_plane = None

    @property
    def nrec(self) -> int:
        return 0 if self.rec_off is None else self.rec_off.numel()

    MODES = ("exchange", "fused", "separate", "native", "native-fused")

    def run(self, nt: int, traces: torch.Tensor | None = None, stream=None,
            mode: str = "exchange") -> torch.Tensor:
        """Advance ``nt`` steps; returns (nt, nrec) device traces (u^{n+1} at receivers).

        Per step, by ``mode``:
        * ``"exchange"`` (default): one fd_step_exchange (u's face halos read from the
          loopback of the faces packed by the previous step, update + source, faces
          of the new field packed into the other face set), then record_receivers;
        * ``"fused"``: halo_unpack of the faces packed by the previous step, then
          fd_step_fused (update + source + pack), then record_receivers;
        * ``"separate"``: halo_pack, halo_unpack, fd_step, inject_source,
          record_receivers as separate calls;
        * ``"native"`` / ``"native-fused"``: the exchange / fused sequence looped in
          the library (fd_forward_run).
        All give the same bits."""
        if mode not in self.MODES:
            raise ValueError(f"mode must be one of {self.MODES}")
        g = self.grid
        if traces is None:
            traces = torch.zeros((nt, max(self.nrec, 1)), dtype=torch.float32, device=self.device)
        geom = self.geom
        w = None
        if geom.src is not None:
            w = ricker(nt, self.dt, geom.f0, geom.t0, n0=self.n)
        if mode != "separate" and self.exchange and not self._faces_current:
            halo_pack(g, self.u, self.send, stream)
        if mode.startswith("native"):
            return self._run_native(nt, w, traces, stream, mode == "native")
        for s in range(nt):
            src = None if w is None else (geom.src, float(w[s]))
            if mode == "exchange":
                face_in = loopback(self.send) if self.exchange else None
                step_exchange(g, self.u_prev, self.u, self.u_next, self.vdt2, self.sponge, src,
                              face_in, self.send2 if self.exchange else None, stream)
                if self.exchange:
                    self.send, self.send2 = self.send2, self.send
            elif mode == "fused":
                if self.exchange:
                    halo_unpack(g, self.u, loopback(self.send), stream)
                step_fused(g, self.u_prev, self.u, self.u_next, self.vdt2, self.sponge, src,
                           self.send if self.exchange else None, stream)
            else:
                if self.exchange:
                    halo_pack(g, self.u, self.send, stream)
                    halo_unpack(g, self.u, loopback(self.send), stream)
                step(g, self.u_prev, self.u, self.u_next, self.vdt2, self.sponge, stream)
                if w is not None:
                    inject_source(g, self.u_next, self.vdt2, self.sponge, geom.src, float(w[s]),
                                  stream)
            if self.rec_off is not None:
                record_receivers(g, self.u_next, self.rec_off, traces[s], stream)
            self.u_prev, self.u, self.u_next = self.u, self.u_next, self.u_prev
            self.n += 1
        # after a packing step the send buffers hold the faces of the current u
        self._faces_current = bool(mode != "separate" and self.exchange and nt > 0) or (
            self._faces_current and nt == 0)
        return traces[:, :self.nrec]

    def _run_native(self, nt, w, traces, stream, one_kernel: bool):
        """The exchange (``one_kernel``) or fused per-step sequence, looped in native
        code (fd_forward_run)."""
        out = forward_run(
            self.grid, self.u_prev, self.u, self.u_next, self.vdt2, self.sponge, nt,
            src=self.geom.src if w is not None else None, wavelet=w, rec_off=self.rec_off,
            traces=traces if self.rec_off is not None else None,
            send=self.send if self.exchange else None,
            send2=self.send2 if self.exchange and one_kernel else None, stream=stream,
            rec_plane=self.rec_plane)
        self.u_prev, self.u, self.u_next = out[:3]
        if len(out) == 5:
            self.send, self.send2 = out[3], out[4]
        self.n += nt
        self._faces_current = bool(self.exchange) or self._faces_current
        return traces[:, :self.nrec]

    def state(self):
        """Interior views of (u^{n-1}, u^n)."""
        return self.grid.interior(self.u_prev), self.grid.interior(self.u)


# -------------------------------------------------- Cannon's matrix multiply (Sec. 4.4)

def _ld(t: torch.Tensor, name: str) -> int:
    """Leading dimension of a 2-D float64 device tensor with unit column stride."""
    if t.dtype != torch.float64 or t.dim() != 2 or not t.is_cuda:
        raise TypeError(f"{name}: a 2-D float64 device tensor is needed")
    if t.numel() and t.shape[1] > 1 and t.stride(1) != 1:
        raise TypeError(f"{name}: unit column stride is needed")
    return t.stride(0) if t.shape[0] > 1 else max(t.shape[1], 1)


def block_gemm(a: torch.Tensor, b: torch.Tensor, c: torch.Tensor, accumulate: bool = True,
               stream=None) -> torch.Tensor:
    """c = (c if accumulate else 0) + a @ b in FP64 on the matrix cores
    (fd_block_gemm_f64): the local product of one Cannon step.  a (m, k), b (k, n),
    c (m, n) may be row views of larger tensors; c is written in place."""
    m, k = a.shape
    k2, n = b.shape
    if k != k2 or tuple(c.shape) != (m, n):
        raise ValueError("block_gemm: shapes do not match")
    check(lib().fd_block_gemm_f64(m, n, k, a.data_ptr(), _ld(a, "a"), b.data_ptr(), _ld(b, "b"),
                                  c.data_ptr(), _ld(c, "c"), 1 if accumulate else 0,
                                  _stream(stream)), "fd_block_gemm_f64")
    return c


def cannon_order(rank: int, P: int) -> list:
    """The B row stripes rank ``rank`` multiplies with, in step order (its own first,
    then the one its ring neighbour passes on after each step)."""
    return [(rank + s) % P for s in range(P)]


def cannon_rank(A_r: torch.Tensor, B: torch.Tensor, C_r: torch.Tensor, rank: int, P: int,
                stream=None) -> torch.Tensor:
    """The P local steps of one rank of Cannon's algorithm (Sec. 4.4) with every B
    stripe resident (the ring shift that would bring them in is not done here):
    C_r += A_r[:, q*Ns:(q+1)*Ns] @ B[q*Ns:(q+1)*Ns, :] for q in cannon_order(rank, P),
    Ns = N / P.  A_r and C_r are the rank's Ns x N stripes, B is N x N."""
    N = B.shape[0]
    if B.shape != (N, N) or N % P or A_r.shape != (N // P, N) or C_r.shape != (N // P, N):
        raise ValueError("cannon_rank: stripes of N/P x N and an N x N B are needed")
    ns = N // P
    for q in cannon_order(rank, P):
        block_gemm(A_r[:, q * ns:(q + 1) * ns], B[q * ns:(q + 1) * ns, :], C_r, True, stream)
    return C_r
