"""ctypes binding of ``libfd.so`` (argument marshalling only).

Loads the in-tree HIP library and declares the C ABI of ``include/fd.h``.  There is no
fallback: if the library is missing or fails to load, every entry point raises.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfd.so")

FD_OK = 0
FD_ENOTFOUND = -2
FD_EDEVICE = -5
FD_EAGAIN = -11
FD_ENOMEM = -12
FD_EINVAL = -22
FD_ECANCELED = -125
FD_HALO = 4
FD_ARENA_FIRST_FIT = 0
FD_ARENA_BUDDY = 1


class fd_grid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("halo", C.c_int32),
                ("origin", C.c_int64), ("ystride", C.c_int64), ("zstride", C.c_int64),
                ("dx", C.c_double), ("dy", C.c_double), ("dz", C.c_double)]


class fd_sponge(C.Structure):
    _fields_ = [("eta_x", C.c_void_p), ("eta_y", C.c_void_p), ("eta_z", C.c_void_p)]


class fd_source(C.Structure):
    _fields_ = [("i", C.c_int32), ("j", C.c_int32), ("k", C.c_int32), ("w", C.c_float)]


class fd_shot_desc(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("nt", C.c_int32),
                ("dx", C.c_double), ("dy", C.c_double), ("dz", C.c_double), ("dt", C.c_double),
                ("f0", C.c_double), ("t0", C.c_double), ("src", C.c_int32 * 3),
                ("sponge_width", C.c_int32), ("sponge_vmax", C.c_double),
                ("v_dev", C.c_void_p), ("v_ystride", C.c_int64), ("v_zstride", C.c_int64),
                ("nrec", C.c_int32), ("rec_ijk_host", C.c_void_p)]


class fd_run(C.Structure):
    _fields_ = [("u_prev", C.c_void_p), ("u", C.c_void_p), ("u_next", C.c_void_p),
                ("vdt2", C.c_void_p), ("sponge", fd_sponge), ("nt", C.c_int32),
                ("src", C.c_int32 * 3), ("wavelet", C.c_void_p), ("nrec", C.c_int32),
                ("rec_off", C.c_void_p), ("traces", C.c_void_p), ("send", C.c_void_p * 6),
                ("send2", C.c_void_p * 6), ("rec_map", C.c_void_p), ("rec_k", C.c_int32)]


class FDError(RuntimeError):
    def __init__(self, code: int, where: str, detail: str):
        super().__init__(f"{where}: {detail or 'error'} (code {code})")
        self.code = code


_P = C.c_void_p
_G = C.POINTER(fd_grid)
_S = C.POINTER(fd_sponge)
_i32, _i64, _f32, _f64 = C.c_int32, C.c_int64, C.c_float, C.c_double
_FACES = _P * 6

# name -> (restype, argtypes)
SIGNATURES = {
    "fd_strerror": (C.c_char_p, [C.c_int]),
    "fd_last_error": (C.c_char_p, []),
    "fd_version": (C.c_int, []),
    "fd_grid_init": (C.c_int, [_G, _i32, _i32, _i32, _f64, _f64, _f64]),
    "fd_grid_elems": (_i64, [_G]),
    "fd_face_elems": (_i64, [_G, _i32]),
    "fd_offset": (_i64, [_G, _i32, _i32, _i32]),
    "fd_set_kchunk": (C.c_int, [_i32]),
    "fd_step_launch": (C.c_int, [_G, C.POINTER(C.c_int32)]),
    "fd_step_kernel": (C.c_int, [_G, C.c_int32, C.POINTER(C.c_int32)]),
    "fd_set_tiles": (C.c_int, [_i32]),
    "fd_cfl_dt": (C.c_int, [_G, _P, _f64, _P, C.POINTER(_f64), C.POINTER(_f64), _P]),
    "fd_cfl_dt_static": (C.c_int, [_G, _P, _f64, C.POINTER(_f64), C.POINTER(_f64), _P]),
    "fd_prepare_vdt2": (C.c_int, [_G, _P, _P, _f64, _P]),
    "fd_block_gemm_f64": (C.c_int, [C.c_int64, C.c_int64, C.c_int64, _P, C.c_int64, _P,
                                    C.c_int64, _P, C.c_int64, _i32, _P]),
    "fd_prepare_vdt2_m": (C.c_int, [_G, _P, _P, _f64, _P]),
    "fd_sponge_eta_max": (_f64, [_f64, _f64, _f64, _i32, _f64]),
    "fd_sponge_profile": (C.c_int, [_P, _i32, _i32, _f64]),
    "fd_ricker": (C.c_int, [_P, _i32, _i32, _f64, _f64, _f64]),
    "fd_receiver_offsets": (C.c_int, [_G, _P, _i32, _P]),
    "fd_step": (C.c_int, [_G, _P, _P, _P, _P, _S, _P]),
    "fd_step_fused": (C.c_int, [_G, _P, _P, _P, _P, _S, C.POINTER(fd_source), C.POINTER(_P),
                                _P]),
    "fd_step_exchange": (C.c_int, [_G, _P, _P, _P, _P, _S, C.POINTER(fd_source),
                                   C.POINTER(_P), C.POINTER(_P), _P]),
    "fd_forward_run": (C.c_int, [_G, C.POINTER(fd_run), _P]),
    "fd_forward_graph": (C.c_int, [_G, C.POINTER(fd_run), C.POINTER(_P)]),
    "fd_graph_launch": (C.c_int, [_P, _P]),
    "fd_graph_destroy": (C.c_int, [_P]),
    "fd_receiver_plane_map": (C.c_int, [_G, _P, _i32, _P, C.POINTER(_i32)]),
    "inject_source": (C.c_int, [_G, _P, _P, _S, _i32, _i32, _i32, _f32, _P]),
    "record_receivers": (C.c_int, [_G, _P, _P, _i32, _P, _P]),
    "halo_pack": (C.c_int, [_G, _P, C.POINTER(_P), _P]),
    "fd_halo_pack_record": (C.c_int, [_G, _P, C.POINTER(_P), _P, _i32, _P, _P]),
    "halo_unpack": (C.c_int, [_G, _P, C.POINTER(_P), _P]),
    "fd_adjoint_step": (C.c_int, [_G, _P, _P, _P, _P, _S, _P, _P, C.POINTER(fd_source), _P]),
    "fd_scatter_add": (C.c_int, [_G, _P, _P, _P, _i32, _P]),
    "fd_grad_finalize": (C.c_int, [_G, _P, _P, _f64, _P, _P]),
    "fd_adjoint_step_scaled": (C.c_int, [_G, _P, _P, _P, _P, _S, _P, _P, C.POINTER(fd_source),
                                         _P]),
    "fd_adjoint_step_scaled_res": (C.c_int, [_G, _P, _P, _P, _P, _S, _P, _P,
                                             C.POINTER(fd_source), _P, _i32, _P, _P]),
    "fd_scatter_add_scaled": (C.c_int, [_G, _P, _P, _P, _P, _S, _i32, _P]),
    "fd_grad_finalize_scaled": (C.c_int, [_G, _P, _P, _f64, _P, _P]),
    "fd_shot_footprint": (_i64, [C.POINTER(fd_shot_desc)]),
    "fd_server_create": (C.c_int, [C.POINTER(_P), _P, C.c_size_t, _i32, _P, _P]),
    "shot_submit": (C.c_int, [_P, C.POINTER(fd_shot_desc), C.POINTER(_i64)]),
    "shot_poll": (C.c_int, [_P, _i64, _P, C.c_size_t, C.POINTER(_i64)]),
    "fd_server_set_admission": (C.c_int, [_P, _i64]),
    "fd_server_set_allocator": (C.c_int, [_P, C.c_int32]),
    "fd_server_stats": (C.c_int, [_P, C.POINTER(_i64)]),
    "fd_server_shutdown": (C.c_int, [_P]),
    "fd_server_destroy": (C.c_int, [_P]),
}

_lib = None


def lib() -> C.CDLL:
    """The loaded library; raises if it was not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build the HIP library first "
                "(python paper_2506_02486_amd/build.py)")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(rc: int, where: str) -> int:
    if rc < 0:
        detail = lib().fd_last_error().decode(errors="replace")
        raise FDError(rc, where, detail)
    return rc


def exported_symbols() -> list[str]:
    return list(SIGNATURES)
