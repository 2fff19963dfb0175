"""C-ABI contract checks that need no GPU: the library loads, exports every function
that include/fd.h declares, and rejects invalid arguments before any launch.

Every call that passes fake (never dereferenced) device pointers here is one that
the validation layer must refuse, so nothing is ever enqueued.
"""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2506_02486_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
FAKE = 0x10000  # non-NULL, never dereferenced: each call below fails validation first


def header_functions():
    src = open(os.path.join(ROOT, "include", "fd.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*([a-z_0-9]+)\s*\(", src,
                                 flags=re.M)))


@pytest.fixture(scope="module")
def L():
    return _lib.lib()


def grid(L, nx=64, ny=48, nz=40, d=(10.0, 10.0, 10.0)):
    g = _lib.fd_grid()
    assert L.fd_grid_init(C.byref(g), nx, ny, nz, *d) == 0
    return g


def test_every_declared_symbol_is_exported_and_bound(L):
    names = header_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(L, n), n
    assert set(names) <= set(_lib.exported_symbols())


def test_strerror_and_last_error(L):
    for code, word in ((0, b"success"), (-22, b"invalid"), (-12, b"memory"), (-2, b"not found"),
                       (-11, b"not finished"), (-125, b"cancel"), (-5, b"device")):
        assert word in L.fd_strerror(code)
    assert L.fd_strerror(12345)
    g = _lib.fd_grid()
    assert L.fd_grid_init(C.byref(g), 0, 4, 4, 1, 1, 1) == _lib.FD_EINVAL
    assert b"extent" in L.fd_last_error()


def test_grid_init_layout(L):
    for n in (1, 5, 63, 64, 100, 512, 1024):
        g = grid(L, n, 7, 3)
        assert g.halo == 4
        assert g.ystride % 32 == 0 and g.ystride >= n + 8
        assert g.zstride == g.ystride * (7 + 8)
        assert g.origin % 32 == 0                       # interior rows 128-byte aligned
        assert (g.origin - 4) % 32 == 28                # x halo sits right before the row
        last = g.origin + (3 + 3) * g.zstride + (7 + 3) * g.ystride + n + 3
        assert L.fd_grid_elems(C.byref(g)) == last + 1
        assert L.fd_offset(C.byref(g), -4, -4, -4) >= 0
        assert L.fd_offset(C.byref(g), n + 4, 0, 0) == -1
    g = grid(L, 10, 11, 12)
    assert [L.fd_face_elems(C.byref(g), f) for f in range(6)] == [4 * 11 * 12] * 2 + \
        [4 * 10 * 12] * 2 + [4 * 10 * 11] * 2
    assert L.fd_face_elems(C.byref(g), 6) == -1


@pytest.mark.parametrize("bad", ["halo", "ystride", "zstride", "origin", "dx", "nz", "big"])
def test_invalid_geometry_rejected(L, bad):
    g = grid(L)
    if bad == "halo":
        g.halo = 3
    elif bad == "ystride":
        g.ystride = g.nx + 7
    elif bad == "zstride":
        g.zstride = g.ystride * (g.ny + 7)
    elif bad == "origin":
        g.origin = 4 * g.zstride
    elif bad == "dx":
        g.dx = float("nan")
    elif bad == "nz":
        g.nz = 0
    elif bad == "big":
        g.zstride = 1 << 31
    assert L.fd_grid_elems(C.byref(g)) == -1
    assert L.fd_step(C.byref(g), FAKE, FAKE * 2, FAKE * 3, FAKE * 4, None, None) == _lib.FD_EINVAL
    big = _lib.fd_grid()
    assert L.fd_grid_init(C.byref(big), 40000, 60000, 8, 1, 1, 1) == _lib.FD_EINVAL  # > 2^31


def test_step_argument_checks(L):
    g = grid(L)
    n = L.fd_grid_elems(C.byref(g)) * 4
    a, b, c, q = FAKE, FAKE + 4 * n, FAKE + 8 * n, FAKE + 12 * n
    EINVAL = _lib.FD_EINVAL
    assert L.fd_step(C.byref(g), a, b, None, q, None, None) == EINVAL          # NULL
    assert L.fd_step(C.byref(g), a, b, b, q, None, None) == EINVAL             # u_next == u
    assert L.fd_step(C.byref(g), a, b, b + 4, q, None, None) == EINVAL         # overlaps u
    assert L.fd_step(C.byref(g), a, b, q, q, None, None) == EINVAL             # overlaps vdt2
    assert L.fd_step(C.byref(g), a, b, a + 16, q, None, None) == EINVAL        # partial alias
    sp = _lib.fd_sponge(FAKE, None, None)
    assert L.fd_step(C.byref(g), a, b, c, q, C.byref(sp), None) == EINVAL      # 1 of 3 tables
    assert L.inject_source(C.byref(g), c, q, None, 64, 0, 0, 1.0, None) == EINVAL
    assert L.inject_source(C.byref(g), c, q, None, -1, 0, 0, 1.0, None) == EINVAL
    assert L.record_receivers(C.byref(g), a, FAKE, -1, FAKE, None) == EINVAL
    assert L.record_receivers(C.byref(g), a, FAKE, 0, FAKE, None) == 0         # nothing to do
    assert L.fd_scatter_add(C.byref(g), a, FAKE, FAKE, -3, None) == EINVAL
    assert L.fd_prepare_vdt2(C.byref(g), a, a + 4, 1e-3, None) == EINVAL
    assert L.fd_prepare_vdt2(C.byref(g), a, b, -1.0, None) == EINVAL
    assert L.fd_grad_finalize(C.byref(g), a, b, 0.0, c, None) == EINVAL
    assert L.fd_cfl_dt(C.byref(g), a, 0.4, None, None, None, None) == EINVAL


def test_exchange_and_scaled_adjoint_argument_checks(L):
    EINVAL = _lib.FD_EINVAL
    g = grid(L)
    n = L.fd_grid_elems(C.byref(g)) * 4
    a, b, c, q, u, gg = (FAKE + i * 4 * n for i in range(6))
    base = FAKE + 8 * 4 * n
    fe = [L.fd_face_elems(C.byref(g), f) * 4 for f in range(6)]
    offs = np.concatenate([[0], np.cumsum(fe)])
    fin = (C.c_void_p * 6)(*[int(base + o) for o in offs[:6]])
    fout = (C.c_void_p * 6)(*[int(base + offs[6] + o) for o in offs[:6]])
    step = L.fd_step_exchange
    assert step(C.byref(g), a, b, None, q, None, None, fin, fout, None) == EINVAL   # NULL u_next
    assert step(C.byref(g), a, b, b, q, None, None, fin, fout, None) == EINVAL      # u_next == u
    src = _lib.fd_source(64, 0, 0, 1.0)
    assert step(C.byref(g), a, b, c, q, None, C.byref(src), fin, fout, None) == EINVAL
    # a face buffer inside a volume array
    bad = (C.c_void_p * 6)(*fin)
    bad[2] = b + 64
    assert step(C.byref(g), a, b, c, q, None, None, bad, fout, None) == EINVAL
    # receive and send sets overlapping
    assert step(C.byref(g), a, b, c, q, None, None, fin, fin, None) == EINVAL
    # a misaligned face pointer
    bad = (C.c_void_p * 6)(*fout)
    bad[0] = int(bad[0]) + 2
    assert step(C.byref(g), a, b, c, q, None, None, fin, bad, None) == EINVAL
    assert b"aligned" in L.fd_last_error()
    # native loop: a second face set needs the first, and must be distinct from it
    r = _lib.fd_run()
    r.u_prev, r.u, r.u_next, r.vdt2, r.nt = a, b, c, q, 1
    for f in range(6):
        r.send2[f] = fout[f]
    assert L.fd_forward_run(C.byref(g), C.byref(r), None) == EINVAL
    for f in range(6):
        r.send[f] = fout[f]
    assert L.fd_forward_run(C.byref(g), C.byref(r), None) == EINVAL
    # scaled adjoint
    sa = L.fd_adjoint_step_scaled
    assert sa(C.byref(g), None, b, c, q, None, None, None, None, None) == EINVAL    # b_nn required
    assert sa(C.byref(g), a, b, b, q, None, None, None, None, None) == EINVAL       # b_out == b_n1
    assert sa(C.byref(g), a, b, c, q, None, None, gg, None, None) == EINVAL         # no u_n
    assert sa(C.byref(g), a, b, c, q, None, u, q, None, None) == EINVAL            # g_b == vdt2
    assert L.fd_scatter_add_scaled(C.byref(g), a, FAKE, FAKE, None, None, 3, None) == EINVAL
    assert L.fd_scatter_add_scaled(C.byref(g), a, FAKE, FAKE, q, None, -1, None) == EINVAL
    assert L.fd_scatter_add_scaled(C.byref(g), a, FAKE, FAKE, q, None, 0, None) == 0
    assert L.fd_grad_finalize_scaled(C.byref(g), a, b, 0.0, c, None) == EINVAL
    assert L.fd_grad_finalize_scaled(C.byref(g), a, b, 1e-3, b, None) == EINVAL  # grad_m == vdt2


def test_halo_and_adjoint_argument_checks(L):
    EINVAL = _lib.FD_EINVAL
    small = grid(L, 3, 8, 8)
    faces = (C.c_void_p * 6)(FAKE, None, None, None, None, None)
    assert L.halo_pack(C.byref(small), FAKE, faces, None) == EINVAL    # nx < 4 on an x face
    assert L.halo_unpack(C.byref(small), FAKE, faces, None) == EINVAL
    assert L.halo_pack(C.byref(small), None, faces, None) == EINVAL
    assert L.halo_pack(C.byref(small), FAKE, None, None) == EINVAL
    pr = L.fd_halo_pack_record
    assert pr(C.byref(small), FAKE, faces, FAKE, 4, FAKE, None) == EINVAL  # nx < 4 on an x face
    ok_faces = (C.c_void_p * 6)(None, None, FAKE, None, None, None)
    assert pr(C.byref(small), None, ok_faces, FAKE, 4, FAKE, None) == EINVAL    # NULL u
    assert pr(C.byref(small), FAKE, ok_faces, FAKE, -1, FAKE, None) == EINVAL   # nrec < 0
    assert pr(C.byref(small), FAKE, ok_faces, None, 4, FAKE, None) == EINVAL    # NULL offsets
    assert pr(C.byref(small), FAKE, ok_faces, FAKE, 4, None, None) == EINVAL    # NULL row
    assert pr(None, FAKE, ok_faces, FAKE, 4, FAKE, None) == EINVAL
    g = grid(L)
    n = L.fd_grid_elems(C.byref(g)) * 4
    a, b, c, q, u, gg = (FAKE + i * 4 * n for i in range(6))
    assert L.fd_adjoint_step(C.byref(g), a, b, b, q, None, None, None, None, None) == EINVAL
    assert L.fd_adjoint_step(C.byref(g), a, b, c, q, None, None, gg, None, None) == EINVAL  # no u_n
    assert L.fd_adjoint_step(C.byref(g), a, b, c, q, None, u, b, None, None) == EINVAL  # g == a_n1
    src = _lib.fd_source(0, 0, 40, 1.0)
    assert L.fd_adjoint_step(C.byref(g), a, b, c, q, None, u, gg, C.byref(src), None) == EINVAL
    assert L.fd_adjoint_step(C.byref(g), a, b, a + 4, q, None, None, None, None, None) == EINVAL


def test_host_helpers(L):
    w = np.empty(8, np.float32)
    assert L.fd_ricker(w.ctypes.data, 8, 0, 1e-3, 15.0, 1.0 / 15) == 0
    assert L.fd_ricker(w.ctypes.data, 8, 0, -1.0, 15.0, 1.0 / 15) == _lib.FD_EINVAL
    e = np.empty(40, np.float32)
    emax = L.fd_sponge_eta_max(4500.0, 10.0, 0.4 * 10 / 4500.0, 16, 1e-3)
    assert abs(emax - 3 * np.log(1000) * 0.4 / 64) < 1e-12
    assert L.fd_sponge_eta_max(4500.0, 10.0, 1e-3, 0, 1e-3) == 0.0
    assert L.fd_sponge_eta_max(4500.0, 10.0, 1e-3, 16, 2.0) == _lib.FD_EINVAL
    assert L.fd_sponge_profile(e.ctypes.data, 40, 16, emax) == 0
    assert e[0] == e[-1] and e[16:24].max() == 0 and e[15] > 0
    g = grid(L, 10, 10, 10)
    ijk = np.array([[0, 0, 0], [9, 9, 9]], np.int32)
    off = np.empty(2, np.int64)
    assert L.fd_receiver_offsets(C.byref(g), ijk.ctypes.data, 2, off.ctypes.data) == 0
    assert off[0] == g.origin and off[1] == g.origin + 9 * (g.zstride + g.ystride + 1)
    ijk[1, 2] = 10
    assert L.fd_receiver_offsets(C.byref(g), ijk.ctypes.data, 2, off.ctypes.data) == _lib.FD_EINVAL
    assert L.fd_set_kchunk(-1) == _lib.FD_EINVAL
    assert L.fd_set_kchunk(0) == 0


def launch(L, nx, ny, nz, tile_rows=None):
    out = (C.c_int32 * 4)()
    assert L.fd_step_launch(C.byref(grid(L, nx, ny, nz)), out) == 0
    tx, ty, kc, zc = out
    rows = tile_rows or (16 if nx * ny * nz <= 1 << 20 else 32)  # 64 x 16 tiles up to 2^20 points
    assert (tx, ty) == (-(-nx // 64), -(-ny // rows))
    assert zc == -(-nz // kc) and 1 <= kc <= nz
    return kc, tx * ty * zc


def test_step_launch_shape(L):
    """The forward stencil's z chunk: 512 resident blocks of 8 waves make one round
    on 256 CUs; the choice fills one round where the x-y tiles allow it and never
    leaves a small second round (a 576-block launch of 384^3 took 210 us against 164
    at 432 blocks)."""
    assert launch(L, 512, 512, 512) == (128, 512)
    assert launch(L, 1024, 1024, 512) == (512, 512)
    assert launch(L, 256, 256, 256) == (16, 512)
    assert launch(L, 64, 64, 64) == (1, 256)  # small grids: 64 x 16 tiles, one-plane chunks
    assert L.fd_set_tiles(1) == 0
    try:
        assert launch(L, 64, 64, 64, tile_rows=32) == (1, 128)
        assert L.fd_set_tiles(2) == 0
        assert launch(L, 512, 512, 512, tile_rows=16) == (256, 512)
    finally:
        assert L.fd_set_tiles(0) == 0
    assert L.fd_set_tiles(6) == _lib.FD_EINVAL and L.fd_set_tiles(-1) == _lib.FD_EINVAL
    assert L.fd_set_tiles(3) == 0  # one thread per point; the marching shape is 64 x 16
    try:
        assert launch(L, 512, 512, 512, tile_rows=16) == (256, 512)
    finally:
        assert L.fd_set_tiles(0) == 0
    # which forward kernel a step takes (host only)
    out = (C.c_int32 * 6)()
    g = _lib.fd_grid()
    # (16-byte lanes with 64 x 64 tiles where a 128-wide tile column would be mostly
    # empty: 320 = 2.5 x 128, 257 = 2.008 x 128; not with the x faces inside)
    for shape, faces, want in (((64, 64, 64), 0, 0), ((64, 64, 64), 1, 0), ((512, 512, 512), 1, 3),
                               ((512, 512, 512), 0, 3), ((320, 320, 320), 1, 1),
                               ((320, 320, 320), 0, 4), ((192, 192, 192), 0, 1),
                               ((257, 256, 256), 0, 4), ((384, 384, 384), 0, 3),
                               ((1024, 1024, 512), 1, 3)):
        assert L.fd_grid_init(C.byref(g), *shape, 10.0, 10.0, 10.0) == 0
        assert L.fd_step_kernel(C.byref(g), faces, out) == 0
        assert out[0] == want, (shape, faces, list(out))
        if want == 3:
            assert (out[1], out[2]) == (128, 32) and 240 <= out[5] <= 256
        if want == 4:
            assert (out[1], out[2]) == (64, 64) and 240 <= out[5] <= 256
    assert L.fd_set_tiles(4) == 0
    try:
        assert L.fd_grid_init(C.byref(g), 64, 64, 64, 10.0, 10.0, 10.0) == 0
        assert L.fd_step_kernel(C.byref(g), 0, out) == 0 and out[0] == 3
        assert L.fd_grid_init(C.byref(g), 320, 320, 320, 10.0, 10.0, 10.0) == 0
        assert L.fd_step_kernel(C.byref(g), 0, out) == 0 and out[0] == 3
        assert L.fd_set_tiles(5) == 0
        assert L.fd_grid_init(C.byref(g), 512, 512, 512, 10.0, 10.0, 10.0) == 0
        assert L.fd_step_kernel(C.byref(g), 0, out) == 0 and out[0] == 4
        assert L.fd_step_kernel(C.byref(g), 1, out) == 0 and out[0] == 3  # faces: 128 x 32
    finally:
        assert L.fd_set_tiles(0) == 0
    assert L.fd_step_kernel(C.byref(g), 0, None) == _lib.FD_EINVAL
    for n in (102, 128, 192, 320, 384, 448):
        kc, blocks = launch(L, n, n, n)
        assert 400 <= blocks <= 512, (n, kc, blocks)
    kc, blocks = launch(L, 64, 32, 5000)  # one x-y tile, deep: split in z alone
    assert 448 <= blocks <= 512 and kc == -(-5000 // blocks)
    kc, blocks = launch(L, 64 * 20, 32 * 30, 64)  # 600 x-y tiles: never 1.17 rounds
    assert blocks % 600 == 0 and blocks != 600
    assert L.fd_set_kchunk(24) == 0
    try:
        assert launch(L, 512, 512, 512) == (24, 128 * 22)
    finally:
        assert L.fd_set_kchunk(0) == 0
    assert launch(L, 512, 512, 512) == (128, 512)
    out = (C.c_int32 * 4)()
    assert L.fd_step_launch(C.byref(grid(L)), None) == _lib.FD_EINVAL
    assert L.fd_step_launch(None, out) == _lib.FD_EINVAL


def test_receiver_plane_map(L):
    g = grid(L, 10, 6, 5)
    ijk = np.array([[3, 2, 4], [0, 0, 4], [9, 5, 4]], np.int32)
    m = np.empty(60, np.int32)
    k = C.c_int32(-7)
    assert L.fd_receiver_plane_map(C.byref(g), ijk.ctypes.data, 3, m.ctypes.data, C.byref(k)) == 0
    want = np.full(60, -1, np.int32)
    want[2 * 10 + 3], want[0], want[5 * 10 + 9] = 0, 1, 2
    assert np.array_equal(m, want) and k.value == 4
    EINVAL = _lib.FD_EINVAL
    for bad in ([[3, 2, 4], [0, 0, 3]],   # two planes
                [[3, 2, 4], [3, 2, 4]],   # the same point twice
                [[10, 2, 4]],             # outside the interior
                [[3, 2, 5]]):
        b = np.array(bad, np.int32)
        assert L.fd_receiver_plane_map(C.byref(g), b.ctypes.data, len(bad), m.ctypes.data,
                                       C.byref(k)) == EINVAL
    assert L.fd_receiver_plane_map(C.byref(g), ijk.ctypes.data, 0, m.ctypes.data, C.byref(k)) == EINVAL
    assert L.fd_receiver_plane_map(C.byref(g), None, 3, m.ctypes.data, C.byref(k)) == EINVAL
    assert L.fd_receiver_plane_map(C.byref(g), ijk.ctypes.data, 3, None, C.byref(k)) == EINVAL


def test_shot_footprint_and_server_argument_checks(L):
    d = _lib.fd_shot_desc()
    d.nx, d.ny, d.nz, d.nt = 256, 256, 256, 500
    d.dx = d.dy = d.dz = 10.0
    d.nrec = 256
    fp = L.fd_shot_footprint(C.byref(d))
    g = grid(L, 256, 256, 256)
    vol = (L.fd_grid_elems(C.byref(g)) * 4 + 255) // 256 * 256
    assert fp >= 4 * vol + 4 * 500 * 256 and fp % 256 == 0
    d.nt = 0
    assert L.fd_shot_footprint(C.byref(d)) == -1
    h = C.c_void_p()
    EINVAL = _lib.FD_EINVAL
    assert L.fd_server_create(C.byref(h), None, 1 << 30, 4, None, None) == EINVAL
    assert L.fd_server_create(C.byref(h), FAKE + 8, 1 << 30, 4, None, None) == EINVAL  # unaligned
    assert L.fd_server_create(C.byref(h), FAKE, 1 << 30, 0, None, None) == EINVAL
    assert L.fd_server_create(C.byref(h), FAKE, 1 << 30, 65, None, None) == EINVAL
    assert L.fd_server_create(C.byref(h), FAKE, 4096, 4, None, None) == _lib.FD_ENOMEM
    assert L.shot_submit(None, C.byref(d), C.byref(C.c_int64())) == EINVAL
    assert L.shot_poll(None, 1, None, 0, None) == EINVAL
    assert L.fd_server_set_admission(None, 0) == EINVAL


def test_forward_graph_argument_checks(L):
    """fd_forward_graph checks its run exactly as fd_forward_run does, before it
    records anything; launching or destroying a NULL graph is refused or a no-op."""
    g = grid(L)
    h = C.c_void_p()
    r = _lib.fd_run()
    assert L.fd_forward_graph(C.byref(g), C.byref(r), None) == _lib.FD_EINVAL
    assert L.fd_forward_graph(C.byref(g), C.byref(r), C.byref(h)) == _lib.FD_EINVAL
    assert b"NULL array" in L.fd_last_error()
    assert h.value is None
    r.u_prev, r.u, r.u_next, r.vdt2 = FAKE, FAKE, FAKE + 4, FAKE + 8
    assert L.fd_forward_graph(C.byref(g), C.byref(r), C.byref(h)) == _lib.FD_EINVAL
    assert b"distinct" in L.fd_last_error()
    assert L.fd_graph_launch(None, None) == _lib.FD_EINVAL
    assert L.fd_graph_destroy(None) == _lib.FD_OK


def test_block_gemm_argument_checks(L):
    """fd_block_gemm_f64 (Cannon's local product) refuses bad extents, NULL arrays,
    short leading dimensions and C overlapping A or B before any launch; empty
    products do nothing."""
    EINVAL = _lib.FD_EINVAL
    m, n, k = 40, 30, 20
    a, b, c = FAKE, FAKE + 8 * m * k, FAKE + 8 * (m * k + k * n)
    G = L.fd_block_gemm_f64
    assert G(-1, n, k, a, k, b, n, c, n, 1, None) == EINVAL
    assert G(m, n, -2, a, k, b, n, c, n, 1, None) == EINVAL
    assert G(m, n, k, None, k, b, n, c, n, 1, None) == EINVAL
    assert G(m, n, k, a, k, None, n, c, n, 1, None) == EINVAL
    assert G(m, n, k, a, k, b, n, None, n, 1, None) == EINVAL
    assert G(m, n, k, a, k - 1, b, n, c, n, 1, None) == EINVAL   # lda < k
    assert G(m, n, k, a, k, b, n - 1, c, n, 1, None) == EINVAL   # ldb < n
    assert G(m, n, k, a, k, b, n, c, n - 1, 1, None) == EINVAL   # ldc < n
    assert G(m, n, k, a, k, b, n, a + 8, n, 1, None) == EINVAL   # c overlaps a
    assert G(m, n, k, a, k, b, n, b + 8 * n, n, 1, None) == EINVAL  # c overlaps b
    assert G(0, n, k, a, k, b, n, c, n, 1, None) == 0            # nothing to do
    assert G(m, 0, k, a, k, b, n, c, n, 1, None) == 0
    assert G(0, 0, 0, None, 0, None, 0, None, 0, 0, None) == 0
