"""GPU parity of the forward path (S0-S7) against the FP64 oracle, through the C ABI.

Tolerances: the FP32 wavefield must match the FP64 oracle to relative L2 <= 1e-6 for one
step fed with the GPU's own state, and <= 1e-4 after 100 steps.  Integer/byte work
(pack/unpack, vdt2 rounding, dt) must be bit-exact.
"""
import numpy as np
import pytest
import torch

import oracle as ora
from workloads import (center_source, layered_velocity, random_field, receivers_plane,
                       receivers_xline, smooth_velocity)
from bitwise import same_bits

pytestmark = pytest.mark.gpu

api = pytest.importorskip("paper_2506_02486_amd.api")
D10 = (10.0, 10.0, 10.0)


def _random_state(g, seed):
    """(u_prev, u) padded device arrays with random interiors and zero halos."""
    out = []
    for s in (seed, seed + 1):
        t = g.zeros()
        g.interior(t).copy_(torch.from_numpy(random_field((g.nz, g.ny, g.nx), s)))
        out.append(t)
    return out


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def oracle_eta(sim, width, vmax, dt, d=D10):
    nz, ny, nx = sim.grid.nz, sim.grid.ny, sim.grid.nx
    return ora.sponge_tables(nx, ny, nz, width, vmax, d, dt)


@pytest.fixture(scope="module", autouse=True)
def _device():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    torch.cuda.set_device(0)
    yield
    torch.cuda.synchronize()


def test_setup_is_bit_exact_with_oracle():
    v = layered_velocity(37, 21, 19, seed=1)
    sim = api.Simulation(v, d=(10.0, 12.0, 9.0))
    dt_o = ora.cfl_dt(v, 9.0)
    assert sim.dt == dt_o
    q = sim.grid.interior(sim.vdt2).cpu().numpy()
    assert same_bits(q, ora.vdt2(v, dt_o).astype(np.float32))
    # face halos of vdt2 carry the periodic image, edges stay zero
    P = sim.grid.padded(sim.vdt2).cpu().numpy()
    assert same_bits(P[4:-4, 4:-4, :4], q[:, :, -4:])
    assert same_bits(P[4:-4, -4:, 4:-4], q[:, :4, :])
    assert same_bits(P[:4, 4:-4, 4:-4], q[-4:, :, :])
    assert np.all(P[:4, :4, :] == 0)
    w = api.ricker(50, dt_o)
    assert np.allclose(w, ora.ricker(50, dt_o), rtol=0, atol=2e-7)
    for n, width in ((37, 16), (21, 5)):
        emax = api.lib().fd_sponge_eta_max(4500.0, 10.0, dt_o, width, 1e-3)
        h = np.empty(n, np.float32)
        api.lib().fd_sponge_profile(h.ctypes.data, n, width, emax)
        assert np.allclose(h, ora.sponge_eta(n, width, 4500.0, 10.0, dt_o), rtol=1e-6, atol=0)


def test_config1_plain_forward_64cubed_100_steps():
    """64^3 layered model, Dirichlet, Ricker 15 Hz at the centre, receivers on k=0."""
    n = 64
    v = layered_velocity(n, n, n, seed=1)
    src = center_source(n, n, n)
    rec = receivers_plane(n, n, 0)
    sim = api.Simulation(v, geom=api.Geometry(src=src, rec=rec))
    tr = sim.run(100).cpu().numpy()
    dt = ora.cfl_dt(v, 10.0)
    w = ora.ricker(100, dt)
    tr_o, up_o, u_o = ora.forward(v, 100, dt, src=src, w=w, rec=rec)
    up, u = (x.cpu().numpy() for x in sim.state())
    assert rel_l2(u, u_o) <= 1e-4
    assert rel_l2(up, up_o) <= 1e-4
    assert rel_l2(tr, tr_o) <= 1e-4
    assert np.abs(tr).max() > 0


def _per_step_check(sim, steps, eta=(None, None, None), periodic=False):
    """Advance the GPU and, at each listed step, feed its FP32 (u^{n-1}, u^n) to one
    oracle step and compare u^{n+1} over the whole interior."""
    g = sim.grid
    q = ora.vdt2(g.interior(sim.v).cpu().numpy(), sim.dt)
    worst = 0.0
    last = sim.n
    for n in steps:
        if n > last:
            sim.run(n - last)
        up, u = (x.cpu().numpy() for x in sim.state())
        w_src = 0.0
        src = sim.geom.src
        if src is not None:
            w_src = float(ora.ricker(1, sim.dt, n0=n)[0])
        sim.run(1)
        got = g.interior(sim.u).cpu().numpy()
        k, j, i = np.meshgrid(np.arange(g.nz), np.arange(g.ny), np.arange(g.nx), indexing="ij")
        pts = np.stack([i.ravel(), j.ravel(), k.ravel()], 1).astype(np.int32)
        want = ora.step_points(up, u, q, pts, d=g.d, eta=eta, periodic=periodic, src=src,
                               w_src=w_src).reshape(got.shape)
        worst = max(worst, rel_l2(got, want))
        last = n + 1
    return worst


def test_config1_per_step_parity():
    n = 64
    v = layered_velocity(n, n, n, seed=1)
    sim = api.Simulation(v, geom=api.Geometry(src=center_source(n, n, n)))
    assert _per_step_check(sim, [1, 10, 40, 99]) <= 1e-6


@pytest.mark.parametrize("shape", [(100, 37, 45), (67, 19, 33), (130, 70, 9)])
def test_ragged_sponge_loopback_parity(shape):
    """Several tiles plus ragged tails in x and y, chunked z, sponge, periodic loopback
    exchange every step: 60 steps vs the oracle, then per-step parity."""
    nx, ny, nz = shape
    v = smooth_velocity(nx, ny, nz, seed=2, sigma=3.0)
    src = (nx // 3, ny // 2, nz // 2)
    rec = receivers_xline(nx, ny // 2, 4)
    width = 6
    sim = api.Simulation(v, sponge_width=width, exchange="loopback",
                         geom=api.Geometry(src=src, rec=rec))
    tr = sim.run(60).cpu().numpy()
    dt = sim.dt
    eta = oracle_eta(sim, width, float(v.max()), dt)
    tr_o, up_o, u_o = ora.forward(v, 60, dt, src=src, w=ora.ricker(60, dt), eta=eta,
                                  periodic=True, rec=rec)
    assert rel_l2(sim.state()[1].cpu().numpy(), u_o) <= 1e-4
    assert rel_l2(tr, tr_o) <= 1e-4
    assert _per_step_check(sim, [60, 75], eta=eta, periodic=True) <= 1e-6
    assert sim.n == 76


@pytest.mark.parametrize("shape,kernel", [((256, 136, 72), "march_64x32"),
                                          ((260, 200, 150), "wide_128x32"),
                                          ((300, 300, 300), "wide_64x64"),
                                          ((512, 512, 512), "wide_128x32")])
def test_marching_exchange_kernel_100_steps_vs_oracle(shape, kernel):
    """The benchmark's step path over 100 steps: fd_step_exchange with both face sets
    (loopback, periodic), sponge 16, Ricker source, centre x-line receivers, against the
    FP64 oracle's periodic forward run, for each z-marching kernel the automatic choice
    takes: 256 x 136 x 72 the kernel of one float per lane with the x faces inside (a
    ragged last tile row, 136 = 4 x 32 + 8, and several z chunks); 260 x 200 x 150 the
    kernel of 16-byte lanes without faces inside (ragged x and y tiles, rows whose last
    float4 holds one interior point); 300^3 the same kernel with 64 x 64 tiles (a
    128-wide tile column would be mostly empty); 512^3, the benchmark's own grid, the
    16-byte-lane kernel with the x faces inside."""
    nx, ny, nz = shape
    assert api.step_kernel(api.Grid(nx, ny, nz), faces=True)["kernel"] == kernel
    nt, width = 100, 16
    v = smooth_velocity(nx, ny, nz, seed=2)
    src = center_source(nx, ny, nz)
    rec = receivers_xline(nx, ny // 2, nz // 2)
    sim = api.Simulation(v, sponge_width=width, exchange="loopback",
                         geom=api.Geometry(src=src, rec=rec))
    tr = sim.run(nt).cpu().numpy()
    up, u = (x.cpu().numpy() for x in sim.state())
    dt = sim.dt
    eta = oracle_eta(sim, width, float(v.max()), dt)
    tr_o, up_o, u_o = ora.forward(v, nt, dt, src=src, w=ora.ricker(nt, dt), eta=eta,
                                  periodic=True, rec=rec)
    e = (rel_l2(u, u_o), rel_l2(up, up_o), rel_l2(tr, tr_o))
    print(f"{shape}: rel L2 after {nt} steps: u {e[0]:.2e}, u_prev {e[1]:.2e}, traces {e[2]:.2e}")
    assert np.abs(tr_o).max() > 0
    assert max(e) <= 1e-4


@pytest.mark.parametrize("shape", [(1, 1, 1), (3, 5, 2), (4, 4, 4), (65, 17, 1)])
def test_degenerate_small_grids(shape):
    nx, ny, nz = shape
    v = np.full((nz, ny, nx), 2000.0, np.float32)
    src = (nx // 2, ny // 2, nz // 2)
    sim = api.Simulation(v, geom=api.Geometry(src=src, rec=np.array([src], np.int32)))
    tr = sim.run(12).cpu().numpy()
    tr_o, _, u_o = ora.forward(v, 12, sim.dt, src=src, w=ora.ricker(12, sim.dt),
                               rec=np.array([src], np.int32))
    assert rel_l2(sim.state()[1].cpu().numpy(), u_o) <= 1e-5
    assert rel_l2(tr, tr_o) <= 1e-5


@pytest.mark.parametrize("shape", [(128, 40, 45), (70, 33, 29), (192, 80, 64), (128, 64, 40),
                                   (260, 36, 20), (256, 72, 30), (133, 21, 17), (135, 37, 12)])
def test_results_independent_of_launch_shape(shape):
    """The kernel shape (fd_set_tiles: 64 x 32 or 64 x 16 tiles, one thread per point,
    which the automatic choice takes for the fused form on these grids, or 128 x 32 tiles
    of 16-byte lanes -- ragged last x tiles of 64 and of 4 points, rows whose last float4
    holds 1, 2 or 3 interior points, and with the x faces inside where nx is a multiple
    of 128) and the z chunk (planes per block, fd_set_kchunk) change the launch, never
    the bits: forward runs in the exchange and fused forms and both adjoint steps give
    the same traces, fields and gradient accumulators in every shape, for chunks that end
    inside, at and past the 9- and 10-plane unrolled loops, one plane and the whole
    depth."""
    nx, ny, nz = shape
    v = smooth_velocity(nx, ny, nz, seed=2, sigma=3.0)
    geom = api.Geometry(src=(nx // 3, ny // 2, nz // 2), rec=receivers_xline(nx, ny // 3, nz // 3))

    def forward(mode):
        sim = api.Simulation(v, sponge_width=6, exchange="loopback", geom=geom)
        tr = sim.run(23, mode=mode)
        return [tr, sim.state()[0].clone(), sim.state()[1].clone()]

    def adjoint():
        sim = api.Simulation(v, sponge_width=6, geom=geom)
        g = sim.grid
        a_nn, a_n1 = _random_state(g, 11)
        u_n = _random_state(g, 13)[0]
        outs = []
        for scaled in (False, True):
            out, acc = g.zeros(), g.zeros()
            if scaled:
                api.adjoint_step_scaled(g, a_nn, a_n1, out, sim.vdt2, sim.sponge, u_n=u_n,
                                        g_b=acc, src=(geom.src, 0.7))
            else:
                api.adjoint_step(g, a_nn, a_n1, out, sim.vdt2, sim.sponge, u_n=u_n,
                                 g_vdt2=acc, src=(geom.src, 0.7))
            outs += [out, acc]
        return outs

    def signed_zeros():
        # a state of random values near the smallest subnormals: the update underflows
        # to zeros of both signs, and a point with eta == 0 must keep its sign whether
        # or not its tile holds damped points
        sim = api.Simulation(v, sponge_width=6, geom=api.Geometry())
        a, b = _random_state(sim.grid, 21)
        sim.u_prev.copy_(a * 1e-43)
        sim.u.copy_(b * 1e-43)
        sim.run(2, mode="fused")
        u = sim.state()[1]
        assert bool(((u == 0) & torch.signbit(u)).any()), "no -0 produced"
        return [sim.state()[0].clone(), u.clone()]

    def everything():
        return forward("exchange") + forward("fused") + adjoint() + signed_zeros()

    api.set_kchunk(0)
    api.set_tiles(0)
    ref = everything()
    try:
        for tiles in (1, 2, 3, 4, 5):
            api.set_tiles(tiles)
            for kc in (0, 1, 2, 5, 9, 10, 17, nz):
                api.set_kchunk(kc)
                for i, (a, b) in enumerate(zip(ref, everything())):
                    assert same_bits(a, b), (tiles, kc, i)
    finally:
        api.set_kchunk(0)
        api.set_tiles(0)


@pytest.mark.parametrize("mode", ["exchange", "fused", "separate", "native", "native-fused"])
def test_empty_runs_and_no_receivers(mode):
    """nt = 0 changes nothing and returns no trace rows; a model without receivers
    or source steps and returns an empty trace table."""
    nx, ny, nz = 64, 32, 9
    v = smooth_velocity(nx, ny, nz, seed=2, sigma=3.0)
    src = (5, 6, 4)
    sim = api.Simulation(v, sponge_width=3, exchange="loopback",
                         geom=api.Geometry(src=src, rec=np.array([src], np.int32)))
    sim.run(5, mode=mode)
    before = [t.clone() for t in sim.state()]
    tr = sim.run(0, mode=mode)
    assert tr.shape[0] == 0
    for a, b in zip(before, sim.state()):
        assert same_bits(a, b)
    assert sim.n == 5
    bare = api.Simulation(v, exchange="loopback")
    tr = bare.run(3, mode=mode)
    assert tr.shape == (3, 0)
    assert not torch.any(bare.state()[1])  # no source: the zero state stays zero


def test_in_place_two_array_stepping_matches_three_arrays():
    n = 40
    v = layered_velocity(n, n, n, seed=1)
    sim = api.Simulation(v, sponge_width=8)
    g = sim.grid
    rng = np.random.default_rng(3)
    a = torch.from_numpy(rng.standard_normal(g.elems).astype(np.float32)).cuda()
    b = torch.from_numpy(rng.standard_normal(g.elems).astype(np.float32)).cuda()
    for t in (a, b):  # Dirichlet halos
        P = g.padded(t)
        P[:4] = 0; P[-4:] = 0; P[:, :4] = 0; P[:, -4:] = 0; P[:, :, :4] = 0; P[:, :, -4:] = 0
    out = g.zeros()
    api.step(g, a, b, out, sim.vdt2, sim.sponge)
    a2 = a.clone()
    api.step(g, a2, b, a2, sim.vdt2, sim.sponge)
    torch.cuda.synchronize()
    assert same_bits(g.interior(out), g.interior(a2))


def test_mirror_symmetry_is_bitwise():
    n = 45
    a = smooth_velocity(n, n, n, seed=7, sigma=3.0).astype(np.float64)
    for ax in range(3):
        a = 0.5 * (a + np.flip(a, axis=ax))
    v = a.astype(np.float32)
    sim = api.Simulation(v, sponge_width=8, geom=api.Geometry(src=(22, 22, 22)))
    sim.run(50)
    u = sim.state()[1].cpu().numpy()
    assert np.abs(u).max() > 0
    for ax in range(3):
        assert same_bits(u, np.flip(u, axis=ax))


def test_resume_is_bitwise():
    n = 48
    v = layered_velocity(n, n, n, seed=1)
    geom = api.Geometry(src=(20, 24, 26), rec=receivers_plane(n, n, 2))
    a = api.Simulation(v, sponge_width=6, geom=geom, exchange="loopback")
    ta = torch.cat([a.run(30), a.run(20)])
    b = api.Simulation(v, sponge_width=6, geom=geom, exchange="loopback")
    tb = b.run(50)
    assert same_bits(ta, tb)
    assert same_bits(a.state()[1], b.state()[1])


@pytest.mark.parametrize("shape,tiles", [((64, 64, 64), 0), ((70, 33, 29), 1), ((70, 33, 29), 2),
                                         ((256, 100, 48), 0), ((128, 64, 40), 1),
                                         ((70, 33, 29), 3), ((70, 33, 29), 4),
                                         ((256, 100, 48), 4), ((135, 37, 12), 4),
                                         ((70, 33, 29), 5), ((135, 37, 12), 5),
                                         ((260, 200, 150), 0), ((300, 260, 100), 0)])
@pytest.mark.parametrize("faces", [0, 1, 2])
def test_receiver_plane_in_stencil_matches_separate_record(shape, tiles, faces):
    """fd_forward_run with a receiver plane map (the stencil launch writes the trace
    row where no faces are packed) gives the bits of the separate receiver launch,
    for Dirichlet runs (faces=0) and the loopback exchange in both forms; with tile
    mode 4 and on the 7.8M-point grid the Dirichlet steps take the 16-byte-lane
    kernel, which loads its receiver map entries before it marches."""
    nx, ny, nz = shape
    if faces == 0 and (tiles in (4, 5) or nx * ny * nz > 7_500_000):
        api.set_tiles(tiles)
        try:
            assert api.step_kernel(api.Grid(nx, ny, nz), faces=False)["kernel"] == (
                "wide_64x64" if tiles == 5 or (nx, ny, nz) == (300, 260, 100) else "wide_128x32")
        finally:
            api.set_tiles(0)
    v = smooth_velocity(nx, ny, nz, seed=2, sigma=3.0)
    rng = np.random.default_rng(11)
    pts = rng.choice(nx * ny, size=min(700, nx * ny), replace=False)
    rec = np.stack([pts % nx, pts // nx, np.full(pts.size, nz // 3)], axis=1).astype(np.int32)
    geom = api.Geometry(src=(nx // 2, ny // 2, nz // 2), rec=rec)
    api.set_tiles(tiles)
    try:
        out = []
        for use_map in (False, True):
            sim = api.Simulation(v, sponge_width=5, geom=geom,
                                 exchange="loopback" if faces else None)
            assert sim.rec_plane is not None and sim.rec_plane.k == nz // 3
            if not use_map:
                sim.rec_plane = None
            tr = sim.run(31, mode="native" if faces != 2 else "native-fused")
            out.append((tr.clone(), sim.state()[0].clone(), sim.state()[1].clone()))
        for a, b in zip(*out):
            assert same_bits(a, b)
    finally:
        api.set_tiles(0)


@pytest.mark.parametrize("nx,ny,nz", [(70, 9, 13), (72, 9, 13), (8, 5, 4), (128, 40, 33)])
def test_pack_record_equals_pack_and_record(nx, ny, nz):
    """fd_halo_pack_record (one launch where the faces take 16-byte accesses, two
    otherwise) writes the same faces and receiver row as halo_pack and
    record_receivers, with all faces, only the y/z faces, none, and no receivers."""
    g = api.Grid(nx, ny, nz)
    u = _random_state(g, 5)[0]
    rng = np.random.default_rng(3)
    ijk = np.stack([rng.integers(0, m, 300) for m in (nx, ny, nz)], axis=1).astype(np.int32)
    off = torch.from_numpy(g.offsets(ijk)).cuda()
    for keep in (range(6), range(2, 6), ()):
        want, got = api.face_buffers(g), api.face_buffers(g)
        for f in range(6):
            if f not in keep:
                want[f] = got[f] = None
        row_want = torch.full((300,), -1.0, device="cuda")
        row_got = torch.full((300,), -1.0, device="cuda")
        if keep:
            api.halo_pack(g, u, want)
        api.record_receivers(g, u, off, row_want)
        api.halo_pack_record(g, u, got, off, row_got)
        assert same_bits(row_got, row_want)
        for a, b in zip(got, want):
            assert (a is None and b is None) or same_bits(a, b)
        empty = api.face_buffers(g)
        api.halo_pack_record(g, u, empty)  # no receivers: the pack alone
        ref = api.face_buffers(g)
        api.halo_pack(g, u, ref)
        for a, b in zip(empty, ref):
            assert same_bits(a, b)


@pytest.mark.parametrize("nx,ny,nz", [(70, 9, 13), (72, 9, 13), (8, 5, 4)])
def test_pack_unpack_bit_exact(nx, ny, nz):
    """nx = 70 takes the scalar kernels; nx a multiple of 4 the 16-byte ones."""
    g = api.Grid(nx, ny, nz)
    u = torch.from_numpy(random_field((g.elems,), 5)).cuda()
    faces = api.face_buffers(g)
    api.halo_pack(g, u, faces)
    I = g.interior(u).cpu().numpy()
    f = [x.cpu().numpy() for x in faces]
    assert same_bits(f[0].reshape(nz, ny, 4), I[:, :, :4])
    assert same_bits(f[1].reshape(nz, ny, 4), I[:, :, -4:])
    assert same_bits(f[2].reshape(nz, 4, nx), I[:, :4, :])
    assert same_bits(f[3].reshape(nz, 4, nx), I[:, -4:, :])
    assert same_bits(f[4].reshape(4, ny, nx), I[:4])
    assert same_bits(f[5].reshape(4, ny, nx), I[-4:])
    before = g.padded(u).cpu().numpy()
    api.halo_unpack(g, u, api.loopback(faces))
    P = g.padded(u).cpu().numpy()
    assert same_bits(P[4:-4, 4:-4, :4], I[:, :, -4:])
    assert same_bits(P[4:-4, 4:-4, -4:], I[:, :, :4])
    assert same_bits(P[4:-4, :4, 4:-4], I[:, -4:, :])
    assert same_bits(P[4:-4, -4:, 4:-4], I[:, :4, :])
    assert same_bits(P[:4, 4:-4, 4:-4], I[-4:])
    assert same_bits(P[-4:, 4:-4, 4:-4], I[:4])
    # interior, edges and corners untouched
    assert same_bits(P[4:-4, 4:-4, 4:-4], before[4:-4, 4:-4, 4:-4])
    assert same_bits(P[:4, :4], before[:4, :4])
    # a NULL face leaves its halo alone
    full = g.zeros()
    g.padded(full).copy_(torch.from_numpy(before))
    api.halo_unpack(g, full, [None, faces[0], None, None, None, None])
    P2 = g.padded(full).cpu().numpy()
    assert same_bits(P2[4:-4, 4:-4, :4], before[4:-4, 4:-4, :4])
    assert same_bits(P2[4:-4, 4:-4, -4:], I[:, :, :4])
    assert same_bits(P2[4:-4, :4], before[4:-4, :4])


def test_full_size_512_sampled_per_step_parity():
    """The benchmark's own shape and launch configuration (512^3, sponge 16, loopback
    exchange): after 30 steps, one GPU step is checked against the oracle at sampled
    points (faces, edges, corners, sponge, source, random interior)."""
    n = 512
    v = smooth_velocity(n, n, n, seed=2)
    src = center_source(n, n, n)
    sim = api.Simulation(v, sponge_width=16, exchange="loopback", geom=api.Geometry(src=src))
    sim.run(30)
    up, u = (x.cpu().numpy() for x in sim.state())
    w_src = float(ora.ricker(1, sim.dt, n0=30)[0])
    sim.run(1)
    got = sim.state()[1].cpu().numpy()
    rng = np.random.default_rng(9)
    edge = np.array([0, 1, 3, 4, 15, 16, 17, 63, 64, 255, 256, 494, 495, 496, 507, 508, 510, 511])
    pts = [np.stack(np.meshgrid(edge, edge, edge, indexing="ij"), -1).reshape(-1, 3)]
    pts.append(rng.integers(0, n, size=(4000, 3)))
    pts.append(np.array([src]) + rng.integers(-6, 7, size=(500, 3)))
    pts = np.ascontiguousarray(np.concatenate(pts), dtype=np.int32)
    q = ora.vdt2(v, sim.dt)
    eta = ora.sponge_tables(n, n, n, 16, float(v.max()), D10, sim.dt)
    want = ora.step_points(up, u, q, pts, eta=eta, periodic=True, src=src, w_src=w_src)
    gv = got[pts[:, 2], pts[:, 1], pts[:, 0]]
    assert np.abs(want).max() > 0
    assert rel_l2(gv, want) <= 1e-6
    assert np.abs(gv - want).max() <= 1e-5 * np.abs(want).max()


def test_full_size_512_random_state_one_step():
    """512^3, sponge 16, loopback, the launch configuration of the benchmark, from a
    random state (nonzero on every face, edge and corner): one fused step against the
    oracle at sampled points, so the halo exchange and the tile/chunk boundaries are
    exercised at full size."""
    n = 512
    v = smooth_velocity(n, n, n, seed=2)
    src = center_source(n, n, n)
    sim = api.Simulation(v, sponge_width=16, exchange="loopback", geom=api.Geometry(src=src))
    up = random_field((n, n, n), 21)
    u = random_field((n, n, n), 22)
    sim.grid.interior(sim.u_prev).copy_(torch.from_numpy(up))
    sim.grid.interior(sim.u).copy_(torch.from_numpy(u))
    sim._faces_current = False  # the faces of the new u^n are packed by the next run
    w_src = float(ora.ricker(1, sim.dt, n0=0)[0])
    sim.run(1)
    got = sim.state()[1].cpu().numpy()
    rng = np.random.default_rng(11)
    edge = np.array([0, 1, 2, 3, 4, 5, 31, 32, 63, 64, 127, 128, 255, 256, 383, 384, 447, 448,
                     506, 507, 508, 509, 510, 511])
    pts = [np.stack(np.meshgrid(edge, edge, edge, indexing="ij"), -1).reshape(-1, 3)]
    pts.append(rng.integers(0, n, size=(6000, 3)))
    pts.append(np.array([src]))
    pts = np.ascontiguousarray(np.concatenate(pts), dtype=np.int32)
    q = ora.vdt2(v, sim.dt)
    eta = ora.sponge_tables(n, n, n, 16, float(v.max()), D10, sim.dt)
    want = ora.step_points(up, u, q, pts, eta=eta, periodic=True, src=src, w_src=w_src)
    gv = got[pts[:, 2], pts[:, 1], pts[:, 0]]
    assert rel_l2(gv, want) <= 1e-6
    assert np.abs(gv - want).max() <= 1e-5 * np.abs(want).max()


def test_full_size_512_energy_is_conserved_across_the_periodic_wrap():
    """Property at full size: with no sponge and no source, the leapfrog conserves
    I^n = sum (u^n^2 - u^{n+1} u^{n-1}) / vdt2 (the discrete energy, written with
    L u^n = (u^{n+1} - 2u^n + u^{n-1}) / vdt2).  A Gaussian pulse centred on a corner
    of the 512^3 periodic (loopback) box crosses every face, edge and corner halo."""
    n = 512
    v = smooth_velocity(n, n, n, seed=2)
    sim = api.Simulation(v, exchange="loopback")
    g = sim.grid
    ax = torch.arange(n, dtype=torch.float64, device="cuda")
    d1 = torch.minimum(ax, n - ax)  # periodic distance to index 0
    e = torch.exp(-(d1 / 3.0) ** 2 / 2)
    pulse = (e[:, None, None] * e[None, :, None] * e[None, None, :]).float()
    g.interior(sim.u_prev).copy_(pulse)
    g.interior(sim.u).copy_(pulse)
    sim._faces_current = False
    del pulse
    q = g.interior(sim.vdt2).double()

    def energy(a, b, c):
        return float(((b.double() ** 2 - c.double() * a.double()) / q).sum())

    hist = [g.interior(sim.u).clone()]
    I = []
    for _ in range(40):
        sim.run(1)
        hist.append(g.interior(sim.u).clone())
        if len(hist) == 3:
            I.append(energy(*hist))
            hist.pop(0)
    I = np.array(I)
    assert I[0] > 0
    assert np.abs(I - I[0]).max() <= 1e-4 * I[0]
    # nothing reached the centre of the box (the support grows 4 cells per step)
    assert float(g.interior(sim.u)[n // 2, n // 2, n // 2]) == 0.0


@pytest.mark.parametrize("shape,width", [((100, 37, 45), 6), ((64, 64, 64), 16), ((9, 70, 5), 2),
                                         ((64, 32, 37), 5), ((128, 96, 4), 3), ((192, 64, 9), 4),
                                         ((64, 37, 11), 4), ((128, 5, 4), 1), ((64, 32, 48), 0),
                                         ((30, 20, 12), 0)])
def test_step_modes_match_bitwise(shape, width):
    """fd_step_exchange (x faces inside the stencil kernel where nx % 64 == 0, else
    unpack, step and pack launches), fd_step_fused after halo_unpack, the separate
    calls halo_pack, halo_unpack, fd_step, inject_source, and the native loops of the
    exchange and fused forms: the same traces, fields and faces, bit for bit."""
    nx, ny, nz = shape
    v = smooth_velocity(nx, ny, nz, seed=2, sigma=3.0)
    src = (1, ny // 2, nz // 2)  # inside the x sponge
    geom = api.Geometry(src=src, rec=receivers_xline(nx, ny // 3, nz // 2))
    runs = []
    for mode in api.Simulation.MODES:
        sim = api.Simulation(v, sponge_width=width, exchange="loopback", geom=geom)
        tr = sim.run(37, mode=mode)
        tr2 = sim.run(4, mode=mode)
        runs.append((torch.cat([tr, tr2]), sim.state()[0].clone(), sim.state()[1].clone()))
        if mode != "separate":  # the send buffers hold the faces of the current u
            ref = api.face_buffers(sim.grid)
            api.halo_pack(sim.grid, sim.u, ref)
            for a, b in zip(sim.send, ref):
                assert same_bits(a, b), mode
    for mode, other in zip(api.Simulation.MODES[1:], runs[1:]):
        for a, b in zip(runs[0], other):
            assert same_bits(a, b), mode


@pytest.mark.parametrize("use_exchange_call", [False, True])
def test_two_subdomains_exchanging_faces_equal_one_domain(use_exchange_call):
    """Domain decomposition on one device: a periodic 64 x 32 x 48 domain split into
    two z slabs of 24 planes, each slab exchanging its z faces with the other (the
    -z halo of one receives the +z face of the other) and its x/y faces with itself,
    reproduces the undivided domain bit for bit after 30 steps -- the exchange a
    slab decomposition over several GPUs would run, with the puts replaced by
    passing the other slab's send buffers."""
    nx, ny, nz, nt = 64, 32, 48, 30
    v = smooth_velocity(nx, ny, nz, seed=2, sigma=3.0)
    src = (10, 11, 5)
    whole = api.Simulation(v, exchange="loopback", geom=api.Geometry(src=src))
    whole.run(nt, mode="separate")
    dt = whole.dt
    w = api.ricker(nt, dt)  # the wavelet the undivided run used
    slabs = [api.Simulation(v[:24], dt=dt), api.Simulation(v[24:], dt=dt)]
    g = slabs[0].grid
    send = [[api.face_buffers(g) for _ in range(2)] for _ in range(2)]  # [slab][set]
    for n in range(nt):
        cur, nxt = n % 2, (n + 1) % 2
        if n == 0:
            for i in range(2):
                api.halo_pack(g, slabs[i].u, send[i][cur])
        recv = []
        for i in range(2):
            own, other = send[i][cur], send[1 - i][cur]
            recv.append([own[1], own[0], own[3], own[2], other[5], other[4]])
        for i, sl in enumerate(slabs):
            s = (src, float(w[n])) if i == 0 else None
            if use_exchange_call:
                api.step_exchange(g, sl.u_prev, sl.u, sl.u_next, sl.vdt2, None, s, recv[i],
                                  send[i][nxt])
            else:
                api.halo_unpack(g, sl.u, recv[i])
                api.step_fused(g, sl.u_prev, sl.u, sl.u_next, sl.vdt2, None, s, send[i][nxt])
            sl.u_prev, sl.u, sl.u_next = sl.u, sl.u_next, sl.u_prev
    got = torch.cat([sl.state()[1] for sl in slabs], dim=0)
    assert same_bits(got, whole.state()[1])
    assert float(got.abs().max()) > 0


def test_exchange_step_reads_only_the_receive_buffers():
    """With face_in given, the one-kernel step does not read u's face halos: garbage
    there changes nothing; and a NULL face_in entry falls back to u's own halo."""
    nx, ny, nz = 64, 32, 20
    v = smooth_velocity(nx, ny, nz, seed=2, sigma=3.0)
    sim = api.Simulation(v, sponge_width=3, exchange="loopback")
    g = sim.grid
    up, u = _random_state(g, 31)
    faces = api.face_buffers(g)
    api.halo_pack(g, u, faces)
    recv = api.loopback(faces)
    out1, out2 = g.zeros(), g.zeros()
    api.step_exchange(g, up, u, out1, sim.vdt2, sim.sponge, None, recv, None)
    ref = g.zeros()
    u_ref = u.clone()
    api.halo_unpack(g, u_ref, recv)
    api.step(g, up, u_ref, ref, sim.vdt2, sim.sponge)
    assert same_bits(g.interior(out1), g.interior(ref))
    # poison u's halo (interior kept): the result does not change
    P = g.padded(u)
    keep = g.interior(u).clone()
    P.fill_(float("nan"))
    g.interior(u).copy_(keep)
    api.step_exchange(g, up, u, out2, sim.vdt2, sim.sponge, None, recv, None)
    assert same_bits(g.interior(out2), g.interior(ref))
    # a NULL entry reads u's own halo on that face: with u's halo poisoned (again:
    # the call above may have left the received values in it) the -z
    # neighbourhood (k < 4) turns NaN and nothing else does
    P.fill_(float("nan"))
    g.interior(u).copy_(keep)
    recv_nz = list(recv)
    recv_nz[4] = None
    out3 = g.zeros()
    api.step_exchange(g, up, u, out3, sim.vdt2, sim.sponge, None, recv_nz, None)
    I3 = g.interior(out3)
    assert torch.isnan(I3[:4]).all()
    assert same_bits(I3[4:], g.interior(ref)[4:])


@pytest.mark.parametrize("tiles", [0, 1])
@pytest.mark.parametrize("nz,kc", [(20, 0), (20, 3), (5, 0), (4, 1)])
def test_exchange_step_with_all_faces_matches_separate_calls(tiles, nz, kc):
    """fd_step_exchange with all twelve face buffers (x faces inside the stencil
    kernel, y and z faces unpacked and packed around it) on a grid the tiles cover
    exactly: with NaN in every halo cell of u, u_next and the six sent faces are bit
    for bit those of halo_unpack + fd_step + inject_source + halo_pack, also for z
    chunks that split the z faces and for grids whose planes are all in both z
    faces; u's edge and corner halo cells, which no point reads, keep their NaN."""
    nx, ny = 64, 32
    v = smooth_velocity(nx, ny, nz, seed=2, sigma=3.0)
    api.set_tiles(tiles)
    api.set_kchunk(kc)
    try:
        sim = api.Simulation(v, sponge_width=3, exchange="loopback")
        g = sim.grid
        up, u = _random_state(g, 37)
        faces = api.face_buffers(g)
        api.halo_pack(g, u, faces)
        recv = api.loopback(faces)
        u_ref = u.clone()
        api.halo_unpack(g, u_ref, recv)
        ref = g.zeros()
        src = (5, 7, nz // 2)
        api.step(g, up, u_ref, ref, sim.vdt2, sim.sponge)
        api.inject_source(g, ref, sim.vdt2, sim.sponge, src, 0.37)
        ref_faces = api.face_buffers(g)
        api.halo_pack(g, ref, ref_faces)
        P = g.padded(u)
        keep = g.interior(u).clone()
        P.fill_(float("nan"))
        g.interior(u).copy_(keep)
        out = g.zeros()
        sent = api.face_buffers(g)
        for f in sent:
            f.fill_(float("nan"))
        api.step_exchange(g, up, u, out, sim.vdt2, sim.sponge, (src, 0.37), recv, sent)
        assert same_bits(g.interior(out), g.interior(ref))
        for a, b in zip(sent, ref_faces):
            assert same_bits(a, b)
        assert bool(torch.isnan(P).any())  # edges and corners are never written
    finally:
        api.set_kchunk(0)
        api.set_tiles(0)


@pytest.mark.parametrize("case", ["dirichlet", "exchange", "fused"])
def test_forward_graph_replays_match_eager_runs(case):
    """fd_forward_graph records a forward run once; every launch re-runs it from a
    zero state (whatever the arrays held) with the bits of the eager native loop, with
    eager work and synchronisations between launches, and a new model written into
    vdt2 is picked up by the next launch: the 64^3 layered receiver-plane run, and
    the loopback exchange with a sponge in its one-kernel and fused forms."""
    if case == "dirichlet":
        nx = ny = nz = 64
        v = layered_velocity(nx, ny, nz, seed=1)
        geom = api.Geometry(src=center_source(nx, ny, nz), rec=receivers_plane(nx, ny, 0))
        width, exchange, mode, nt = 0, None, "native", 100
    else:
        nx, ny, nz = 64, 32, 24
        v = smooth_velocity(nx, ny, nz, seed=2, sigma=3.0)
        geom = api.Geometry(src=(5, 7, 11), rec=receivers_xline(nx, ny // 2, nz // 3))
        width, exchange, nt = 4, "loopback", 40
        mode = "native" if case == "exchange" else "native-fused"

    def eager(vel, dt=None):
        sim = api.Simulation(vel, sponge_width=width, exchange=exchange, geom=geom, dt=dt)
        tr = sim.run(nt, mode=mode).clone()
        return sim, tr, sim.state()[0].clone(), sim.state()[1].clone()

    ref, tr_ref, up_ref, u_ref = eager(v)
    sim = api.Simulation(v, sponge_width=width, exchange=exchange, geom=geom)
    g = sim.grid
    send = sim.send if exchange else None
    send2 = sim.send2 if case == "exchange" else None

    def poison():  # whole padded arrays (halos too) and face buffers: the graph must
        # start from zero anyway
        for a in (sim.u_prev, sim.u, sim.u_next):
            a.copy_(torch.randn_like(a))
        for f in (send or []) + (send2 or []):
            f.copy_(torch.randn_like(f))

    tr = torch.full((nt, sim.nrec), float("nan"), device="cuda")
    poison()
    G = api.ForwardGraph(g, sim.u_prev, sim.u, sim.u_next, sim.vdt2, sim.sponge, nt,
                         src=geom.src, wavelet=api.ricker(nt, sim.dt), rec_off=sim.rec_off,
                         traces=tr, send=send, send2=send2, rec_plane=sim.rec_plane)
    try:
        for rep in range(3):
            tr.fill_(float("nan"))
            G.launch()
            torch.cuda.synchronize()
            assert same_bits(tr, tr_ref), rep
            assert same_bits(g.interior(G.u_prev), up_ref), rep
            assert same_bits(g.interior(G.u), u_ref), rep
            if send is not None:  # the faces of the final u
                faces = api.face_buffers(g)
                api.halo_pack(g, G.u, faces)
                for a, b in zip(G.send, faces):
                    assert same_bits(a, b), rep
            x = torch.randn(1 << 16, device="cuda")
            assert float((x * 2).sum()) == float((x * 2).sum())
            poison()
            torch.cuda.synchronize()
        if case == "dirichlet":  # a new model in the same vdt2 array
            other, tr_o, up_o, u_o = eager(v * 0.95, dt=ref.dt)
            sim.vdt2.copy_(other.vdt2)
            G.launch()
            torch.cuda.synchronize()
            assert same_bits(tr, tr_o)
            assert same_bits(g.interior(G.u), u_o)
            assert not same_bits(tr_o, tr_ref)
    finally:
        G.close()


def test_large_subdomain_sampled_parity():
    """1024 x 1024 x 512 (four padded volumes of 2.3 GB), the smooth model, 16-cell
    sponge, Dirichlet halo, receivers on x = 0..1023 at y = 512, z = 4: after 12 steps
    one GPU step is checked against the oracle at sampled points, and the receiver row
    of that step against the same oracle values."""
    nx, ny, nz = 1024, 1024, 512
    v = smooth_velocity(nx, ny, nz, seed=2)
    src = center_source(nx, ny, nz)
    rec = receivers_xline(nx, 512, 4)
    sim = api.Simulation(v, sponge_width=16, geom=api.Geometry(src=src, rec=rec))
    sim.run(12)
    up, u = (x.cpu().numpy() for x in sim.state())
    w_src = float(ora.ricker(1, sim.dt, n0=12)[0])
    tr = sim.run(1).cpu().numpy()[0]
    got = sim.state()[1].cpu().numpy()
    rng = np.random.default_rng(10)
    pts = [rec[::37], np.stack([rng.integers(0, n, 3000) for n in (nx, ny, nz)], 1),
           np.array([src]) + rng.integers(-5, 6, size=(300, 3)),
           np.array([[0, 0, 0], [nx - 1, ny - 1, nz - 1], [0, ny - 1, 3], [nx - 1, 0, nz - 4]])]
    pts = np.ascontiguousarray(np.concatenate(pts), dtype=np.int32)
    q = ora.vdt2(v, sim.dt)
    eta = ora.sponge_tables(nx, ny, nz, 16, float(v.max()), D10, sim.dt)
    want = ora.step_points(up, u, q, pts, eta=eta, src=src, w_src=w_src)
    gv = got[pts[:, 2], pts[:, 1], pts[:, 0]]
    assert rel_l2(gv, want) <= 1e-6
    # the receiver row is u^{n+1} at the receivers
    assert same_bits(tr, got[4, 512, :])
