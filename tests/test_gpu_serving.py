"""GPU tests of the continuous-batching shot server (S8, S9).

Every shot's traces from the batched server must be bitwise equal to the same shot run
alone through fd_step_fused + record_receivers (the batched kernels run the same
per-point code); the smallest shots are also checked against the FP64 oracle
(relative L2 <= 1e-4).  Admission is checked under an arena that holds only a few
shots, with the buddy allocator, with many more shots than slots and admission
streams, under a cap on the points running at once and under the default launch-model
policy, with both kernel families in one step, and the error paths (oversize, unknown
id, unstable dt, shutdown, allocator change after submit) end as documented.
"""
import numpy as np
import pytest
import torch

import oracle as ora
from workloads import receivers_xline, serving_shots, smooth_velocity
from bitwise import same_bits

pytestmark = pytest.mark.gpu

api = pytest.importorskip("paper_2506_02486_amd.api")
serving = pytest.importorskip("paper_2506_02486_amd.serving")
_lib = pytest.importorskip("paper_2506_02486_amd._lib")


@pytest.fixture(scope="module", autouse=True)
def _device():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    torch.cuda.set_device(0)
    yield
    torch.cuda.synchronize()


@pytest.fixture(scope="module")
def model():
    n = 96
    v = smooth_velocity(n, n, n, seed=2, sigma=4.0)
    dt = ora.cfl_dt(v, 10.0)
    return v, torch.from_numpy(v).cuda(), dt, float(v.max())


def make_shots(model, count, lo=24, hi=72, nt=50, width=6, seed=3):
    v, vd, dt, vmax = model
    shots = []
    for s in serving_shots(count, seed=seed, lo=lo, hi=hi, margin=width):
        nx, ny, nz = s["nx"], s["ny"], s["nz"]
        rec = receivers_xline(nx, ny // 2, min(4, nz - 1))
        shots.append(serving.Shot(vd[:nz, :ny, :nx], nt, dt, s["src"], rec,
                                  sponge_width=width, sponge_vmax=vmax))
    return shots


def solo(shot):
    nx, ny, nz = shot.shape
    sim = api.Simulation(shot.v.contiguous(), dt=shot.dt, sponge_width=shot.sponge_width,
                         sponge_vmax=shot.sponge_vmax,
                         geom=api.Geometry(src=shot.src, rec=shot.rec))
    return sim.run(shot.nt).cpu().numpy()


def test_mix_equals_solo_bitwise_and_overlaps(model):
    shots = make_shots(model, 10)
    with serving.ShotServer(4 << 30, max_slots=4) as srv:
        ids = [srv.submit(s) for s in shots]
        res = [srv.wait(i) for i in ids]
        st = srv.stats()
    for shot, (code, tr, t) in zip(shots, res):
        assert code == _lib.FD_OK
        assert same_bits(tr, solo(shot))
        assert t[0] <= t[1] <= t[2]
    # FIFO admission, and shots really ran together: some shot was admitted before
    # an earlier-submitted one finished
    admits = [r[2][1] for r in res]
    assert admits == sorted(admits)
    assert any(res[i + 1][2][1] < res[i][2][2] for i in range(len(res) - 1))
    assert st["running"] == 0 and st["queued"] == 0
    # fewer launches than the plain loop would issue
    assert st["steps"] < sum(s.nt for s in shots)


def test_admission_cap_runs_shots_in_turn(model):
    """max_active_points = 1 admits a shot only when none runs: every batched step
    then advances exactly one shot, so the steps launched are the sum of the nt."""
    shots = make_shots(model, 4, nt=20, seed=5)
    with serving.ShotServer(2 << 30, max_slots=8, max_active_points=1) as srv:
        ids = [srv.submit(s) for s in shots]
        res = [srv.wait(i) for i in ids]
        st = srv.stats()
        with pytest.raises(_lib.FDError) as e:
            srv.set_admission(-1)
        assert e.value.code == _lib.FD_EINVAL
        srv.set_admission(0)  # no limit again: the next shot still runs
        assert srv.wait(srv.submit(shots[0]))[0] == _lib.FD_OK
    assert st["steps"] == sum(s.nt for s in shots)
    admits = [r[2][1] for r in res]
    assert admits == sorted(admits)
    for shot, (code, tr, _) in zip(shots, res):
        assert code == _lib.FD_OK
        assert same_bits(tr, solo(shot))


def test_receiver_rows_with_and_without_plane(model):
    """Shots whose receivers share one plane get their rows from the batched stencil
    kernel, the others from the batched receiver launch; in one mix both equal the
    solo runs bit for bit."""
    v, vd, dt, vmax = model
    shots = make_shots(model, 4, nt=25, seed=13)
    for i in (1, 3):  # receivers on two planes
        s = shots[i]
        nx, ny, nz = s.shape
        rec = np.concatenate([receivers_xline(nx, ny // 2, 2), receivers_xline(nx, ny // 3, nz - 3)])
        shots[i] = serving.Shot(s.v, s.nt, s.dt, s.src, rec, sponge_width=s.sponge_width,
                                sponge_vmax=s.sponge_vmax)
    with serving.ShotServer(2 << 30, max_slots=8) as srv:
        ids = [srv.submit(s) for s in shots]
        res = [srv.wait(i) for i in ids]
    for shot, (code, tr, _) in zip(shots, res):
        assert code == _lib.FD_OK
        assert same_bits(tr, solo(shot))


def test_plain_loop_equals_server(model):
    """The comparison loop of the serving benchmark (one shot at a time in the native
    step loop, the receiver row taken by the stencil) gives the server's bits."""
    shots = make_shots(model, 5, nt=30, seed=9)
    plain = serving.PlainLoop((72, 72, 72))
    want = [plain.run(s) for s in shots]
    with serving.ShotServer(2 << 30, max_slots=8) as srv:
        ids = [srv.submit(s) for s in shots]
        got = [srv.wait(i) for i in ids]
    for (code, tr, _), w in zip(got, want):
        assert code == _lib.FD_OK
        assert same_bits(tr, w)


def test_small_shots_match_oracle(model):
    v, _, dt, vmax = model
    shots = sorted(make_shots(model, 8, nt=40), key=lambda s: np.prod(s.shape))[:4]
    with serving.ShotServer(2 << 30, max_slots=8) as srv:
        ids = [srv.submit(s) for s in shots]
        res = [srv.wait(i) for i in ids]
    for shot, (code, tr, _) in zip(shots, res):
        nx, ny, nz = shot.shape
        eta = ora.sponge_tables(nx, ny, nz, shot.sponge_width, vmax, (10.0,) * 3, dt)
        want = ora.forward(v[:nz, :ny, :nx], shot.nt, dt, src=shot.src, w=ora.ricker(shot.nt, dt),
                           eta=eta, rec=shot.rec)[0]
        assert code == _lib.FD_OK
        assert np.linalg.norm(tr - want) <= 1e-4 * np.linalg.norm(want)


def test_admission_waits_for_arena_memory(model):
    shots = make_shots(model, 6, lo=56, hi=72, nt=30)
    biggest = max(s.footprint() for s in shots)
    arena = int(2.2 * biggest) + (2 << 20)
    with serving.ShotServer(arena, max_slots=8) as srv:
        ids = [srv.submit(s) for s in shots]
        res = [srv.wait(i) for i in ids]
    assert all(r[0] == _lib.FD_OK for r in res)
    # whenever a shot was admitted, the shots running at that moment fit the arena
    span = [(r[2][1], r[2][2], s.footprint()) for s, r in zip(shots, res)]
    for a, _, _ in span:
        live = sum(f for (a2, d2, f) in span if a2 <= a < d2)
        assert live <= arena
    # and memory, not slots, made some shot wait for another to finish
    assert any(any(d2 <= a for (_, d2, _) in span) for (a, _, _) in span[2:])
    for shot, r in zip(shots, res):
        assert same_bits(r[1], solo(shot))


def test_error_paths(model):
    v, vd, dt, vmax = model
    with serving.ShotServer(16 << 20, max_slots=2) as srv:
        big = serving.Shot(vd, 10, dt, (40, 40, 40))
        assert big.footprint() > (16 << 20)
        with pytest.raises(_lib.FDError) as e:
            srv.submit(big)                       # 4 padded 96^3 volumes > the arena
        assert e.value.code == _lib.FD_ENOMEM
        with pytest.raises(_lib.FDError) as e:
            srv.submit(serving.Shot(vd[:20, :20, :20], 10, dt, (25, 5, 5)))
        assert e.value.code == _lib.FD_EINVAL
        with pytest.raises(_lib.FDError) as e:
            srv.poll(12345)
        assert e.value.code == _lib.FD_ENOTFOUND
        unstable = serving.Shot(vd[:20, :20, :20], 10, 1.2 * 0.45286 * 10.0 / vmax, (5, 5, 5))
        code, tr, _ = srv.wait(srv.submit(unstable))
        assert code == _lib.FD_EINVAL and tr is None
        # with the sponge's design velocity given (or no sponge) the shot may join the
        # step before its stability check: found unstable it leaves the step, and a
        # shot running with it keeps its bits
        dt_bad = 1.2 * 0.45286 * 10.0 / vmax
        bad = [serving.Shot(vd[:20, :20, :20], 300, dt_bad, (5, 5, 5), sponge_width=4,
                            sponge_vmax=vmax),
               serving.Shot(vd[:20, :20, :20], 300, dt_bad, (5, 5, 5), sponge_width=0)]
        good = make_shots(model, 1, nt=40, seed=31)[0]
        ids = [srv.submit(bad[0]), srv.submit(good), srv.submit(bad[1])]
        res = [srv.wait(i) for i in ids]
        assert res[0][0] == _lib.FD_EINVAL and res[0][1] is None
        assert res[2][0] == _lib.FD_EINVAL and res[2][1] is None
        assert res[1][0] == _lib.FD_OK and same_bits(res[1][1], solo(good))
        ok = serving.Shot(vd[:20, :20, :20], 10, dt, (5, 5, 5), np.array([[1, 1, 1]], np.int32))
        sid = srv.submit(ok)
        assert srv.wait(sid)[0] == _lib.FD_OK
        with pytest.raises(_lib.FDError):
            srv.poll(sid)                         # already collected
        # queued shots are cancelled by shutdown; later submits fail
        long = [serving.Shot(vd[:32, :32, :32], 400, dt, (9, 9, 9)) for _ in range(4)]
        ids = [srv.submit(s) for s in long]
        srv.shutdown()
        codes = [srv.wait(i)[0] for i in ids]
        assert all(c in (_lib.FD_OK, _lib.FD_ECANCELED) for c in codes)
        assert codes[-1] == _lib.FD_ECANCELED
        with pytest.raises(_lib.FDError) as e:
            srv.submit(ok)
        assert e.value.code == _lib.FD_ECANCELED


def test_buddy_allocator_mix_equals_solo(model):
    shots = make_shots(model, 8, seed=21)
    with serving.ShotServer(3 << 30, max_slots=4, allocator="buddy") as srv:
        ids = [srv.submit(s) for s in shots]
        res = [srv.wait(i) for i in ids]
        with pytest.raises(_lib.FDError) as e:  # the allocator is fixed once shots came
            _lib.check(_lib.lib().fd_server_set_allocator(srv.h, _lib.FD_ARENA_FIRST_FIT),
                       "fd_server_set_allocator")
        assert e.value.code == _lib.FD_EINVAL
    for shot, (code, tr, t) in zip(shots, res):
        assert code == _lib.FD_OK
        assert same_bits(tr, solo(shot))
    with pytest.raises(ValueError):
        serving.ShotServer(1 << 20, allocator="slab")


def test_many_shots_few_slots_and_admission_streams(model):
    """40 short shots through 2 slots: admission work of up to four shots ahead runs on
    the bounded stream pool (reused, partially synchronised) while others step; strict
    FIFO activation and every trace equal to its solo run."""
    shots = make_shots(model, 40, lo=16, hi=40, nt=6, width=4, seed=17)
    with serving.ShotServer(2 << 30, max_slots=2) as srv:
        ids = [srv.submit(s) for s in shots]
        res = [srv.wait(i) for i in ids]
        st = srv.stats()
    assert st == {"queued": 0, "running": 0, "finished": 0, "steps": st["steps"]}
    admits = [r[2][1] for r in res]
    assert admits == sorted(admits)
    for shot, (code, tr, _) in zip(shots, res):
        assert code == _lib.FD_OK
        assert same_bits(tr, solo(shot))


def test_both_kernel_families_in_one_step():
    """A grid of at least 7.5M points running in the same steps as small grids: all of
    them then take the 16-byte-lane kernel, in one launch with their parameters as
    kernel arguments (the small grids' tiles fill the large grid's launch; receiver
    rows in the kernel; the small grids, whose 128-wide tile columns would be mostly
    empty, in 64 x 64 tiles and the large one in 128 x 32, then all of them in 64 x 64
    with fd_set_tiles(5)); ten small grids in the one-float-per-lane tile table; the
    same ten forced onto 16-byte lanes (fd_set_tiles(4)), more than one such launch
    carries, through its tile table: traces equal to the solo runs bit for bit."""
    v = smooth_velocity(200, 200, 192, seed=2, sigma=4.0)  # the 10 small grids fit inside
    vd = torch.from_numpy(v).cuda()
    dt = ora.cfl_dt(v, 10.0)
    vmax = float(v.max())

    def shot(nx, ny, nz, src):
        return serving.Shot(vd[:nz, :ny, :nx], 12, dt, src, receivers_xline(nx, ny // 2, 4),
                            sponge_width=8, sponge_vmax=vmax)

    mix = [shot(40, 36, 30, (20, 18, 15)), shot(200, 200, 192, (100, 90, 96)),
           shot(52, 47, 33, (26, 23, 16)), shot(37, 61, 29, (18, 30, 14))]
    many = [shot(20 + 3 * i, 18 + 2 * i, 12 + i, (9, 8, 6)) for i in range(10)]
    assert api.step_kernel(api.Grid(200, 200, 192))["kernel"] == "wide_128x32"
    for tiles, shots in ((0, mix), (5, mix), (0, many), (4, many)):
        api.set_tiles(tiles)
        try:
            with serving.ShotServer(4 << 30, max_slots=16, max_active_points=1 << 40) as srv:
                ids = [srv.submit(s) for s in shots]
                res = [srv.wait(i) for i in ids]
                st = srv.stats()
            # they ran together (the point cap lets every one join): fewer steps than shots
            # times steps
            assert st["steps"] < sum(s.nt for s in shots)
            for s, (code, tr, _) in zip(shots, res):
                assert code == _lib.FD_OK
                assert same_bits(tr, solo(s))
        finally:
            api.set_tiles(0)


def test_default_policy_runs_device_filling_grids_alone():
    """Under the default policy a shot joins running ones within 8,388,608 points, or
    within 16,777,216 while more shots wait behind it: grids of 37.7M points (384 x 384
    x 256), submitted together, run one after the other, each activated when the one
    before has finished; grids of 8.0M (200^3) share the steps two at a time while a
    backlog waits (small grids share them too:
    test_mix_equals_solo_bitwise_and_overlaps)."""
    v = smooth_velocity(384, 384, 256, seed=2, sigma=4.0)
    vd = torch.from_numpy(v).cuda()
    dt = ora.cfl_dt(v, 10.0)
    shots = [serving.Shot(vd, 15, dt, (192, 192, 100 + i), receivers_xline(384, 192, 4),
                          sponge_width=16, sponge_vmax=float(v.max())) for i in range(3)]
    with serving.ShotServer(10 << 30, max_slots=8) as srv:
        ids = [srv.submit(s) for s in shots]
        res = [srv.wait(i) for i in ids]
        st = srv.stats()
    assert all(r[0] == _lib.FD_OK for r in res)
    admits = [r[2][1] for r in res]
    assert admits == sorted(admits)
    assert st["steps"] == sum(s.nt for s in shots)  # never two of them in one step
    assert same_bits(res[1][1], solo(shots[1]))
    mid = [serving.Shot(vd[:200, :200, :200], 15, dt, (100, 100, 90 + i),
                        receivers_xline(200, 100, 4), sponge_width=16,
                        sponge_vmax=float(v.max())) for i in range(4)]
    with serving.ShotServer(10 << 30, max_slots=8) as srv:
        ids = [srv.submit(s) for s in mid]
        res = [srv.wait(i) for i in ids]
        st = srv.stats()
    assert all(r[0] == _lib.FD_OK for r in res)
    # two at a time (three would hold 24M points): between half the steps and all of them
    assert sum(s.nt for s in mid) // 2 <= st["steps"] < sum(s.nt for s in mid)
    for s, r in zip(mid, res):
        assert same_bits(r[1], solo(s))
