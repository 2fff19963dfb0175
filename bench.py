"""Benchmark of the acoustic FD hot path on one MI355X.

``python bench.py [--gpus 1] [--steps K] [--warmup W]`` times K time steps of the
single-subdomain workload -- a 512^3 interior with a radius-4 halo, smooth random
velocity in [1500, 4500] m/s, 16-cell quadratic sponge, 15 Hz Ricker source at the
centre, receivers on the centre x-line, the six faces packed and unpacked into
contiguous buffers every step (loopback exchange) -- after W untimed warm-up steps,
and prints one JSON line.

A step is one pass of the per-step path, the launches of fd_step_exchange: the y and
z face halos of u^n unpacked from the receive buffers (the loopback of the faces the
previous step packed); the stencil kernel, which reads the x face halos from their
receive buffers, applies the leapfrog update with the source term and writes the x
faces of u^{n+1} to the other face set; the y and z faces of u^{n+1} packed, with the
receiver row in the same launch; then the pointer rotation.  ``value`` is interior
points x steps / wall time in Gpts/s with every array resident in HBM.  ``roofline``
rates the stencil kernel by its algorithmic bytes (16 B per interior point: u^n,
u^{n-1} and vdt2 read once, u^{n+1} written once; plus 4 B per x-face point read and
4 B written) over its average launch time from HIP events on its own stream.
``cpu_baseline`` times the FP64 CPU oracle on a bounded sample of the same workload.

Further legs in the same line (each skippable): ``serving`` (the continuous-batching
shot server against the plain per-shot loop), ``small`` (64^3 parity configuration),
``large`` (1024 x 1024 x 512, with its own roofline and CPU baseline), ``cannon`` (one
rank's block products of Cannon's matrix multiply, N = 30240, P = 8, against the FP64
matrix peak), ``fwi`` (the 256^3 FWI gradient, with its roofline against the
gradient's algorithmic bytes).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBPS = 8000.0
METRIC = "Gpts/s + % HBM roofline; shots/s and p50/p99 latency vs plain per-shot loop"
CSRC = os.path.join(ROOT, "paper_2506_02486_amd", "csrc")
# source file of each forward kernel (the counter summary is valid for one version)
KERNEL_SRC = {"wide_128x32": "fd_stencil4.hip", "wide_64x64": "fd_stencil4.hip",
              "march_64x32": "fd_stencil.hip",
              "march_64x16": "fd_stencil.hip", "point": "fd_point.hip"}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "fd_step_512_traffic.txt")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def stencil_hash(kernel: str = "wide_128x32") -> str:
    """sha256[:16] of the kernel's source code, comments removed and whitespace runs
    collapsed: an edit of comments keeps the counter summary valid, any change of code
    voids it."""
    src = open(os.path.join(CSRC, KERNEL_SRC[kernel])).read()
    src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
    src = re.sub(r"//[^\n]*", " ", src)
    return hashlib.sha256(" ".join(src.split()).encode()).hexdigest()[:16]


def read_traffic(path: str, kernel: str):
    """HBM bytes per stencil launch from a committed counter summary, if it was taken
    on the current source of that kernel; else None."""
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m_h = re.search(r"stencil_source_sha256_16:\s*([0-9a-f]+)", txt)
    m_b = re.search(r"traffic_bytes_per_launch:\s*([0-9.eE+]+)", txt)
    if not m_h or not m_b or m_h.group(1) != stencil_hash(kernel):
        return None
    return float(m_b.group(1))


def copy_bandwidth(torch, nbytes=1 << 31, reps=10):
    """Device-to-device copy bandwidth (read + write bytes / time) of a plain copy."""
    n = nbytes // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    s = e0.elapsed_time(e1) / 1e3 / reps
    del a, b
    return 2 * nbytes / s / 1e9


def stream_bandwidth(torch, n=140_000_000, reps=20):
    """Bandwidth of torch's own elementwise kernel on the stencil's access mix: three
    arrays read and one written per element (addcmul, 16 B/element), the three
    working arrays rotating as the wavefields do (560 MB each, far above the 256 MB
    last-level cache).  A reference for what plain streaming of that mix reaches."""
    bufs = [torch.ones(n, dtype=torch.float32, device="cuda") for _ in range(3)]
    q = torch.full((n,), 0.25, dtype=torch.float32, device="cuda")

    def step(i):
        torch.addcmul(bufs[i % 3], bufs[(i + 1) % 3], q, out=bufs[(i + 2) % 3])

    for i in range(3):
        step(i)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for i in range(reps):
        step(i)
    e1.record()
    torch.cuda.synchronize()
    s = e0.elapsed_time(e1) / 1e3 / reps
    del bufs, q
    return 16.0 * n / s / 1e9


def cpu_baseline(v, dt, src, steps):
    """FP64 oracle on the same 512^3 workload: (time of 1+steps) - (time of 1 step)."""
    import numpy as np

    import oracle

    n = v.shape[0]
    q = oracle.vdt2(v, dt)
    eta = oracle.sponge_tables(n, n, n, 16, float(v.max()), (10.0,) * 3, dt)
    w = oracle.ricker(steps + 1, dt)
    def per_step_s(k):
        t0 = time.perf_counter()
        oracle.forward(None, 1, dt, src=src, w=w[:1], eta=eta, periodic=True, q=q)
        t1 = time.perf_counter()
        oracle.forward(None, k + 1, dt, src=src, w=w[:k + 1], eta=eta, periodic=True, q=q)
        t2 = time.perf_counter()
        return ((t2 - t1) - (t1 - t0)) / k

    cores = oracle.threads()
    per_step = per_step_s(steps)
    oracle.set_threads(1)
    per_step_1 = per_step_s(1)
    oracle.set_threads(cores)
    del q
    # the 64^3 parity configuration (layered model, Dirichlet, 100 steps) in full
    from workloads import center_source as _cs, layered_velocity, receivers_plane
    v64 = layered_velocity(64, 64, 64, seed=1)
    dt64 = oracle.cfl_dt(v64, 10.0)
    t0 = time.perf_counter()
    oracle.forward(v64, 100, dt64, src=_cs(64, 64, 64), w=oracle.ricker(100, dt64),
                   rec=receivers_plane(64, 64, 0))
    t64 = time.perf_counter() - t0
    return {
        "value": round(n ** 3 / per_step / 1e9, 5),
        "unit": "Gpts/s",
        "cores": cores,
        "kind": "oracle",
        "sample": f"FP64 oracle, same {n}^3 sponge-16 periodic workload, {steps} steps "
                  f"(time of {steps + 1} steps minus 1 step, set-up excluded); "
                  f"{per_step:.3f} s/step",
        "one_core_Gpts_per_s": round(n ** 3 / per_step_1 / 1e9, 5),
        "config_64cubed_100_steps_Gpts_per_s": round(64 ** 3 * 100 / t64 / 1e9, 5),
        "host_cpu": host_cpu(),
        "host_nproc": os.cpu_count(),
    }


def host_cpu() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def serving_bench(nshots=256, nt=500, lo=128, hi=384, max_slots=32, arena_gb=48.0,
                  warm=16, load=2.0, reps=3, buddy=False, cap=0):
    """Poisson stream of shots of uneven size: the batching server against the plain
    per-shot loop (same kernels, one shot at a time, arrival order), each run `reps`
    times, alternately, on the same arrivals; reported per run, as the mean, and as
    the spread (max - min) of the runs.  cap > 0: the server's admission cap on the
    points running at once (fd_server_set_admission) in place of its default policy."""
    import threading

    import numpy as np
    import torch

    from paper_2506_02486_amd import serving
    from workloads import poisson_arrivals, receivers_xline, serving_shots, smooth_velocity

    log(f"serving: generating the {hi}^3 shared model")
    vm = smooth_velocity(hi, hi, hi, seed=2)
    vd = torch.from_numpy(vm).cuda()
    vmax = float(vm.max())
    dt = 0.4 * 10.0 / vmax
    specs = serving_shots(nshots, seed=3, lo=lo, hi=hi)

    def shot(s):
        nx, ny, nz = s["nx"], s["ny"], s["nz"]
        return serving.Shot(vd[:nz, :ny, :nx], nt, dt, s["src"], receivers_xline(nx, ny // 2, 4),
                            sponge_width=16, sponge_vmax=vmax)

    shots = [shot(s) for s in specs]
    plain = serving.PlainLoop((hi, hi, hi))
    # plain-loop service rate from warm-up shots (drawn after the stream's shots)
    warm_specs = serving_shots(nshots + warm, seed=3, lo=lo, hi=hi)[nshots:]
    t0 = time.perf_counter()
    for s in warm_specs:
        plain.run(shot(s))
    mu = warm / (time.perf_counter() - t0)
    lam = load * mu
    arr = poisson_arrivals(nshots, lam, seed=4)
    pts = float(sum(np.prod(s.shape) for s in shots)) * nt
    log(f"serving: plain service rate {mu:.2f} shots/s, arrivals at {lam:.2f} shots/s")
    pct = lambda x, q: float(np.percentile(np.array(x), q))  # noqa: E731
    plain_tr = {}

    def run_plain():
        lat = []
        base = time.monotonic()
        for i, s in enumerate(shots):
            wait = base + arr[i] - time.monotonic()
            if wait > 0:
                time.sleep(wait)
            tr = plain.run(s)
            lat.append(time.monotonic() - (base + arr[i]))
            if i < 8:
                plain_tr[i] = tr
        span = time.monotonic() - base
        return {"shots_per_s": nshots / span, "p50_s": pct(lat, 50), "p99_s": pct(lat, 99),
                "lat": lat}

    def run_server(allocator):
        srv = serving.ShotServer(int(arena_gb * (1 << 30)), max_slots=max_slots,
                                 allocator=allocator, max_active_points=cap)
        ids = [None] * nshots
        t_arr = [0] * nshots

        def submitter():
            b = time.monotonic()
            for i, s in enumerate(shots):
                wait = b + arr[i] - time.monotonic()
                if wait > 0:
                    time.sleep(wait)
                t_arr[i] = time.monotonic_ns()
                ids[i] = srv.submit(s)

        th = threading.Thread(target=submitter)
        th.start()
        res = [None] * nshots
        pending = set(range(nshots))
        while pending:
            for i in list(pending):
                if ids[i] is None:
                    continue
                r = srv.poll(ids[i])
                if r is not None:
                    res[i] = r
                    pending.discard(i)
            time.sleep(2e-4)
        th.join()
        steps = srv.stats()["steps"]
        srv.close()
        lat = [(r[2][2] - t_arr[i]) / 1e9 for i, r in enumerate(res)]
        span = (max(r[2][2] for r in res) - min(t_arr)) / 1e9
        return {"shots_per_s": nshots / span, "p50_s": pct(lat, 50), "p99_s": pct(lat, 99),
                "lat": lat, "batched_steps": steps, "all_ok": all(r[0] == 0 for r in res),
                "traces_bitwise_equal_first8": all(np.array_equal(res[i][1], plain_tr[i])
                                                   for i in plain_tr)}

    def summary(runs):
        out = {}
        for k in ("shots_per_s", "p50_s", "p99_s"):
            x = [r[k] for r in runs]
            out[k] = round(float(np.mean(x)), 4)
            out[k + "_runs"] = [round(v, 4) for v in x]
            out[k + "_spread"] = round(float(max(x) - min(x)), 4)
        out["Gpts_per_s"] = round(pts * out["shots_per_s"] / nshots / 1e9, 2)
        return out

    runs_p, runs_s = [], []
    for rep in range(reps):
        log(f"serving: plain loop (run {rep + 1} of {reps})")
        runs_p.append(run_plain())
        log(f"serving: batching server (run {rep + 1} of {reps})")
        runs_s.append(run_server("first_fit"))
    del plain
    torch.cuda.empty_cache()
    p, srv = summary(runs_p), summary(runs_s)
    srv["batched_steps"] = runs_s[-1]["batched_steps"]
    srv["all_ok"] = all(r["all_ok"] for r in runs_s)
    srv["traces_bitwise_equal_first8"] = all(r["traces_bitwise_equal_first8"] for r in runs_s)
    srv["speedup_shots_per_s"] = round(srv["shots_per_s"] / p["shots_per_s"], 4)
    # the server's gain over the plain loop against the larger run-to-run spread
    srv["gain_shots_per_s"] = round(srv["shots_per_s"] - p["shots_per_s"], 4)
    srv["spread_shots_per_s"] = max(p["shots_per_s_spread"], srv["shots_per_s_spread"])
    # per shot, server latency minus plain-loop latency on the same arrivals (paired
    # over the runs): robust where the latency distribution is sparse at its median
    diff = [b - a for rp, rs in zip(runs_p, runs_s) for a, b in zip(rp["lat"], rs["lat"])]
    srv["paired_latency_diff_median_s"] = round(float(np.median(diff)), 5)
    srv["paired_latency_diff_mean_s"] = round(float(np.mean(diff)), 5)
    out = {
        "workload": f"{nshots} shots, grids uniform in [{lo},{hi}]^3 (seed 3), {nt} steps, "
                    f"sponge 16, Ricker 15 Hz, x-line receivers, Poisson arrivals at "
                    f"{load:g}x the plain loop's service rate (seed 4); {reps} runs of each, "
                    f"alternating",
        "arrival_rate": round(lam, 3),
        "plain_loop": p,
        "server": srv,
        "max_slots": max_slots,
        "arena_GB": arena_gb,
        "admission": f"cap {cap} points" if cap else "default policy",
    }
    if buddy:  # the same with the buddy arena, one run
        log("serving: batching server (buddy arena)")
        b = run_server("buddy")
        out["server_buddy"] = {"shots_per_s": round(b["shots_per_s"], 3),
                               "p50_s": round(b["p50_s"], 4), "p99_s": round(b["p99_s"], 4),
                               "all_ok": b["all_ok"],
                               "traces_bitwise_equal_first8": b["traces_bitwise_equal_first8"]}
    return out


def small_bench(steps=100, repeats=5):
    """64^3 plain forward: layered model (seed 1), Dirichlet halo, no sponge, Ricker at
    the centre, 4096 receivers on the k = 0 plane, run by the library's native step
    loop.  The arrays (1.2 MB each) stay in cache, so the rate is bound by latency
    and its HBM fraction means nothing; reported as the median of `repeats` runs."""
    import numpy as np
    import torch

    from paper_2506_02486_amd import api
    from workloads import center_source, layered_velocity, receivers_plane

    n = 64
    v = layered_velocity(n, n, n, seed=1)
    geom = api.Geometry(src=center_source(n, n, n), rec=receivers_plane(n, n, 0))
    times = []
    for r in range(repeats + 1):
        sim = api.Simulation(v, geom=geom)
        tr = torch.zeros((steps, sim.nrec), dtype=torch.float32, device="cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.run(steps, tr, mode="native")
        torch.cuda.synchronize()
        if r:  # the first run warms the code paths
            times.append(time.perf_counter() - t0)
        del sim, tr
    el = float(np.median(times))
    # the same run recorded once as a HIP graph (fd_forward_graph) and launched again
    # and again: each launch starts from zero and writes the same traces
    sim = api.Simulation(v, geom=geom)
    tr = torch.zeros((steps, sim.nrec), dtype=torch.float32, device="cuda")
    G = api.ForwardGraph(sim.grid, sim.u_prev, sim.u, sim.u_next, sim.vdt2, sim.sponge, steps,
                         src=geom.src, wavelet=api.ricker(steps, sim.dt), rec_off=sim.rec_off,
                         traces=tr, rec_plane=sim.rec_plane)
    gtimes = []
    for r in range(repeats + 1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        G.launch()
        torch.cuda.synchronize()
        if r:
            gtimes.append(time.perf_counter() - t0)
    G.close()
    gel = float(np.median(gtimes))
    return {"workload": "64^3 layered model, Dirichlet, no sponge, 4096 receivers at k=0, "
                        f"{steps} steps (in cache, latency-bound; HBM fraction not meaningful)",
            "steps": steps, "repeats": repeats,
            "Gpts_per_s": round(n ** 3 * steps / el / 1e9, 2),
            "us_per_step": round(el * 1e6 / steps, 2),
            "graph_Gpts_per_s": round(n ** 3 * steps / gel / 1e9, 2),
            "graph_us_per_step": round(gel * 1e6 / steps, 2)}


def small_exchange_bench(n=64, steps=200, repeats=5):
    """A small subdomain's exchange step: n^3 smooth model (seed 2), sponge 8, Ricker at
    the centre, receivers on the centre x-line, the six faces exchanged (loopback) every
    step, run by the library's native loop with two face sets (on a grid this small the
    whole step is one launch of the one-thread-per-point kernel); median of `repeats`."""
    import numpy as np
    import torch

    from paper_2506_02486_amd import api
    from workloads import center_source, receivers_xline, smooth_velocity

    v = smooth_velocity(n, n, n, seed=2, sigma=4.0)
    geom = api.Geometry(src=center_source(n, n, n), rec=receivers_xline(n, n // 2, n // 2))
    times = []
    for r in range(repeats + 1):
        sim = api.Simulation(v, sponge_width=8, exchange="loopback", geom=geom)
        tr = torch.zeros((steps, sim.nrec), dtype=torch.float32, device="cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.run(steps, tr, mode="native")
        torch.cuda.synchronize()
        if r:
            times.append(time.perf_counter() - t0)
        del sim, tr
    el = float(np.median(times))
    return {"workload": f"{n}^3 smooth model, sponge 8, six faces exchanged (loopback) every "
                        f"step, {n}-point x-line receivers, {steps} steps (in cache, latency-bound)",
            "steps": steps, "repeats": repeats,
            "Gpts_per_s": round(n ** 3 * steps / el / 1e9, 2),
            "us_per_step": round(el * 1e6 / steps, 2)}


def large_bench(steps=500, warmup=5, every=8, cpu=True, cpu_steps=10, vcache=None):
    """1024 x 1024 x 512 subdomain (the large single-GPU configuration), smooth model
    (seed 2), sponge 16, Dirichlet halo, Ricker at the centre, receivers on the
    1024-point line y = 512, z = 4: the per-step path without the exchange (the fused
    update with the source, then the receiver row), `steps` steps after `warmup`.
    The stencil is bracketed with HIP events on every `every`-th step for its roofline
    line; `cpu` also times the FP64 oracle on `cpu_steps` steps of the same grid."""
    import numpy as np
    import torch

    from paper_2506_02486_amd import api
    from workloads import center_source, receivers_xline, smooth_velocity

    nx, ny, nz = 1024, 1024, 512
    if vcache and os.path.exists(vcache):
        v = np.load(vcache)
    else:
        log("large: generating the 1024x1024x512 model")
        v = smooth_velocity(nx, ny, nz, seed=2)
        if vcache:
            np.save(vcache, v)
    src = center_source(nx, ny, nz)
    rec = receivers_xline(nx, 512, 4)
    sim = api.Simulation(v, sponge_width=16, geom=api.Geometry(src=src, rec=rec))
    sim.run(warmup)
    g = sim.grid
    kern = api.step_kernel(g, faces=False)
    w = api.ricker(steps, sim.dt, n0=sim.n)
    tr = torch.zeros((steps, sim.nrec), dtype=torch.float32, device="cuda")
    ev = {s: (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for s in range(0, steps, max(1, every))}
    log(f"large: timing {steps} steps ({kern['kernel']} kernel)")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(steps):
        if s in ev:
            ev[s][0].record()
        api.step_fused(g, sim.u_prev, sim.u, sim.u_next, sim.vdt2, sim.sponge,
                       (src, float(w[s])), None)
        if s in ev:
            ev[s][1].record()
        api.record_receivers(g, sim.u_next, sim.rec_off, tr[s])
        sim.u_prev, sim.u, sim.u_next = sim.u, sim.u_next, sim.u_prev
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    k_ms = float(np.mean([a.elapsed_time(b) for a, b in ev.values()]))
    pts = nx * ny * nz
    algo = 16.0 * pts  # u^n, u^{n-1}, vdt2 read once, u^{n+1} written once
    achieved = algo / (k_ms / 1e3) / 1e9
    finite = bool(torch.isfinite(g.interior(sim.u)).all().item())
    dt = sim.dt
    del sim, tr
    torch.cuda.empty_cache()
    traffic = read_traffic(os.path.join(ROOT, "profiles", "fd_step_large_traffic.txt"),
                           kern["kernel"])
    out = {"workload": "1024x1024x512 + radius-4 halo, smooth model (seed 2), sponge 16, "
                       "Dirichlet halo, Ricker 15 Hz at the centre, 1024 receivers at y=512, z=4",
           "steps": steps, "warmup": warmup,
           "value": round(pts * steps / el / 1e9, 3), "unit": "Gpts/s",
           "ms_per_step": round(el * 1e3 / steps, 4), "finite": finite,
           "roofline": {"bound": "hbm",
                        "kernel": f"{kern['kernel']} forward update with the source term "
                                  f"({kern['tile'][0]} x {kern['tile'][1]} tiles, "
                                  f"{kern['kchunk']} planes per block, {kern['blocks']} blocks)",
                        "achieved": round(achieved, 1), "peak": PEAK_HBM_GBPS, "unit": "GB/s",
                        "frac": round(achieved / PEAK_HBM_GBPS, 4),
                        "traffic": (round(traffic) if traffic is not None else None),
                        "algorithmic_bytes_per_launch": algo,
                        "avg_launch_ms": round(k_ms, 5)}}
    if cpu:
        log(f"large: CPU oracle baseline ({cpu_steps} steps after 1)")
        out["cpu_baseline"] = cpu_baseline_dirichlet(v, dt, src, cpu_steps)
    del v
    return out


def cpu_baseline_dirichlet(v, dt, src, steps):
    """FP64 oracle on a Dirichlet, sponge-16 grid: (time of 1+steps) - (time of 1)."""
    import oracle

    nz, ny, nx = v.shape
    q = oracle.vdt2(v, dt)
    eta = oracle.sponge_tables(nx, ny, nz, 16, float(v.max()), (10.0,) * 3, dt)
    w = oracle.ricker(steps + 1, dt)
    t0 = time.perf_counter()
    oracle.forward(None, 1, dt, src=src, w=w[:1], eta=eta, q=q)
    t1 = time.perf_counter()
    oracle.forward(None, steps + 1, dt, src=src, w=w, eta=eta, q=q)
    t2 = time.perf_counter()
    per_step = ((t2 - t1) - (t1 - t0)) / steps
    del q
    pts = nx * ny * nz
    return {"value": round(pts / per_step / 1e9, 5), "unit": "Gpts/s",
            "cores": oracle.threads(), "kind": "oracle",
            "sample": f"FP64 oracle, the same {nx}x{ny}x{nz} sponge-16 Dirichlet grid and "
                      f"source, {steps} steps (time of {steps + 1} steps minus 1 step, set-up "
                      f"excluded); {per_step:.3f} s/step",
            "host_cpu": host_cpu(), "host_nproc": os.cpu_count()}


def fwi_bench(n=256, nt=1000, every=32):
    """FWI gradient w.r.t. squared slowness: n^3, nt steps, checkpoints every `every`
    steps (0: every state kept), sponge 16, source (n/2, n/2, 20), receivers on the
    plane z = 20, observed data from a +5% Gaussian blob at the centre.  Roofline: the
    algorithmic bytes of one gradient -- per point and step 16 B forward, 16 B
    recomputed forward (none when every state is kept) and 28 B for the adjoint step
    with the gradient fused (a^{n+1}, vdt2, a^{n+2}, u^n, g read, a^n and g written)
    -- over the time of one gradient against 8 TB/s."""
    import numpy as np
    import torch

    from paper_2506_02486_amd import fwi
    from workloads import blob_perturbed, receivers_plane, smooth_velocity

    log(f"fwi: {n}^3, {nt} steps, checkpoints every {every}")
    v0 = smooth_velocity(n, n, n, seed=2)
    vt = blob_perturbed(v0)
    dt = 0.4 * 10.0 / float(v0.max())
    prob = fwi.FWIProblem((n, n, n), dt, (n // 2, n // 2, 20), receivers_plane(n, n, 20), nt,
                          sponge_width=16, sponge_vmax=float(v0.max()), checkpoint_every=every)
    m0 = torch.from_numpy((1.0 / v0.astype(np.float64) ** 2).astype(np.float32)).cuda()
    mt = torch.from_numpy((1.0 / vt.astype(np.float64) ** 2).astype(np.float32)).cuda()
    obs = prob.forward(mt, checkpoints=False)
    fwi.misfit_gradient(prob, m0, obs)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    J, g = fwi.misfit_gradient(prob, m0, obs)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    pts = n ** 3
    algo = (16.0 + (16.0 if every else 0.0) + 28.0) * pts * nt
    what = f"checkpoints every {every}" if every else "every state kept in HBM"
    achieved = algo / el / 1e9
    out = {"workload": f"FWI gradient {n}^3, {nt} steps, {what}, sponge 16, source "
                       f"({n // 2},{n // 2},20), receivers on the plane z=20, observed data "
                       f"from a +5% Gaussian blob",
           "value": round(el, 4), "unit": "s per gradient", "misfit": J,
           "roofline": {"bound": "hbm", "kernel": "whole gradient (forward, recompute, "
                                                  "adjoint and gradient kernels)",
                        "achieved": round(achieved, 1), "peak": PEAK_HBM_GBPS, "unit": "GB/s",
                        "frac": round(achieved / PEAK_HBM_GBPS, 4), "traffic": None,
                        "algorithmic_bytes": algo,
                        "roofline_seconds": round(algo / (PEAK_HBM_GBPS * 1e9), 4)},
           "finite": bool(torch.isfinite(g).all().item())}
    del prob, g, m0, mt, obs
    torch.cuda.empty_cache()
    return out


PEAK_FP64_MFMA_TFLOPS = 78.6


def cannon_bench(N=30240, P=8, reps=3, cpu=True, cpu_cols=32):
    """Cannon's matrix multiply (Sec. 4.4), the local work of one rank: N = 30240,
    P = 8 ranks (Ns = 3780), rank 0's P block products C_0 += A_0[:, q-block] @ B_q
    (3780 x 30240 x 3780 each, FP64 on the matrix cores) with every B stripe resident
    (the ring shift between ranks needs other GPUs).  Seeded normal operands made on
    the device.  ``value`` is TFLOP/s over `reps` timed rank passes after one warm-up;
    the roofline rates the block-product kernel against the FP64 matrix peak; the CPU
    baseline times the FP64 oracle on `cpu_cols` columns of C_0 over all P steps."""
    import numpy as np
    import torch

    from paper_2506_02486_amd import api

    ns = N // P
    log(f"cannon: N={N}, P={P}, rank 0's {P} products of {ns} x {N} x {ns}")
    g = torch.Generator(device="cuda")
    g.manual_seed(11)
    A0 = torch.randn((ns, N), generator=g, device="cuda", dtype=torch.float64)
    B = torch.randn((N, N), generator=g, device="cuda", dtype=torch.float64)
    C0 = torch.zeros((ns, N), device="cuda", dtype=torch.float64)
    stream = torch.cuda.current_stream()
    api.cannon_rank(A0, B, C0, 0, P, stream)  # warm-up
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        api.cannon_rank(A0, B, C0, 0, P, stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_launch = e0.elapsed_time(e1) / (reps * P)
    flops_launch = 2.0 * ns * N * ns
    tflops = flops_launch / ms_launch / 1e9
    finite = bool(torch.isfinite(C0).all().item())
    out = {"workload": f"Cannon's matrix multiply, N={N}, P={P}: one rank's {P} local block "
                       f"products C_r += A_r[:, q-block] @ B_q ({ns} x {N} x {ns}, FP64), "
                       f"all B stripes resident, seeded normal operands",
           "value": round(tflops, 2), "unit": "TFLOP/s", "dtype": "f64",
           "ms_per_rank_pass": round(ms_launch * P, 3),
           "roofline": {"bound": "mfma", "kernel": "gemm_f64_kernel (256 x 128 tiles, 16 waves, "
                                                   "v_mfma_f64_16x16x4f64)",
                        "achieved": round(tflops, 2), "peak": PEAK_FP64_MFMA_TFLOPS,
                        "unit": "TFLOP/s", "frac": round(tflops / PEAK_FP64_MFMA_TFLOPS, 4),
                        "traffic": None, "algorithmic_flops_per_launch": flops_launch,
                        "avg_launch_ms": round(ms_launch, 4)},
           "finite": finite}
    if cpu:
        import oracle
        log(f"cannon: CPU oracle on {cpu_cols} columns of C_0")
        cols = np.linspace(0, N - 1, cpu_cols).astype(np.int64)
        a_h = A0.cpu().numpy()
        bcols = np.ascontiguousarray(B[:, torch.from_numpy(cols).cuda()].cpu().numpy())
        t0 = time.perf_counter()
        got = np.zeros((ns, cpu_cols))
        for q in api.cannon_order(0, P):
            oracle.block_gemm(a_h[:, q * ns:(q + 1) * ns], bcols[q * ns:(q + 1) * ns], got,
                              accumulate=True)
        el = time.perf_counter() - t0
        ref = C0[:, torch.from_numpy(cols).cuda()].cpu().numpy() / (reps + 1)
        out["cpu_baseline"] = {
            "value": round(2.0 * ns * N * cpu_cols / el / 1e12, 6), "unit": "TFLOP/s",
            "cores": oracle.threads(), "kind": "oracle",
            "sample": f"FP64 oracle (plain loops), {cpu_cols} columns of C_0 over the {P} "
                      f"steps ({2.0 * ns * N * cpu_cols / 1e9:.2f} GFLOP) in {el:.2f} s"}
        # the GPU ran the rank pass reps + 1 times into C_0: compare the mean
        out["sampled_columns_rel_err"] = float(np.linalg.norm(ref - got) / np.linalg.norm(got))
    del A0, B, C0
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--n", type=int, default=512, help="interior edge (default 512)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=20)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="after the timed region, run a plain 1 GiB device copy (for counters)")
    ap.add_argument("--kchunk", type=int, default=0)
    ap.add_argument("--event-every", type=int, default=8,
                    help="bracket the stencil with HIP events on every N-th timed step")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-large", action="store_true", help="skip the 1024x1024x512 leg")
    ap.add_argument("--large-steps", type=int, default=500)
    ap.add_argument("--vcache-large", default=None,
                    help="optional .npy path to cache the 1024x1024x512 velocity model")
    ap.add_argument("--no-fwi", action="store_true", help="skip the 256^3 FWI gradient legs")
    ap.add_argument("--no-small", action="store_true", help="skip the 64^3 small-grid leg")
    ap.add_argument("--no-cannon", action="store_true",
                    help="skip the Cannon block-product leg (N=30240, P=8)")
    ap.add_argument("--shots", type=int, default=256, help="shots in the serving stream")
    ap.add_argument("--serving-cap", type=int, default=0,
                    help="with --only serving: the server's cap on running points (0: its "
                         "default admission policy)")
    ap.add_argument("--only", choices=["cannon", "fwi", "large", "serving"], default=None,
                    help="run only this leg (no 512^3 step) and print its JSON object; for "
                         "profiling a leg by itself")
    ap.add_argument("--vcache", default=None,
                    help="optional .npy path to cache the generated velocity model")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: this library runs on one GPU only (asked for --gpus {args.gpus}); "
              "multi-GPU sharding of the subdomain is not built.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2506_02486_amd import api
    from workloads import center_source, receivers_xline, smooth_velocity

    assert torch.cuda.is_available(), "bench.py needs a ROCm device"
    torch.cuda.set_device(0)
    if args.only:
        cpu = not args.no_cpu_baseline
        if args.only == "cannon":
            leg = cannon_bench(cpu=cpu)
        elif args.only == "fwi":
            leg = fwi_bench()
        elif args.only == "large":
            leg = large_bench(steps=args.large_steps, cpu=cpu, vcache=args.vcache_large)
        else:  # the three serving legs of the full run
            leg = {"serving": serving_bench(nshots=args.shots, buddy=True, cap=args.serving_cap),
                   "serving_latency": serving_bench(nshots=max(16, args.shots // 2), load=0.5),
                   "serving_small": serving_bench(nshots=args.shots, lo=48, hi=128)}
        print(json.dumps(leg), flush=True)
        return
    n = args.n
    log(f"bench: generating {n}^3 smooth velocity model")
    if args.vcache and os.path.exists(args.vcache):
        v = np.load(args.vcache)
    else:
        v = smooth_velocity(n, n, n, seed=2)
        if args.vcache:
            np.save(args.vcache, v)
    src = center_source(n, n, n)
    rec = receivers_xline(n, n // 2, n // 2)
    sim = api.Simulation(v, sponge_width=16, exchange="loopback",
                         geom=api.Geometry(src=src, rec=rec))
    if args.kchunk:
        api.set_kchunk(args.kchunk)
    g = sim.grid
    kern = api.step_kernel(g, faces=True)
    K, W = args.steps, args.warmup
    log(f"bench: dt={sim.dt:.6e} s, vmax={sim.vmax:.1f}; {kern['kernel']} kernel; "
        f"warm-up {W} steps")
    sim.run(W)
    torch.cuda.synchronize()

    w = api.ricker(K, sim.dt, n0=sim.n)
    traces = torch.zeros((K, sim.nrec), dtype=torch.float32, device="cuda")
    # HIP events bracket the stencil kernel on every `every`-th step of the timed
    # loop: each timing event recorded between two kernels leaves the device idle
    # for a few microseconds, so bracketing every step would slow the loop it times
    every = max(1, args.event_every)
    ev = {s: (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for s in range(0, K, every)}
    log(f"bench: timing {K} steps")
    assert sim._faces_current  # the warm-up left the faces of u^n in the send buffers
    torch.cuda.synchronize()
    # face sets: `cur` holds the faces of u^n (its loopback is this step's receive
    # side), `nxt` receives the faces of u^{n+1}.  fd_step_exchange of the full
    # sets runs unpack(y, z faces), the stencil (x faces inside), pack(y, z faces);
    # the same kernels are issued here through the split calls (the pack launch
    # also takes the receiver row) so that the events bracket the stencil alone.
    cur, nxt = sim.send, sim.send2

    def split(F):
        lb = api.loopback(F)
        return ([None, None] + lb[2:], lb[:2] + [None] * 4, [None, None] + list(F[2:]),
                list(F[:2]) + [None] * 4)

    parts = {id(cur): split(cur), id(nxt): split(nxt)}
    t0 = time.perf_counter()
    for s in range(K):
        in_yz, in_x = parts[id(cur)][:2]
        out_yz, out_x = parts[id(nxt)][2:]
        api.halo_unpack(g, sim.u, in_yz)
        if s in ev:
            ev[s][0].record()
        api.step_exchange(g, sim.u_prev, sim.u, sim.u_next, sim.vdt2, sim.sponge,
                          (src, float(w[s])), in_x, out_x)
        if s in ev:
            ev[s][1].record()
        api.halo_pack_record(g, sim.u_next, out_yz, sim.rec_off, traces[s])
        sim.u_prev, sim.u, sim.u_next = sim.u, sim.u_next, sim.u_prev
        cur, nxt = nxt, cur
        sim.n += 1
    sim.send, sim.send2 = cur, nxt
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    kern_ms = [a.elapsed_time(b) for a, b in ev.values()]
    avg_ms = float(np.mean(kern_ms))
    pts = n ** 3
    gpts = pts * K / elapsed / 1e9
    face_pts = 6 * 4 * n * n
    # the stencil kernel reads u^n, u^{n-1}, vdt2 and the two received x faces once
    # and writes u^{n+1} and the two sent x faces once
    algo_bytes = 16.0 * pts + 8.0 * (2 * 4 * n * n)
    achieved = algo_bytes / (avg_ms / 1e3) / 1e9
    path_bytes = 16.0 * pts + 8.0 * face_pts
    finite = bool(torch.isfinite(g.interior(sim.u)).all().item())
    log(f"bench: {elapsed * 1e3 / K:.3f} ms/step, fd_step {avg_ms * 1e3:.1f} us avg, "
        f"{gpts:.1f} Gpts/s, finite={finite}")

    copy_gbps = copy_bandwidth(torch)
    stream_gbps = stream_bandwidth(torch)
    if args.copy_calibration:
        # a plain copy of exactly 1 GiB read + 1 GiB written, for the counter factor
        a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    traffic = read_traffic(TRAFFIC_FILE, kern["kernel"])
    out = {
        "metric": METRIC,
        "value": round(gpts, 3),
        "unit": "Gpts/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": round(elapsed * 1e3 / K, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"single-subdomain step: {n}^3 interior + radius-4 halo, smooth random "
                        f"velocity 1500-4500 m/s (seed 2, Gaussian sigma 8), 16-cell quadratic "
                        f"sponge, Ricker 15 Hz at the centre, receivers on the centre x-line, "
                        f"six faces packed/unpacked each step (loopback)",
            "grid": [n, n, n],
            "halo": 4,
            "stencil": "25-point star, 8th order space, 2nd order time",
            "steps_timed": K,
        },
        "roofline": {
            "bound": "hbm",
            "kernel": f"stencil of fd_step_exchange: {kern['kernel']} kernel "
                      f"({kern['tile'][0]} x {kern['tile'][1]} tiles, {kern['kchunk']} planes "
                      f"per block, {kern['blocks']} blocks; update + source, x faces received "
                      f"and sent in the same kernel)",
            "achieved": round(achieved, 1),
            "peak": PEAK_HBM_GBPS,
            "unit": "GB/s",
            "frac": round(achieved / PEAK_HBM_GBPS, 4),
            "traffic": (round(traffic) if traffic is not None else None),
            "algorithmic_bytes_per_launch": algo_bytes,
            "avg_launch_ms": round(avg_ms, 5),
        },
        "path": {
            "algorithmic_bytes_per_step": path_bytes,
            "achieved_GBps": round(path_bytes / (elapsed / K) / 1e9, 1),
            "frac": round(path_bytes / (elapsed / K) / 1e9 / PEAK_HBM_GBPS, 4),
        },
        "copy_GBps": round(copy_gbps, 1),
        # torch addcmul over rotating 560 MB arrays: 3 reads + 1 write, the stencil's mix
        "stream_3r1w_GBps": round(stream_gbps, 1),
        "stencil_vs_stream_3r1w": round(achieved / stream_gbps, 3),
        "gpu": torch.cuda.get_device_name(0),
        "hip": torch.version.hip,
        "finite": finite,
        "_dt": sim.dt,
    }
    del sim, traces
    torch.cuda.empty_cache()
    if not args.no_serving:
        out["serving"] = serving_bench(nshots=args.shots, buddy=True)  # arrivals at 2x
        # latency: arrivals at half the plain loop's service rate, half as many shots
        out["serving_latency"] = serving_bench(nshots=max(16, args.shots // 2), load=0.5)
        # small shots, which leave the device part idle when run one at a time
        out["serving_small"] = serving_bench(nshots=args.shots, lo=48, hi=128)
    if not args.no_small:
        out["small"] = small_bench()
        out["small_exchange"] = small_exchange_bench()
    if not args.no_large:
        out["large"] = large_bench(steps=args.large_steps, cpu=not args.no_cpu_baseline,
                                   vcache=args.vcache_large)
    if not args.no_cannon:
        out["cannon"] = cannon_bench(cpu=not args.no_cpu_baseline)
    if not args.no_fwi:
        out["fwi"] = fwi_bench()
        # the same gradient keeping all 1000 states in HBM (89 GB): no recompute
        out["fwi_all_states"] = fwi_bench(every=0)
    if not args.no_cpu_baseline:
        log(f"bench: CPU oracle baseline ({args.cpu_steps} steps of {n}^3)")
        out["cpu_baseline"] = cpu_baseline(v, out["_dt"], src, args.cpu_steps)
    else:
        out["cpu_baseline"] = None
    out.pop("_dt", None)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
