// fd_server.cpp -- continuous-batching server for independent forward shots.
//
// One progress thread per server owns the device work:
//   admit   : strict FIFO; the head shot enters when a slot is free and a
//             first-fit search of the arena finds its footprint.  Admission
//             zeroes its wavefields, reduces max(v) (checking stability),
//             builds vdt2 from the caller's velocity view and uploads sponge
//             tables and receiver offsets, all on the server's own admission
//             stream (its host waits never drain the steps queued on the
//             compute stream), then writes the shot's entry of the slot table.
//   step    : one batched stencil launch over the tile table of all active
//             shots (each at its own step n, its source amplitude w[n] passed
//             by value), which also writes the trace rows of shots whose
//             receivers lie on one z plane; then one batched receiver launch
//             for the other shots with receivers.
//   retire  : a shot that reached nt has its traces copied to pinned host
//             memory on the copy stream; when that copy has landed the shot
//             is done and its arena block is released.
// At most kInflight steps are queued ahead of the device.  The arena, the
// streams and all device memory are the caller's; the server only carves.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "fd_arena.h"
#include "fd_internal.h"

namespace fd {
namespace {

constexpr size_t kAlign = 256;
// The progress thread runs at most kEventEvery * kInflight batched steps ahead of
// the device.  It records a throttle event once per kEventEvery steps, not every
// step: each default event between two launches left the device idle ~5.5 us
// (kernel trace of lone 192^3 shots: 27 us steps)
constexpr int kInflight = 2;
constexpr int kEventEvery = 4;
constexpr int kTileCap = 1 << 16;   // tile-table entries
// z planes per tile-table entry counted against kTileCap at admission.  The table
// itself uses the z chunk the stencil's launch model picks for the active shots
// together (a lone 128^3 shot: 2 planes, 512 blocks; 32 shots of the 128..384^3
// mix: tens of planes), within kTileCap entries.
constexpr int kServeKchunk = 24;
constexpr double kSpongeR = 1e-3;

size_t align_up(size_t n) { return (n + kAlign - 1) / kAlign * kAlign; }

int64_t now_ns() {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

// Layout of one shot's arena block.
struct ShotLayout {
  fd_grid g;
  int64_t elems;
  size_t vol, sponge, rec, traces, rmap, total;  // byte offsets and total
  int tiles;
};

double symbol_at_nyquist() {
  // -c0 - 2 sum_m c_m cos(m pi) of the 8th-order second difference
  const double c[5] = {-205.0 / 72.0, 8.0 / 5.0, -1.0 / 5.0, 8.0 / 315.0, -1.0 / 560.0};
  double s = -c[0];
  for (int m = 1; m <= 4; ++m) s -= 2.0 * c[m] * ((m & 1) ? -1.0 : 1.0);
  return s;
}

int layout_for(const fd_shot_desc* d, ShotLayout* L) {
  if (!d) return fail(FD_EINVAL, "shot: descriptor is NULL");
  if (fd_grid_init(&L->g, d->nx, d->ny, d->nz, d->dx, d->dy, d->dz) != FD_OK) return FD_EINVAL;
  if (d->nt < 1) return fail(FD_EINVAL, "shot: nt must be >= 1");
  if (d->nrec < 0) return fail(FD_EINVAL, "shot: nrec < 0");
  L->elems = fd_grid_elems(&L->g);
  const size_t vbytes = align_up((size_t)L->elems * 4);
  L->vol = 0;
  L->sponge = 4 * vbytes;
  L->rec = L->sponge + align_up(4 * (size_t)(d->nx + d->ny + d->nz));
  L->traces = L->rec + align_up(8 * (size_t)std::max(d->nrec, 1));
  L->rmap = L->traces + align_up(4 * (size_t)d->nt * (size_t)std::max(d->nrec, 1));
  // receiver plane map (receivers on one z plane), nx * ny int32
  L->total = L->rmap + (d->nrec > 0 ? align_up(4 * (size_t)d->nx * (size_t)d->ny) : 0);
  int tx, ty;
  batch_tile_shape(&tx, &ty);
  const long long t = (long long)((d->nx + tx - 1) / tx) * ((d->ny + ty - 1) / ty) *
                      ((d->nz + kServeKchunk - 1) / kServeKchunk);
  L->tiles = (int)std::min<long long>(t, 1LL << 30);
  return FD_OK;
}

struct Shot {
  int64_t id = 0;
  fd_shot_desc d{};
  std::vector<int32_t> rec;
  ShotLayout L{};
  int status = FD_EAGAIN;     // final code once finished
  bool finished = false;
  int64_t t_submit = 0, t_admit = 0, t_done = 0;
  int slot = -1;
  size_t off = 0;             // arena block
  bool has_block = false;
  int n = 0;                  // steps done
  std::vector<float> w;       // source wavelet
  float* host = nullptr;      // pinned traces
  size_t host_cap = 0;        // floats
  hipEvent_t copied = nullptr;
};

struct Server {
  char* base = nullptr;
  size_t bytes = 0;
  int max_slots = 0;
  int device = 0;
  hipStream_t cs = nullptr, xs = nullptr;
  hipStream_t as = nullptr;  // admission work (always the server's own)
  bool own_cs = false, own_xs = false;
  std::unique_ptr<Arena> arena;
  // device tables (head of the arena), the host master slot table and two
  // pinned staging sets used in turn, so that rebuilding the tables never waits
  // for the copy of the previous upload
  BatchShot* d_shots = nullptr;
  int4* d_tiles = nullptr;
  int* d_slots = nullptr;
  int32_t* d_scratch = nullptr;
  std::vector<BatchShot> shots_host;
  BatchShot* h_shots[2] = {};
  int4* h_tiles[2] = {};
  int* h_slots[2] = {};
  hipEvent_t table_ev[2] = {};
  int stage = 0;
  int32_t* h_scratch = nullptr;
  float* h_stage = nullptr;   // sponge and receiver upload staging
  size_t h_stage_cap = 0;
  hipEvent_t step_ev[kInflight] = {};
  int ntiles = 0, nactive = 0, max_nrec = 0;
  bool table_dirty = false;
  // shared state
  std::mutex mu;
  std::condition_variable cv;
  std::deque<Shot*> queue;
  std::map<int64_t, std::unique_ptr<Shot>> shots;
  std::vector<Shot*> slots;
  std::vector<Shot*> draining;
  std::vector<std::pair<size_t, float*>> pinned_pool;
  int64_t next_id = 1;
  int64_t steps = 0;
  int64_t max_points = 0;  // admission waits while the slots hold this many points
  int queued = 0, running = 0, finished = 0;
  bool stopping = false, stopped = false;
  std::thread th;
};

// ---- pinned trace buffers (reused: hipHostFree can stall the device)
float* take_pinned(Server* S, size_t floats) {
  for (size_t i = 0; i < S->pinned_pool.size(); ++i)
    if (S->pinned_pool[i].first >= floats) {
      float* p = S->pinned_pool[i].second;
      S->pinned_pool.erase(S->pinned_pool.begin() + i);
      return p;
    }
  void* p = nullptr;
  if (hipHostMalloc(&p, std::max<size_t>(floats, 1) * 4, hipHostMallocDefault) != hipSuccess)
    return nullptr;
  return static_cast<float*>(p);
}
void give_pinned(Server* S, float* p, size_t floats) {
  if (p) S->pinned_pool.emplace_back(std::max<size_t>(floats, 1), p);
}

void finish_locked(Server* S, Shot* s, int code) {
  s->status = code;
  s->finished = true;
  s->t_done = now_ns();
  S->finished++;
}

// Device-side admission of `s` into `slot` with its arena block at s->off.
// Runs on the progress thread without the lock.  Returns FD_OK or the code
// the shot ends with.
int admit_device(Server* S, Shot* s, int slot) {
  const fd_shot_desc& d = s->d;
  const ShotLayout& L = s->L;
  char* blk = S->base + s->off;
  float* vol[4];
  for (int i = 0; i < 4; ++i) vol[i] = reinterpret_cast<float*>(blk + i * align_up(L.elems * 4));
  float* sp = reinterpret_cast<float*>(blk + L.sponge);
  int64_t* rec = reinterpret_cast<int64_t*>(blk + L.rec);
  float* tr = reinterpret_cast<float*>(blk + L.traces);
  int32_t* rmap = reinterpret_cast<int32_t*>(blk + L.rmap);
  const Geo geo = make_geo(&L.g);
  hipError_t e = hipSuccess;
  for (int i = 0; i < 3 && e == hipSuccess; ++i) e = launch_zero(vol[i], L.elems, S->as);
  if (e == hipSuccess)
    e = launch_vmax_view(d.nx, d.ny, d.nz, d.v_dev, d.v_ystride, d.v_zstride, S->d_scratch, S->as);
  if (e == hipSuccess)
    e = hipMemcpyAsync(S->h_scratch, S->d_scratch, 8, hipMemcpyDeviceToHost, S->as);
  if (e == hipSuccess) e = hipStreamSynchronize(S->as);
  if (e != hipSuccess) return check_hip(e, "shot admission");
  float vmax, vmin;
  memcpy(&vmax, &S->h_scratch[0], 4);
  memcpy(&vmin, &S->h_scratch[1], 4);
  if (!(isfinite(vmax) && vmax > 0.f && vmin > 0.f))
    return fail(FD_EINVAL, "shot %lld: velocity must be finite and > 0", (long long)s->id);
  const double inv2 = 1.0 / (d.dx * d.dx) + 1.0 / (d.dy * d.dy) + 1.0 / (d.dz * d.dz);
  if ((double)vmax * d.dt * sqrt(symbol_at_nyquist() * inv2) > 2.0)
    return fail(FD_EINVAL, "shot %lld: dt %g is unstable for max(v) %g", (long long)s->id, d.dt,
                (double)vmax);
  e = launch_prepare_vdt2_view(geo, d.v_dev, d.v_ystride, d.v_zstride, vol[3], d.dt, S->as);
  if (e != hipSuccess) return check_hip(e, "shot vdt2");
  // sponge tables and receiver offsets through the pinned staging buffer
  const size_t need = (size_t)(d.nx + d.ny + d.nz) + 2 + 2 * (size_t)std::max(d.nrec, 1) +
                      (d.nrec > 0 ? (size_t)d.nx * (size_t)d.ny : 0);
  if (need > S->h_stage_cap) {
    if (S->h_stage) (void)hipHostFree(S->h_stage);
    S->h_stage = nullptr;
    if (hipHostMalloc((void**)&S->h_stage, need * 4, hipHostMallocDefault) != hipSuccess)
      return fail(FD_ENOMEM, "shot: pinned staging allocation failed");
    S->h_stage_cap = need;
  }
  const double vdesign = d.sponge_vmax > 0 ? d.sponge_vmax : (double)vmax;
  const int n3[3] = {d.nx, d.ny, d.nz};
  const double d3[3] = {d.dx, d.dy, d.dz};
  float* h = S->h_stage;
  for (int a = 0; a < 3; ++a) {
    const double emax = fd_sponge_eta_max(vdesign, d3[a], d.dt, d.sponge_width, kSpongeR);
    fd_sponge_profile(h, n3[a], d.sponge_width, emax < 0 ? 0.0 : emax);
    h += n3[a];
  }
  int64_t* hrec = reinterpret_cast<int64_t*>(S->h_stage + (d.nx + d.ny + d.nz + 1) / 2 * 2);
  if (d.nrec > 0) fd_receiver_offsets(&L.g, s->rec.data(), d.nrec, hrec);
  e = hipMemcpyAsync(sp, S->h_stage, 4 * (size_t)(d.nx + d.ny + d.nz), hipMemcpyHostToDevice,
                     S->as);
  if (e == hipSuccess && d.nrec > 0)
    e = hipMemcpyAsync(rec, hrec, 8 * (size_t)d.nrec, hipMemcpyHostToDevice, S->as);
  // receivers on one plane: the batched kernel writes their rows (no record launch)
  int32_t plane_k = -1;
  if (d.nrec > 0) {
    int32_t* hmap = reinterpret_cast<int32_t*>(hrec + d.nrec);
    if (fd_receiver_plane_map(&L.g, s->rec.data(), d.nrec, hmap, &plane_k) != FD_OK) plane_k = -1;
    if (e == hipSuccess && plane_k >= 0)
      e = hipMemcpyAsync(rmap, hmap, 4 * (size_t)d.nx * (size_t)d.ny, hipMemcpyHostToDevice,
                         S->as);
  }
  // the staging buffer is reused, and the compute stream may use the shot from
  // its next step on: all of the shot's admission work has finished after this
  if (e == hipSuccess) e = hipStreamSynchronize(S->as);
  if (e != hipSuccess) return check_hip(e, "shot upload");
  BatchShot& b = S->shots_host[slot];
  b.g = geo;
  b.c = make_coef(&L.g);
  for (int i = 0; i < 3; ++i) b.arr[i] = vol[i];
  b.q = vol[3];
  b.ex = sp;
  b.ey = sp + d.nx;
  b.ez = sp + d.nx + d.ny;
  b.si = d.src[0];
  b.sj = d.src[1];
  b.sk = d.src[2];
  b.kchunk = kServeKchunk;
  b.rec = rec;
  b.traces = tr;
  b.nrec = d.nrec;
  b.rk = plane_k;
  b.rmap = plane_k >= 0 ? rmap : nullptr;
  s->w.resize(d.nt);
  fd_ricker(s->w.data(), d.nt, 0, d.dt, d.f0, d.t0);
  return FD_OK;
}

// Rebuild and upload the tile table, slot list and slot table.
hipError_t upload_tables(Server* S) {
  const int st = S->stage ^= 1;
  // the upload before the previous one used this staging set; it has landed
  hipError_t e = hipEventSynchronize(S->table_ev[st]);
  if (e != hipSuccess) return e;
  int4* h_tiles = S->h_tiles[st];
  int* h_slots = S->h_slots[st];
  memcpy(S->h_shots[st], S->shots_host.data(), sizeof(BatchShot) * S->max_slots);
  int nt = 0, na = 0, mr = 0;
  int tx, ty;
  const int wpb = batch_tile_shape(&tx, &ty) / 64;  // waves per block
  // one z chunk for all active shots, chosen by the stencil's launch-time model
  // within kTileCap entries (a chunk of kServeKchunk planes always fits)
  std::vector<long long> xy;
  std::vector<int> nzs;
  for (const Shot* s : S->slots)
    if (s) {
      xy.push_back((long long)((s->d.nx + tx - 1) / tx) * ((s->d.ny + ty - 1) / ty));
      nzs.push_back(s->d.nz);
    }
  const int kc = xy.empty() ? kServeKchunk
                            : choose_kchunk(xy.data(), nzs.data(), (int)xy.size(), wpb, 0, kTileCap);
  for (int slot = 0; slot < S->max_slots; ++slot) {
    Shot* s = S->slots[slot];
    if (!s) continue;
    if (s->d.nrec > 0 && !S->shots_host[slot].rmap) {  // rows left to batched_record
      h_slots[na++] = slot;
      mr = std::max(mr, s->d.nrec);
    }
    const int bxn = (s->d.nx + tx - 1) / tx, byn = (s->d.ny + ty - 1) / ty;
    const int bzn = (s->d.nz + kc - 1) / kc;
    S->h_shots[st][slot].kchunk = kc;
    for (int bz = 0; bz < bzn; ++bz)
      for (int by = 0; by < byn; ++by)
        for (int bx = 0; bx < bxn; ++bx) h_tiles[nt++] = make_int4(slot, bx, by, bz);
  }
  S->ntiles = nt;
  S->nactive = na;
  S->max_nrec = mr;
  e = hipMemcpyAsync(S->d_shots, S->h_shots[st], sizeof(BatchShot) * S->max_slots,
                     hipMemcpyHostToDevice, S->cs);
  if (e == hipSuccess && nt)
    e = hipMemcpyAsync(S->d_tiles, h_tiles, sizeof(int4) * nt, hipMemcpyHostToDevice, S->cs);
  if (e == hipSuccess && na)
    e = hipMemcpyAsync(S->d_slots, h_slots, sizeof(int) * na, hipMemcpyHostToDevice, S->cs);
  if (e == hipSuccess) e = hipEventRecord(S->table_ev[st], S->cs);
  S->table_dirty = false;
  return e;
}

int tiles_in_use(Server* S) {
  int t = 0;
  for (Shot* s : S->slots)
    if (s) t += s->L.tiles;
  return t;
}

long long points_in_use(Server* S) {
  long long p = 0;
  for (Shot* s : S->slots)
    if (s) p += (long long)s->d.nx * s->d.ny * s->d.nz;
  return p;
}

void progress(Server* S) {
  const hipError_t dev = hipSetDevice(S->device);
  std::unique_lock<std::mutex> lk(S->mu);
  // without its device the thread can run nothing: every shot fails with FD_EDEVICE
  int fatal = dev == hipSuccess ? FD_OK : check_hip(dev, "server thread: hipSetDevice");
  while (!S->stopping) {
    // ---- admission (strict FIFO)
    while (!S->queue.empty() && fatal == FD_OK) {
      Shot* s = S->queue.front();
      int slot = -1;
      for (int i = 0; i < S->max_slots; ++i)
        if (!S->slots[i]) { slot = i; break; }
      if (slot < 0) break;
      if (tiles_in_use(S) + s->L.tiles > kTileCap) break;
      if (S->max_points > 0 && points_in_use(S) >= S->max_points) break;
      size_t off;
      if (!S->arena->alloc(s->L.total, &off)) break;
      S->queue.pop_front();
      S->queued--;
      s->off = off;
      s->has_block = true;
      s->slot = slot;
      S->slots[slot] = s;  // reserve
      lk.unlock();
      int rc = admit_device(S, s, slot);
      lk.lock();
      s->t_admit = now_ns();
      if (rc == FD_OK) {
        s->host_cap = (size_t)s->d.nt * (size_t)s->d.nrec;
        s->host = take_pinned(S, s->host_cap);
        if (!s->host) rc = fail(FD_ENOMEM, "shot: pinned trace buffer allocation failed");
      }
      if (rc != FD_OK) {
        S->slots[slot] = nullptr;
        S->arena->release(s->off, s->L.total);
        s->has_block = false;
        give_pinned(S, s->host, s->host_cap);
        s->host = nullptr;
        finish_locked(S, s, rc);
        if (rc == FD_EDEVICE) fatal = rc;
        continue;
      }
      S->running++;
      S->table_dirty = true;
    }
    // ---- drain finished copies
    for (size_t i = 0; i < S->draining.size();) {
      Shot* s = S->draining[i];
      const hipError_t q = hipEventQuery(s->copied);
      if (q == hipErrorNotReady) { ++i; continue; }
      S->arena->release(s->off, s->L.total);
      s->has_block = false;
      (void)hipEventDestroy(s->copied);
      s->copied = nullptr;
      S->running--;
      finish_locked(S, s, q == hipSuccess ? FD_OK : FD_EDEVICE);
      S->draining.erase(S->draining.begin() + i);
      S->cv.notify_all();
    }
    if (fatal != FD_OK) {  // the device failed: nothing queued can run
      for (Shot* s : S->queue) {
        finish_locked(S, s, fatal);
        S->queued--;
      }
      S->queue.clear();
    }
    bool any = false;
    for (Shot* s : S->slots) any = any || s != nullptr;
    if (!any || fatal != FD_OK) {
      if (S->draining.empty())
        S->cv.wait_for(lk, std::chrono::milliseconds(2));
      else
        S->cv.wait_for(lk, std::chrono::microseconds(200));
      continue;
    }
    // ---- one batched step of every active shot
    BatchStep a;
    for (int i = 0; i < MAX_BATCH_SLOTS; ++i) {
      a.n[i] = 0;
      a.w[i] = 0.f;
    }
    for (int slot = 0; slot < S->max_slots; ++slot)
      if (Shot* s = S->slots[slot]) {
        a.n[slot] = s->n;
        a.w[slot] = s->w[s->n];
      }
    const bool dirty = S->table_dirty;
    lk.unlock();
    hipError_t e = hipSuccess;
    const int64_t step = S->steps, grp = step / kEventEvery;
    // the first step of group grp waits for the end of group grp - kInflight
    if (step % kEventEvery == 0 && grp >= kInflight)
      e = hipEventSynchronize(S->step_ev[grp % kInflight]);
    if (e == hipSuccess && dirty) e = upload_tables(S);
    if (e == hipSuccess) e = launch_batched(S->d_shots, S->d_tiles, S->ntiles, a, S->cs);
    if (e == hipSuccess)
      e = launch_batched_record(S->d_shots, S->d_slots, S->nactive, S->max_nrec, a, S->cs);
    if (e == hipSuccess && step % kEventEvery == kEventEvery - 1)
      e = hipEventRecord(S->step_ev[grp % kInflight], S->cs);
    lk.lock();
    S->steps++;
    if (e != hipSuccess) {
      check_hip(e, "batched step");
      fatal = FD_EDEVICE;
      for (int slot = 0; slot < S->max_slots; ++slot)
        if (Shot* s = S->slots[slot]) {
          S->slots[slot] = nullptr;
          if (s->has_block) S->arena->release(s->off, s->L.total);
          s->has_block = false;
          S->running--;
          finish_locked(S, s, FD_EDEVICE);
        }
      continue;
    }
    // ---- advance; retire shots that reached nt
    for (int slot = 0; slot < S->max_slots; ++slot) {
      Shot* s = S->slots[slot];
      if (!s) continue;
      s->n++;
      if (s->n < s->d.nt) continue;
      S->slots[slot] = nullptr;
      S->table_dirty = true;
      hipError_t r = hipEventCreateWithFlags(&s->copied, hipEventDisableTiming);
      hipEvent_t stepped = nullptr;
      if (r == hipSuccess) r = hipEventCreateWithFlags(&stepped, hipEventDisableTiming);
      if (r == hipSuccess) r = hipEventRecord(stepped, S->cs);
      if (r == hipSuccess) r = hipStreamWaitEvent(S->xs, stepped, 0);
      if (r == hipSuccess && s->host_cap)
        r = hipMemcpyAsync(s->host, reinterpret_cast<char*>(S->base) + s->off + s->L.traces,
                           4 * s->host_cap, hipMemcpyDeviceToHost, S->xs);
      if (r == hipSuccess) r = hipEventRecord(s->copied, S->xs);
      if (stepped) (void)hipEventDestroy(stepped);
      if (r != hipSuccess) {
        check_hip(r, "trace copy");
        S->arena->release(s->off, s->L.total);
        s->has_block = false;
        S->running--;
        finish_locked(S, s, FD_EDEVICE);
        continue;
      }
      S->draining.push_back(s);
    }
  }
  lk.unlock();
  // let queued device work finish before the caller frees anything
  (void)hipStreamSynchronize(S->cs);
  (void)hipStreamSynchronize(S->xs);
}

void stop_server(Server* S) {
  {
    std::lock_guard<std::mutex> g(S->mu);
    if (S->stopped) return;
    S->stopping = true;
  }
  S->cv.notify_all();
  if (S->th.joinable()) S->th.join();
  std::lock_guard<std::mutex> g(S->mu);
  for (Shot* s : S->queue) {
    finish_locked(S, s, FD_ECANCELED);
    S->queued--;
  }
  S->queue.clear();
  for (int slot = 0; slot < S->max_slots; ++slot)
    if (Shot* s = S->slots[slot]) {
      S->slots[slot] = nullptr;
      if (s->has_block) S->arena->release(s->off, s->L.total);
      s->has_block = false;
      S->running--;
      finish_locked(S, s, FD_ECANCELED);
    }
  for (Shot* s : S->draining) {  // copies ended in the final synchronisation
    const bool landed = s->copied && hipEventQuery(s->copied) == hipSuccess;
    if (s->copied) (void)hipEventDestroy(s->copied);
    s->copied = nullptr;
    if (s->has_block) S->arena->release(s->off, s->L.total);
    s->has_block = false;
    S->running--;
    finish_locked(S, s, landed ? FD_OK : FD_EDEVICE);
  }
  S->draining.clear();
  S->stopped = true;
}

}  // namespace
}  // namespace fd

using namespace fd;

extern "C" {

int64_t fd_shot_footprint(const fd_shot_desc* d) {
  ShotLayout L;
  if (layout_for(d, &L) != FD_OK) return -1;
  return (int64_t)L.total;
}

int fd_server_create(void** srv, void* arena_dev, size_t arena_bytes, int32_t max_slots,
                     void* compute_stream, void* copy_stream) {
  if (!srv) return fail(FD_EINVAL, "fd_server_create: srv is NULL");
  *srv = nullptr;
  if (!arena_dev || ((uintptr_t)arena_dev % kAlign) != 0)
    return fail(FD_EINVAL, "fd_server_create: arena must be non-NULL and 256-byte aligned");
  if (max_slots < 1 || max_slots > MAX_BATCH_SLOTS)
    return fail(FD_EINVAL, "fd_server_create: max_slots must be in 1..%d", MAX_BATCH_SLOTS);
  const size_t head = align_up(sizeof(BatchShot) * MAX_BATCH_SLOTS) +
                      align_up(sizeof(int4) * kTileCap) + align_up(sizeof(int) * MAX_BATCH_SLOTS) +
                      align_up(8);
  if (arena_bytes < head + kAlign)
    return fail(FD_ENOMEM, "fd_server_create: arena of %zu bytes is too small", arena_bytes);
  std::unique_ptr<Server> S(new Server());
  S->base = static_cast<char*>(arena_dev);
  S->max_slots = max_slots;
  char* p = S->base;
  S->d_shots = reinterpret_cast<BatchShot*>(p);
  p += align_up(sizeof(BatchShot) * MAX_BATCH_SLOTS);
  S->d_tiles = reinterpret_cast<int4*>(p);
  p += align_up(sizeof(int4) * kTileCap);
  S->d_slots = reinterpret_cast<int*>(p);
  p += align_up(sizeof(int) * MAX_BATCH_SLOTS);
  S->d_scratch = reinterpret_cast<int32_t*>(p);
  p += align_up(8);
  S->base = p;  // shot blocks live after the tables
  S->bytes = arena_bytes - head;
  S->arena.reset(new Arena(S->bytes / kAlign * kAlign));
  S->slots.assign(max_slots, nullptr);
  int rc = check_hip(hipGetDevice(&S->device), "fd_server_create");
  if (rc) return rc;
  hipError_t e = hipSuccess;
  S->cs = reinterpret_cast<hipStream_t>(compute_stream);
  S->xs = reinterpret_cast<hipStream_t>(copy_stream);
  if (!S->cs) {
    e = hipStreamCreateWithFlags(&S->cs, hipStreamNonBlocking);
    S->own_cs = e == hipSuccess;
  }
  if (e == hipSuccess && !S->xs) {
    e = hipStreamCreateWithFlags(&S->xs, hipStreamNonBlocking);
    S->own_xs = e == hipSuccess;
  }
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&S->as, hipStreamNonBlocking);
  for (int i = 0; i < 2 && e == hipSuccess; ++i) {
    e = hipHostMalloc((void**)&S->h_shots[i], sizeof(BatchShot) * MAX_BATCH_SLOTS,
                      hipHostMallocDefault);
    if (e == hipSuccess)
      e = hipHostMalloc((void**)&S->h_tiles[i], sizeof(int4) * kTileCap, hipHostMallocDefault);
    if (e == hipSuccess)
      e = hipHostMalloc((void**)&S->h_slots[i], sizeof(int) * MAX_BATCH_SLOTS,
                        hipHostMallocDefault);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&S->table_ev[i], hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(S->table_ev[i], S->cs);
  }
  if (e == hipSuccess) e = hipHostMalloc((void**)&S->h_scratch, 8, hipHostMallocDefault);
  // throttle events only tell how far the device got; without the system-scope
  // release (an L2 write-back) an event between two steps costs no idle time
  for (int i = 0; i < kInflight && e == hipSuccess; ++i)
    e = hipEventCreateWithFlags(&S->step_ev[i], hipEventDisableTiming | hipEventDisableSystemFence);
  if (e != hipSuccess) {
    rc = check_hip(e, "fd_server_create");
    Server* raw = S.release();
    raw->stopped = true;
    fd_server_destroy(raw);
    return rc;
  }
  S->shots_host.assign(MAX_BATCH_SLOTS, BatchShot{});
  Server* raw = S.release();
  raw->th = std::thread(progress, raw);
  *srv = raw;
  return FD_OK;
}

int shot_submit(void* srv, const fd_shot_desc* d, int64_t* shot_id) {
  Server* S = static_cast<Server*>(srv);
  if (!S || !shot_id) return fail(FD_EINVAL, "shot_submit: NULL server or id");
  ShotLayout L;
  int rc = layout_for(d, &L);
  if (rc) return rc;
  if (!d->v_dev) return fail(FD_EINVAL, "shot_submit: v_dev is NULL");
  if (d->v_ystride < d->nx || d->v_zstride < d->v_ystride * (int64_t)d->ny)
    return fail(FD_EINVAL, "shot_submit: velocity view strides too small");
  if (!(d->dt > 0) || !isfinite(d->dt) || !(d->f0 > 0) || !isfinite(d->t0))
    return fail(FD_EINVAL, "shot_submit: bad dt, f0 or t0");
  if (d->sponge_width < 0) return fail(FD_EINVAL, "shot_submit: sponge_width < 0");
  if (d->src[0] < 0 || d->src[0] >= d->nx || d->src[1] < 0 || d->src[1] >= d->ny ||
      d->src[2] < 0 || d->src[2] >= d->nz)
    return fail(FD_EINVAL, "shot_submit: source outside the interior");
  if (d->nrec > 0 && !d->rec_ijk_host) return fail(FD_EINVAL, "shot_submit: receivers NULL");
  std::unique_ptr<Shot> s(new Shot());
  s->rec.assign(d->rec_ijk_host, d->rec_ijk_host + 3 * (size_t)std::max(d->nrec, 0));
  for (int32_t r = 0; r < d->nrec; ++r) {
    const int32_t i = s->rec[3 * r], j = s->rec[3 * r + 1], k = s->rec[3 * r + 2];
    if (i < 0 || i >= d->nx || j < 0 || j >= d->ny || k < 0 || k >= d->nz)
      return fail(FD_EINVAL, "shot_submit: receiver %d outside the interior", r);
  }
  if (L.total > S->bytes || L.tiles > kTileCap)
    return fail(FD_ENOMEM, "shot_submit: footprint %zu bytes can never fit the arena (%zu)",
                L.total, S->bytes);
  s->d = *d;
  s->d.rec_ijk_host = nullptr;
  s->L = L;
  s->t_submit = now_ns();
  std::lock_guard<std::mutex> g(S->mu);
  if (S->stopping) return fail(FD_ECANCELED, "shot_submit: server is shut down");
  s->id = S->next_id++;
  *shot_id = s->id;
  S->queue.push_back(s.get());
  S->queued++;
  S->shots[s->id] = std::move(s);
  S->cv.notify_all();
  return FD_OK;
}

int shot_poll(void* srv, int64_t shot_id, float* traces_host, size_t cap, int64_t t_ns[3]) {
  Server* S = static_cast<Server*>(srv);
  if (!S) return fail(FD_EINVAL, "shot_poll: NULL server");
  std::lock_guard<std::mutex> g(S->mu);
  auto it = S->shots.find(shot_id);
  if (it == S->shots.end()) return fail(FD_ENOTFOUND, "shot %lld not known", (long long)shot_id);
  Shot* s = it->second.get();
  if (!s->finished) return FD_EAGAIN;
  if (traces_host && s->host && s->status == FD_OK)
    memcpy(traces_host, s->host, 4 * std::min(cap, s->host_cap));
  if (t_ns) {
    t_ns[0] = s->t_submit;
    t_ns[1] = s->t_admit;
    t_ns[2] = s->t_done;
  }
  const int code = s->status;
  give_pinned(S, s->host, s->host_cap);
  S->finished--;
  S->shots.erase(it);
  if (code != FD_OK) fail(code, "shot %lld ended with %s", (long long)shot_id, fd_strerror(code));
  return code;
}

int fd_server_set_admission(void* srv, int64_t max_active_points) {
  Server* S = static_cast<Server*>(srv);
  if (!S) return fail(FD_EINVAL, "fd_server_set_admission: NULL server");
  if (max_active_points < 0) return fail(FD_EINVAL, "max_active_points must be >= 0");
  {
    std::lock_guard<std::mutex> g(S->mu);
    S->max_points = max_active_points;
  }
  S->cv.notify_all();
  return FD_OK;
}

int fd_server_stats(void* srv, int64_t out[4]) {
  Server* S = static_cast<Server*>(srv);
  if (!S || !out) return fail(FD_EINVAL, "fd_server_stats: NULL argument");
  std::lock_guard<std::mutex> g(S->mu);
  out[0] = S->queued;
  out[1] = S->running;
  out[2] = S->finished;
  out[3] = S->steps;
  return FD_OK;
}

int fd_server_shutdown(void* srv) {
  Server* S = static_cast<Server*>(srv);
  if (!S) return fail(FD_EINVAL, "fd_server_shutdown: NULL server");
  stop_server(S);
  return FD_OK;
}

int fd_server_destroy(void* srv) {
  Server* S = static_cast<Server*>(srv);
  if (!S) return fail(FD_EINVAL, "fd_server_destroy: NULL server");
  stop_server(S);
  for (auto& kv : S->shots) give_pinned(S, kv.second->host, kv.second->host_cap);
  for (auto& pb : S->pinned_pool) (void)hipHostFree(pb.second);
  if (S->h_stage) (void)hipHostFree(S->h_stage);
  for (int i = 0; i < 2; ++i) {
    if (S->h_shots[i]) (void)hipHostFree(S->h_shots[i]);
    if (S->h_tiles[i]) (void)hipHostFree(S->h_tiles[i]);
    if (S->h_slots[i]) (void)hipHostFree(S->h_slots[i]);
    if (S->table_ev[i]) (void)hipEventDestroy(S->table_ev[i]);
  }
  if (S->h_scratch) (void)hipHostFree(S->h_scratch);
  for (int i = 0; i < kInflight; ++i)
    if (S->step_ev[i]) (void)hipEventDestroy(S->step_ev[i]);
  if (S->own_cs) (void)hipStreamDestroy(S->cs);
  if (S->own_xs) (void)hipStreamDestroy(S->xs);
  if (S->as) (void)hipStreamDestroy(S->as);
  delete S;
  return FD_OK;
}

}  // extern "C"
