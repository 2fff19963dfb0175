// fd_server.cpp -- continuous-batching server for independent forward shots.
//
// One progress thread per server owns the device work.  A shot moves through:
//   queued  : submitted, waiting in strict FIFO order;
//   staging : its arena block is reserved (first fit or buddy, one caller-owned
//             arena: the paper's global segment, Sec. 3.1) and its admission work
//             runs asynchronously on a stream of a bounded pool (lazy creation,
//             reuse, MAX_ACTIVE_STREAMS with partial synchronisation, Sec. 3.2):
//             phase 1 zeroes its wavefields and reduces max(v) into its block;
//             phase 2, once the maximum is on the host (stability checked), builds
//             vdt2 from the caller's velocity view and uploads sponge tables,
//             receiver offsets and a receiver-plane map; at most kPrepareAhead
//             shots are staging or staged at once, so their admission overlaps
//             the steps of the running shots;
//   staged  : ready, waiting to join the batched step;
//   active  : in a slot: every active shot advances one time step per batched
//             step, each at its own step n (u^n in arr[n % 3]);
//   draining: all steps done, traces copying to pinned host memory;
//   done    : collected by shot_poll.
// Activation (strict FIFO) needs a free slot and tile-table room, and the points of
// the running shots and the new one within the fill (kFillPoints; kBacklogPoints
// while more shots wait; else the caller's cap): a grid that fills the device runs
// alone, grids that are small together share it.
// A batched step advances every active shot by one launch: a lone shot by the
// kernel its grid takes alone; several, if one of them is a grid of at least 7.5M
// points, all by the 16-byte-lane kernel (up to kWideMulti grids with their
// parameters in the kernel arguments, each in 128 x 32 tiles or, where those would
// leave a tenth more of its plane empty, 64 x 64; more through a tile table of
// 128 x 32 tiles), else by the
// one-float-per-lane kernel over a tile table (64 x 32 tiles).  Both write the trace
// rows of shots whose receivers share one plane; one batched receiver launch takes
// the others.
// At most kEventEvery * kInflight steps are queued ahead of the device.  The arena,
// compute and copy streams and all device memory are the caller's; the server only
// carves.
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
#include "fd_stream_pool.h"

namespace fd {
namespace {

constexpr size_t kAlign = 256;
// The progress thread runs at most kEventEvery * kInflight batched steps ahead of
// the device: enough that a lone small grid's short steps (10 us at 128^3) never
// wait for the thread to wake, few enough that a shot that becomes ready joins within
// a few milliseconds.  It records a throttle event once per kEventEvery steps, not
// every step: each event between two launches leaves the device idle ~4.7 us even
// without the system-scope release (kernel trace of lone shots of the 128..384^3
// mix: one event per 8 steps cost 0.5 ms of a 30 ms shot)
constexpr int kInflight = 4;
constexpr int kEventEvery = 32;
constexpr int kTileCap = 1 << 16;   // tile-table entries
// z planes per tile-table entry counted against kTileCap at activation (64 x 32
// tiles: the larger count of the two families).  The table itself uses the z chunk
// the launch model picks for the active shots of each family, within kTileCap.
constexpr int kServeKchunk = 24;
constexpr double kSpongeR = 1e-3;
constexpr int kPrepareAhead = 4;      // shots staging or staged at once
constexpr int kAdmitStreams = 4;      // bound of the admission stream pool
// Activation fills the device: the running shots are enough for it when they give
// every CU one 128 x 32 tile of 8 planes (the z chunk whose 8-plane z halo is as deep
// as the chunk itself): 256 x 4096 x 8 points.  Measured against the plain loop on
// the Poisson streams of the 128..384^3 mix (throughput at 2x its rate, p50 at 0.5x)
// and of the 48..128^3 mix: 8.4M points 1.000x / 41.0 ms / 1.56x; 16.8M 1.002x /
// 44.6 ms / 1.52x; 4.2M 0.996x / 40.9 ms / 1.42x; one shot at a time 0.995x / 41.0 ms /
// 0.95x (plain: 39.8 ms).
constexpr long long kFillPoints = 256LL * 128 * 32 * 8;
// Under a backlog the running shots may hold up to this many points.  One launch of
// two mid-size grids beats two launches (336 x 150 x 174 twice: 59.0 us against 2 x
// 32.8; 256^3 twice: 90.6 against 2 x 47.8), of a large and a small grid it does not
// (384^3 and 256^3: 222 us against 162 + 48).  Throughput at twice the plain loop's
// rate on the 128..384^3 mix, with a cap on the running points at all steps (the same
// box, three alternating runs each): 8.4M points 1.001x, 16.8M 1.004x, no co-running
// 1.003x, against 0.999x for the fill with 25.2M under a backlog (before the 64 x 64
// tiles for ragged grids, on another box: 8.4M 1.006x, 16.8M 1.009x, 25.2M 1.020x,
// 33.6M 1.016x, 67.1M 0.916x).  Joining wherever the launch model (choose_kchunk's)
// prices one launch of the running shots and the new one below the two launches apart
// ran more shots together and gave 0.987x: the model overrates one launch of two large
// grids.
constexpr long long kBacklogPoints = 2 * kFillPoints;

size_t align_up(size_t n) { return (n + kAlign - 1) / kAlign * kAlign; }

int64_t now_ns() {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

struct HipStreams {  // stream operations of the admission pool
  using Stream = hipStream_t;
  bool create(Stream* s) { return hipStreamCreateWithFlags(s, hipStreamNonBlocking) == hipSuccess; }
  bool done(Stream s) { return hipStreamQuery(s) != hipErrorNotReady; }
  void sync(Stream s) { (void)hipStreamSynchronize(s); }
  void destroy(Stream s) { (void)hipStreamDestroy(s); }
};

// Layout of one shot's arena block.
struct ShotLayout {
  fd_grid g;
  int64_t elems;
  size_t vol, sponge, rec, traces, rmap, vm, total;  // byte offsets and total
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
  L->vm = L->rmap + (d->nrec > 0 ? align_up(4 * (size_t)d->nx * (size_t)d->ny) : 0);
  L->total = L->vm + kAlign;  // two int32: max and min of v
  int tx, ty;
  batch_tile_shape(&tx, &ty);
  const long long t = (long long)((d->nx + tx - 1) / tx) * ((d->ny + ty - 1) / ty) *
                      ((d->nz + kServeKchunk - 1) / kServeKchunk);
  L->tiles = (int)std::min<long long>(t, 1LL << 30);
  return FD_OK;
}

// Staging: the admission work waits for max(v) on the host before building the model
// (the sponge is designed for the shot's own maximum); Issued: all admission work is
// enqueued, the shot may join the step (the compute stream then waits for that work),
// its stability check may still be pending; Staged: all admission work has finished.
enum class State { Queued, Staging, Issued, Staged, Active, Draining, Done };

struct Shot {
  int64_t id = 0;
  fd_shot_desc d{};
  std::vector<int32_t> rec;
  ShotLayout L{};
  State state = State::Queued;
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
  // admission
  hipStream_t as = nullptr;   // pool stream of its admission work
  hipEvent_t ev = nullptr;    // end of the current admission phase
  hipEvent_t mev = nullptr;   // end of the model's uploads, before the stability check
                              // of the same phase (NULL: ev ends both)
  float* stage = nullptr;     // pinned: max/min of v, then the tables to upload
  size_t stage_cap = 0;       // floats
  bool wide = false;          // a grid the 16-byte-lane kernel steps when alone
  bool in_wide = false;       // stepped by the 16-byte-lane kernels now
  int plane_k = -1;           // receivers on one z plane (else -1)
  bool check_pending = false; // max(v) not yet checked for stability
  int abort_code = FD_OK;     // an active shot removed before its end ends with this
  Geo geo{};
  Coef coef{};
};

struct Server {
  char* base = nullptr;
  size_t bytes = 0;
  int max_slots = 0;
  int device = 0;
  hipStream_t cs = nullptr, xs = nullptr;
  bool own_cs = false, own_xs = false;
  std::unique_ptr<ArenaAllocator> arena;
  int arena_kind = FD_ARENA_FIRST_FIT;
  bool submitted = false;  // the allocator can no longer change
  std::unique_ptr<StreamPool<HipStreams>> pool;
  // device tables (head of the arena), the host master slot table and two pinned
  // staging sets used in turn, so that rebuilding the tables never waits for the
  // copy of the previous upload
  BatchShot* d_shots = nullptr;
  int4* d_tiles = nullptr;  // the 64 x 32 family's entries, then the 16-byte-lane family's
  int* d_slots = nullptr;
  std::vector<BatchShot> shots_host;
  BatchShot* h_shots[2] = {};
  int4* h_tiles[2] = {};
  int* h_slots[2] = {};
  hipEvent_t table_ev[2] = {};
  int stage = 0;
  hipEvent_t step_ev[kInflight] = {};
  int ntiles = 0, ntiles4 = 0, nactive = 0, max_nrec = 0;
  // a family with one active shot steps it with the single-grid launch instead (the
  // kernels and launch shape the same grid takes alone; the batched kernels' per-block
  // look-up of its tile and shot costs 5-9% of a short step)
  Shot* direct[2] = {nullptr, nullptr};
  bool direct_rows[2] = {false, false};  // the direct launch writes the receiver row
  // 2..kWideMulti shots of the 16-byte-lane family: one launch with their parameters
  // in the kernel arguments (no tile table, no per-block look-up)
  std::vector<Shot*> multi;
  bool table_dirty = false;
  // shared state
  std::mutex mu;
  std::condition_variable cv;
  std::deque<Shot*> queue;  // queued
  std::deque<Shot*> prep;   // staging or staged, in submission order
  std::map<int64_t, std::unique_ptr<Shot>> shots;
  std::vector<Shot*> slots;
  std::vector<Shot*> draining;
  std::vector<std::pair<size_t, float*>> pinned_pool;
  int64_t next_id = 1;
  int64_t steps = 0;
  int64_t max_points = 0;  // > 0: activation waits while the slots hold this many points
  int queued = 0, running = 0, finished = 0;
  bool stopping = false, stopped = false;
  std::thread th;
};

// ---- pinned host buffers (reused: hipHostFree can stall the device)
float* take_pinned(Server* S, size_t floats, size_t* cap) {
  size_t best = S->pinned_pool.size();
  for (size_t i = 0; i < S->pinned_pool.size(); ++i)
    if (S->pinned_pool[i].first >= floats &&
        (best == S->pinned_pool.size() || S->pinned_pool[i].first < S->pinned_pool[best].first))
      best = i;
  if (best < S->pinned_pool.size()) {
    float* p = S->pinned_pool[best].second;
    *cap = S->pinned_pool[best].first;
    S->pinned_pool.erase(S->pinned_pool.begin() + best);
    return p;
  }
  void* p = nullptr;
  *cap = std::max<size_t>(floats, 1);
  if (hipHostMalloc(&p, *cap * 4, hipHostMallocDefault) != hipSuccess) return nullptr;
  return static_cast<float*>(p);
}
void give_pinned(Server* S, float* p, size_t cap) {
  if (p) S->pinned_pool.emplace_back(cap, p);
}

void finish_locked(Server* S, Shot* s, int code) {
  s->status = code;
  s->finished = true;
  s->state = State::Done;
  s->t_done = now_ns();
  S->finished++;
}

float* shot_vol(Server* S, const Shot* s, int i) {
  return reinterpret_cast<float*>(S->base + s->off + (size_t)i * align_up(s->L.elems * 4));
}
char* shot_at(Server* S, const Shot* s, size_t field) { return S->base + s->off + field; }

// Stability of the shot's time step for the max(v) its admission work copied to
// the staging buffer.  FD_OK or FD_EINVAL.
int check_vmax(const Shot* s) {
  const fd_shot_desc& d = s->d;
  float vmax, vmin;
  memcpy(&vmax, &s->stage[0], 4);
  memcpy(&vmin, &s->stage[1], 4);
  if (!(isfinite(vmax) && vmax > 0.f && vmin > 0.f))
    return fail(FD_EINVAL, "shot %lld: velocity must be finite and > 0", (long long)s->id);
  const double inv2 = 1.0 / (d.dx * d.dx) + 1.0 / (d.dy * d.dy) + 1.0 / (d.dz * d.dz);
  if ((double)vmax * d.dt * sqrt(symbol_at_nyquist() * inv2) > 2.0)
    return fail(FD_EINVAL, "shot %lld: dt %g is unstable for max(v) %g", (long long)s->id, d.dt,
                (double)vmax);
  return FD_OK;
}

// The model on the shot's admission stream: vdt2 from the caller's velocity view, and
// (host) sponge tables for the design velocity vdesign, receiver offsets and plane
// map into the staging buffer, uploaded; then event `end`.
hipError_t admit_model(Server* S, Shot* s, double vdesign, hipEvent_t end) {
  const fd_shot_desc& d = s->d;
  const ShotLayout& L = s->L;
  const Geo geo = make_geo(&L.g);
  hipError_t e = launch_prepare_vdt2_view(geo, d.v_dev, d.v_ystride, d.v_zstride,
                                          shot_vol(S, s, 3), d.dt, s->as);
  if (e != hipSuccess) return e;
  // staging layout (floats): [2: max/min] [nx+ny+nz: sponge] [pad to even]
  // [2*nrec: int64 offsets] [nx*ny: int32 plane map]
  float* h = s->stage + 2;
  const int n3[3] = {d.nx, d.ny, d.nz};
  const double d3[3] = {d.dx, d.dy, d.dz};
  for (int a = 0; a < 3; ++a) {
    const double emax = fd_sponge_eta_max(vdesign, d3[a], d.dt, d.sponge_width, kSpongeR);
    fd_sponge_profile(h, n3[a], d.sponge_width, emax < 0 ? 0.0 : emax);
    h += n3[a];
  }
  int64_t* hrec = reinterpret_cast<int64_t*>(s->stage + 2 + (d.nx + d.ny + d.nz + 1) / 2 * 2);
  if (d.nrec > 0) fd_receiver_offsets(&L.g, s->rec.data(), d.nrec, hrec);
  e = hipMemcpyAsync(shot_at(S, s, L.sponge), s->stage + 2, 4 * (size_t)(d.nx + d.ny + d.nz),
                     hipMemcpyHostToDevice, s->as);
  if (e == hipSuccess && d.nrec > 0)
    e = hipMemcpyAsync(shot_at(S, s, L.rec), hrec, 8 * (size_t)d.nrec, hipMemcpyHostToDevice,
                       s->as);
  // receivers on one plane: the stencil kernels write their rows themselves
  s->plane_k = -1;
  if (d.nrec > 0) {
    int32_t* hmap = reinterpret_cast<int32_t*>(hrec + d.nrec);
    if (fd_receiver_plane_map(&L.g, s->rec.data(), d.nrec, hmap, &s->plane_k) != FD_OK)
      s->plane_k = -1;
    if (e == hipSuccess && s->plane_k >= 0)
      e = hipMemcpyAsync(shot_at(S, s, L.rmap), hmap, 4 * (size_t)d.nx * (size_t)d.ny,
                         hipMemcpyHostToDevice, s->as);
  }
  if (e == hipSuccess) e = hipEventRecord(end, s->as);
  s->w.resize(d.nt);
  fd_ricker(s->w.data(), d.nt, 0, d.dt, d.f0, d.t0);
  s->wide = forward_wide_tiles(geo);
  return e;
}

// The admission work that needs nothing from the host, on the shot's pool stream:
// zero the three wavefields, reduce max(v) and min(v) into the block and copy them to
// the staging buffer.  When the sponge's design velocity is known without that
// maximum (given, or no sponge), the model (admit_model) comes first, ending with
// event mev, so that the shot can join the step as soon as its model has landed, its
// stability checked when the maximum arrives (event ev); else the maximum comes
// first (ev) and the host builds the model from it.  *whole tells which.
hipError_t admit_start(Server* S, Shot* s, bool* whole) {
  const fd_shot_desc& d = s->d;
  int32_t* vm = reinterpret_cast<int32_t*>(shot_at(S, s, s->L.vm));
  *whole = d.sponge_width == 0 || d.sponge_vmax > 0;
  // the three wavefields are adjacent in the block: one launch zeroes them
  hipError_t e = launch_zero(shot_vol(S, s, 0), (long long)(shot_vol(S, s, 3) - shot_vol(S, s, 0)), s->as);
  if (e == hipSuccess && *whole) {
    e = hipEventCreateWithFlags(&s->mev, hipEventDisableTiming);
    if (e == hipSuccess) e = admit_model(S, s, d.sponge_width ? d.sponge_vmax : 0.0, s->mev);
  }
  if (e == hipSuccess)
    e = launch_vmax_view(d.nx, d.ny, d.nz, d.v_dev, d.v_ystride, d.v_zstride, vm, s->as);
  if (e == hipSuccess) e = hipMemcpyAsync(s->stage, vm, 8, hipMemcpyDeviceToHost, s->as);
  if (e != hipSuccess) return e;
  return hipEventRecord(s->ev, s->as);
}

// Destroy the admission events of a shot whose admission work has all landed (or
// whose stream was synchronised).
void drop_events(Shot* s) {
  if (s->ev) (void)hipEventDestroy(s->ev);
  if (s->mev) (void)hipEventDestroy(s->mev);
  s->ev = s->mev = nullptr;
}

// Staging floats a shot needs (see admit_model).
size_t stage_floats(const fd_shot_desc& d) {
  return 2 + (size_t)(d.nx + d.ny + d.nz + 1) / 2 * 2 + 2 * (size_t)std::max(d.nrec, 0) +
         (d.nrec > 0 ? (size_t)d.nx * (size_t)d.ny : 0);
}

// The slot-table entry of an activated shot.
void fill_slot(Server* S, Shot* s, int slot) {
  const ShotLayout& L = s->L;
  BatchShot& b = S->shots_host[slot];
  s->geo = make_geo(&L.g);
  s->coef = make_coef(&L.g);
  b.g = s->geo;
  b.c = s->coef;
  for (int i = 0; i < 3; ++i) b.arr[i] = shot_vol(S, s, i);
  b.q = shot_vol(S, s, 3);
  float* sp = reinterpret_cast<float*>(shot_at(S, s, L.sponge));
  b.ex = sp;
  b.ey = sp + s->d.nx;
  b.ez = sp + s->d.nx + s->d.ny;
  b.si = s->d.src[0];
  b.sj = s->d.src[1];
  b.sk = s->d.src[2];
  b.kchunk = kServeKchunk;
  b.rec = reinterpret_cast<int64_t*>(shot_at(S, s, L.rec));
  b.traces = reinterpret_cast<float*>(shot_at(S, s, L.traces));
  b.nrec = s->d.nrec;
  // receivers on one plane: the batched stencil kernels write their rows
  const bool in_kernel = s->plane_k >= 0;
  b.rk = in_kernel ? s->plane_k : -1;
  b.rmap = in_kernel ? reinterpret_cast<int32_t*>(shot_at(S, s, L.rmap)) : nullptr;
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

// Whether shot s (the head of the staged shots) may join the active ones now (a shot
// always joins when none runs).  Shots of one batched launch advance one step per
// launch, in lockstep, so a grid that joins a smaller running one slows it to its
// own pace: that trades the running shots' latency for throughput.  With a caller's
// cap: when their points and its own stay within it.  By default: within the fill
// (grids that together still leave the device short of work), or, while more shots
// wait behind s (a backlog, where throughput decides), within kBacklogPoints.
bool activation_pays(Server* S, const Shot* s) {
  bool any = false;
  for (const Shot* r : S->slots) any = any || r != nullptr;
  if (!any) return true;
  const long long after = points_in_use(S) + (long long)s->d.nx * s->d.ny * s->d.nz;
  if (S->max_points > 0) return after <= S->max_points;
  if (after <= kFillPoints) return true;
  const bool backlog = S->prep.size() > 1 || !S->queue.empty();
  return backlog && after <= kBacklogPoints;
}

// Rebuild and upload the tile tables, slot list and slot table.
hipError_t upload_tables(Server* S) {
  const int st = S->stage ^= 1;
  // the upload before the previous one used this staging set; it has landed
  hipError_t e = hipEventSynchronize(S->table_ev[st]);
  if (e != hipSuccess) return e;
  int4* h_tiles = S->h_tiles[st];
  int* h_slots = S->h_slots[st];
  memcpy(S->h_shots[st], S->shots_host.data(), sizeof(BatchShot) * S->max_slots);
  int na = 0, mr = 0;
  int counts[2] = {0, 0};
  // each family: one z chunk for its shots from the launch model, within the table
  // (a chunk of the deepest grid's depth always fits: activation keeps the tiles of
  // kServeKchunk-plane chunks within kTileCap)
  int kc[2] = {kServeKchunk, kServeKchunk};
  int tws[2][2];
  int wpb[2];
  wpb[0] = batch_tile_shape(&tws[0][0], &tws[0][1]) / 64;
  wpb[1] = batch4_tile_shape(&tws[1][0], &tws[1][1]);
  std::vector<long long> xy[2];
  std::vector<int> nzs[2];
  long long least[2] = {0, 0};  // entries at one chunk per grid
  int fam[2] = {0, 0};
  // the family of every active shot: where one of them is a grid for the 16-byte-lane
  // kernel, all of them are stepped by it (one launch of all the grids: a smaller
  // grid's tiles fill the launch of a larger one; every kernel gives the same bits),
  // else by the one-float-per-lane kernels
  bool any_wide = false;
  for (const Shot* s : S->slots) any_wide = any_wide || (s && s->wide);
  for (Shot* s : S->slots)
    if (s) s->in_wide = any_wide;
  for (int f = 0; f < 2; ++f) S->direct[f] = nullptr;
  for (Shot* s : S->slots)
    if (s) {
      ++fam[s->in_wide ? 1 : 0];
      S->direct[s->in_wide ? 1 : 0] = s;
    }
  S->multi.clear();
  if (fam[1] >= 2 && fam[1] <= kWideMulti)
    for (Shot* s : S->slots)
      if (s && s->in_wide) S->multi.push_back(s);
  for (int f = 0; f < 2; ++f) {
    if (fam[f] != 1) S->direct[f] = nullptr;
    S->direct_rows[f] = false;
    if (const Shot* s = S->direct[f])  // as fd_forward_run samples a lone grid
      S->direct_rows[f] = s->plane_k >= 0 &&
                          (f == 1 || point_kernel_pays(s->geo) || receiver_plane_pays(s->geo));
  }
  for (const Shot* s : S->slots)
    if (s && s != S->direct[s->in_wide ? 1 : 0] && !(s->in_wide && !S->multi.empty())) {
      const int f = s->in_wide ? 1 : 0;
      xy[f].push_back((long long)((s->d.nx + tws[f][0] - 1) / tws[f][0]) *
                      ((s->d.ny + tws[f][1] - 1) / tws[f][1]));
      nzs[f].push_back(s->d.nz);
      least[f] += xy[f].back();
    }
  // the 16-byte-lane family first, leaving the other at least one chunk per grid
  long long budget = kTileCap - least[0];
  for (int f = 1; f >= 0; --f) {
    if (xy[f].empty()) continue;
    kc[f] = choose_kchunk(xy[f].data(), nzs[f].data(), (int)xy[f].size(), wpb[f], 0, budget);
    long long used = 0;
    for (size_t i = 0; i < xy[f].size(); ++i) used += xy[f][i] * ((nzs[f][i] + kc[f] - 1) / kc[f]);
    budget = kTileCap - used;
  }
  int nt = 0;
  for (int f = 0; f < 2; ++f) {
    for (int slot = 0; slot < S->max_slots; ++slot) {
      Shot* s = S->slots[slot];
      if (!s || (int)s->in_wide != f) continue;
      // rows left to the batched receiver launch: those of shots whose step does not
      // write them (receivers not on one plane, or a lone small grid whose direct
      // launch leaves them out)
      const bool in_kernel = s == S->direct[f] ? S->direct_rows[f]
                                               : S->shots_host[slot].rmap != nullptr;
      if (s->d.nrec > 0 && !in_kernel) {
        h_slots[na++] = slot;
        mr = std::max(mr, s->d.nrec);
      }
      if (s == S->direct[f] || (f == 1 && !S->multi.empty())) continue;
      const int bxn = (s->d.nx + tws[f][0] - 1) / tws[f][0];
      const int byn = (s->d.ny + tws[f][1] - 1) / tws[f][1];
      const int bzn = (s->d.nz + kc[f] - 1) / kc[f];
      S->h_shots[st][slot].kchunk = kc[f];
      for (int bz = 0; bz < bzn; ++bz)
        for (int by = 0; by < byn; ++by)
          for (int bx = 0; bx < bxn; ++bx) {
            if (nt >= kTileCap) return hipErrorInvalidValue;  // (the budget above prevents it)
            h_tiles[nt++] = make_int4(slot, bx, by, bz);
          }
    }
    counts[f] = nt - (f ? counts[0] : 0);
  }
  S->ntiles = counts[0];
  S->ntiles4 = counts[1];
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

// One step of a lone shot of its family by the single-grid launch (as fd_forward_run
// steps it: the one-thread-per-point kernel on small grids, the marching kernels
// above; with `rows` the receiver row is written by the same launch).
hipError_t step_direct(Server* S, Shot* s, bool rows) {
  const int n = s->n;
  float* arr[3];
  for (int i = 0; i < 3; ++i) arr[i] = shot_vol(S, s, i);
  const float* q = shot_vol(S, s, 3);
  const float* sp = reinterpret_cast<const float*>(shot_at(S, s, s->L.sponge));
  const float* ex = sp;
  const float* ey = sp + s->d.nx;
  const float* ez = sp + s->d.nx + s->d.ny;
  const fd_source src{s->d.src[0], s->d.src[1], s->d.src[2], s->w[n]};
  RecPlane rp{nullptr, -1, nullptr};
  if (rows) {
    rp.map = reinterpret_cast<const int32_t*>(shot_at(S, s, s->L.rmap));
    rp.k = s->plane_k;
    rp.row = reinterpret_cast<float*>(shot_at(S, s, s->L.traces)) + (size_t)n * s->d.nrec;
  }
  const float* up = arr[(n + 2) % 3];
  const float* u = arr[n % 3];
  float* un = arr[(n + 1) % 3];
  if (s->in_wide)
    return launch_forward_wide(s->geo, s->coef, up, u, un, q, ex, ey, ez, &src, nullptr, nullptr,
                               S->cs, rows ? &rp : nullptr);
  if (point_kernel_pays(s->geo))
    return launch_step_point(s->geo, s->coef, up, u, un, q, ex, ey, ez, &src, rows ? &rp : nullptr,
                             S->cs);
  return launch_step(s->geo, s->coef, up, u, un, q, ex, ey, ez, &src, S->cs, rows ? &rp : nullptr);
}

// One step of the 16-byte-lane family's shots in one launch, their parameters in the
// kernel arguments.
hipError_t step_multi(Server* S) {
  WideStep w[kWideMulti];
  int n = 0;
  for (Shot* s : S->multi) {
    const int k = s->n;
    float* arr[3];
    for (int i = 0; i < 3; ++i) arr[i] = shot_vol(S, s, i);
    const float* sp = reinterpret_cast<const float*>(shot_at(S, s, s->L.sponge));
    WideStep& x = w[n++];
    x.g = s->geo;
    x.c = s->coef;
    x.up = arr[(k + 2) % 3];
    x.u = arr[k % 3];
    x.un = arr[(k + 1) % 3];
    x.q = shot_vol(S, s, 3);
    x.ex = sp;
    x.ey = sp + s->d.nx;
    x.ez = sp + s->d.nx + s->d.ny;
    x.src = fd_source{s->d.src[0], s->d.src[1], s->d.src[2], s->w[k]};
    if (s->plane_k >= 0)
      x.rec = RecPlane{reinterpret_cast<const int32_t*>(shot_at(S, s, s->L.rmap)), s->plane_k,
                       reinterpret_cast<float*>(shot_at(S, s, s->L.traces)) +
                           (size_t)k * s->d.nrec};
  }
  return launch_wide_multi(w, n, S->cs);
}

// Release a shot's block and admission resources (nothing of the shot's may still
// run: its admission event was seen or its stream synchronised, and no queued step
// uses it).
void drop_prepared(Server* S, Shot* s) {
  if (s->has_block) S->arena->release(s->off, s->L.total);
  s->has_block = false;
  give_pinned(S, s->stage, s->stage_cap);
  s->stage = nullptr;
  drop_events(s);
}

void progress(Server* S) {
  const hipError_t dev = hipSetDevice(S->device);
  std::unique_lock<std::mutex> lk(S->mu);
  // without its device the thread can run nothing: every shot fails with FD_EDEVICE
  int fatal = dev == hipSuccess ? FD_OK : check_hip(dev, "server thread: hipSetDevice");
  while (!S->stopping) {
    bool busy = false;  // admission work in flight: poll again soon
    // ---- stage: reserve blocks and start admission work, in FIFO order
    while (!S->queue.empty() && fatal == FD_OK && (int)S->prep.size() < kPrepareAhead) {
      Shot* s = S->queue.front();
      size_t off;
      if (!S->arena->alloc(s->L.total, &off)) break;
      S->queue.pop_front();
      S->queued--;  // counted again below while it waits for a slot
      s->off = off;
      s->has_block = true;
      S->prep.push_back(s);
      s->stage = take_pinned(S, stage_floats(s->d), &s->stage_cap);
      lk.unlock();
      int rc = FD_OK;
      if (!s->stage) rc = fail(FD_ENOMEM, "shot: pinned staging allocation failed");
      hipError_t e = hipSuccess;
      bool whole = false;
      if (rc == FD_OK) e = hipEventCreateWithFlags(&s->ev, hipEventDisableTiming);
      if (rc == FD_OK && e == hipSuccess && !S->pool->acquire(&s->as))
        e = hipErrorOutOfMemory;
      if (rc == FD_OK && e == hipSuccess) e = admit_start(S, s, &whole);
      if (rc == FD_OK && e != hipSuccess) rc = check_hip(e, "shot admission");
      if (rc != FD_OK && s->as) (void)hipStreamSynchronize(s->as);
      lk.lock();
      S->queued++;
      s->state = whole ? State::Issued : State::Staging;
      s->check_pending = true;
      if (rc != FD_OK) {
        S->prep.pop_back();
        S->queued--;
        drop_prepared(S, s);
        finish_locked(S, s, rc);
        if (rc == FD_EDEVICE) fatal = rc;
      }
    }
    // ---- admission work that has finished
    for (size_t i = 0; i < S->prep.size();) {
      Shot* s = S->prep[i];
      if (s->state != State::Staging && s->state != State::Issued) { ++i; continue; }
      const hipError_t q = hipEventQuery(s->ev);
      if (q == hipErrorNotReady) { busy = true; ++i; continue; }
      int rc = q == hipSuccess ? FD_OK : check_hip(q, "shot admission");
      if (rc == FD_OK && s->check_pending) {
        rc = check_vmax(s);
        s->check_pending = false;
      }
      if (rc == FD_OK && s->state == State::Staging) {  // the model needs the maximum
        float vmax;
        memcpy(&vmax, &s->stage[0], 4);
        lk.unlock();
        const hipError_t e = admit_model(S, s, (double)vmax, s->ev);
        lk.lock();
        if (e == hipSuccess) {
          s->state = State::Issued;
          busy = true;
          ++i;
          continue;
        }
        rc = check_hip(e, "shot admission");
        (void)hipStreamSynchronize(s->as);  // nothing of the shot's may still run
      }
      if (rc == FD_OK) {  // all admission work has landed
        s->state = State::Staged;
        give_pinned(S, s->stage, s->stage_cap);
        s->stage = nullptr;
        drop_events(s);
        ++i;
        continue;
      }
      S->prep.erase(S->prep.begin() + i);
      S->queued--;
      drop_prepared(S, s);
      s->t_admit = now_ns();
      finish_locked(S, s, rc);
      if (rc == FD_EDEVICE) fatal = rc;
      S->cv.notify_all();
    }
    // ---- active shots whose admission work was still running when they joined
    for (int slot = 0; slot < S->max_slots; ++slot) {
      Shot* s = S->slots[slot];
      if (!s || !s->ev) continue;
      const hipError_t q = hipEventQuery(s->ev);
      if (q == hipErrorNotReady) continue;
      int rc = q == hipSuccess ? FD_OK : check_hip(q, "shot admission");
      if (rc == FD_OK && s->check_pending) rc = check_vmax(s);
      s->check_pending = false;
      give_pinned(S, s->stage, s->stage_cap);
      s->stage = nullptr;
      drop_events(s);
      if (rc == FD_OK) continue;
      // unstable (or failed): leave the step; its block is released once the steps
      // already queued with it have run
      S->slots[slot] = nullptr;
      S->table_dirty = true;
      s->abort_code = rc;
      s->state = State::Draining;
      hipError_t r = hipEventCreateWithFlags(&s->copied, hipEventDisableTiming);
      if (r == hipSuccess) r = hipEventRecord(s->copied, S->cs);
      if (r != hipSuccess) {
        (void)hipStreamSynchronize(S->cs);
        if (s->copied) (void)hipEventDestroy(s->copied);
        s->copied = nullptr;
        S->arena->release(s->off, s->L.total);
        s->has_block = false;
        S->running--;
        finish_locked(S, s, rc);
        continue;
      }
      S->draining.push_back(s);
      if (rc == FD_EDEVICE) fatal = rc;
    }
    // ---- activate prepared shots (strict FIFO)
    while (!S->prep.empty() && fatal == FD_OK &&
           (S->prep.front()->state == State::Staged || S->prep.front()->state == State::Issued)) {
      Shot* s = S->prep.front();
      int slot = -1;
      for (int i = 0; i < S->max_slots; ++i)
        if (!S->slots[i]) { slot = i; break; }
      if (slot < 0) break;
      if (tiles_in_use(S) + s->L.tiles > kTileCap) break;
      if (!activation_pays(S, s)) break;
      size_t cap = 0;
      s->host_cap = (size_t)s->d.nt * (size_t)s->d.nrec;
      s->host = take_pinned(S, s->host_cap, &cap);
      if (!s->host) break;  // retried on the next pass
      // admission work still running: the compute stream waits for the model's part
      // of it (the stability check may land later), not the host
      if (s->ev && hipStreamWaitEvent(S->cs, s->mev ? s->mev : s->ev, 0) != hipSuccess) {
        give_pinned(S, s->host, cap);
        s->host = nullptr;
        break;
      }
      S->prep.pop_front();
      S->queued--;
      s->t_admit = now_ns();
      s->host_cap = cap;
      s->slot = slot;
      S->slots[slot] = s;
      fill_slot(S, s, slot);
      s->state = State::Active;
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
      finish_locked(S, s, q != hipSuccess ? FD_EDEVICE : s->abort_code);
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
      // nothing to step: wait for the oldest admission phase in flight (the shot that
      // joins next), else for a copy, a submission or a short timeout
      hipEvent_t wait_ev = nullptr;
      for (Shot* s : S->prep)
        if (s->state == State::Staging || s->state == State::Issued) {
          wait_ev = s->ev;
          break;
        }
      if (wait_ev && fatal == FD_OK) {
        lk.unlock();
        (void)hipEventSynchronize(wait_ev);
        lk.lock();
      } else if (busy || !S->draining.empty()) {
        S->cv.wait_for(lk, std::chrono::microseconds(20));
      } else {
        S->cv.wait_for(lk, std::chrono::milliseconds(2));
      }
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
    for (int f = 0; f < 2 && e == hipSuccess; ++f) {
      if (Shot* s = S->direct[f]) {
        e = step_direct(S, s, S->direct_rows[f]);
      } else if (f == 0) {
        e = launch_batched(S->d_shots, S->d_tiles, S->ntiles, a, S->cs);
      } else if (!S->multi.empty()) {
        e = step_multi(S);
      } else {
        e = launch_batched4(S->d_shots, S->d_tiles + S->ntiles, S->ntiles4, a, S->cs);
      }
    }
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
      s->state = State::Draining;
      hipError_t r = hipEventCreateWithFlags(&s->copied, hipEventDisableTiming);
      hipEvent_t stepped = nullptr;
      if (r == hipSuccess) r = hipEventCreateWithFlags(&stepped, hipEventDisableTiming);
      if (r == hipSuccess) r = hipEventRecord(stepped, S->cs);
      if (r == hipSuccess) r = hipStreamWaitEvent(S->xs, stepped, 0);
      if (r == hipSuccess && s->d.nrec > 0)
        r = hipMemcpyAsync(s->host, shot_at(S, s, s->L.traces),
                           4 * (size_t)s->d.nt * (size_t)s->d.nrec, hipMemcpyDeviceToHost, S->xs);
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
  S->pool->sync_all();
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
  for (Shot* s : S->prep) {  // their admission streams were synchronised
    drop_prepared(S, s);
    S->queued--;
    finish_locked(S, s, FD_ECANCELED);
  }
  S->prep.clear();
  for (int slot = 0; slot < S->max_slots; ++slot)
    if (Shot* s = S->slots[slot]) {
      S->slots[slot] = nullptr;
      drop_prepared(S, s);  // the block, and admission resources still held
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
    finish_locked(S, s, landed ? s->abort_code : FD_EDEVICE);
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
                      align_up(sizeof(int4) * kTileCap) + align_up(sizeof(int) * MAX_BATCH_SLOTS);
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
  S->base = p;  // shot blocks live after the tables
  S->bytes = (arena_bytes - head) / kAlign * kAlign;
  S->arena.reset(new Arena(S->bytes));
  S->slots.assign(max_slots, nullptr);
  int rc = check_hip(hipGetDevice(&S->device), "fd_server_create");
  if (rc) return rc;
  S->pool.reset(new StreamPool<HipStreams>(HipStreams{}, kAdmitStreams));
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

int fd_server_set_allocator(void* srv, int32_t kind) {
  Server* S = static_cast<Server*>(srv);
  if (!S) return fail(FD_EINVAL, "fd_server_set_allocator: NULL server");
  if (kind != FD_ARENA_FIRST_FIT && kind != FD_ARENA_BUDDY)
    return fail(FD_EINVAL, "fd_server_set_allocator: kind %d is not FD_ARENA_FIRST_FIT or "
                           "FD_ARENA_BUDDY", kind);
  std::lock_guard<std::mutex> g(S->mu);
  if (S->submitted)
    return fail(FD_EINVAL, "fd_server_set_allocator: shots were submitted already");
  if (kind == FD_ARENA_BUDDY) S->arena.reset(new BuddyArena(S->bytes, kAlign));
  else S->arena.reset(new Arena(S->bytes));
  S->arena_kind = kind;
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
  s->d = *d;
  s->d.rec_ijk_host = nullptr;
  s->L = L;
  s->t_submit = now_ns();
  std::lock_guard<std::mutex> g(S->mu);
  // a buddy block is the footprint rounded up to a power of two times 256 bytes
  size_t need = L.total;
  if (S->arena_kind == FD_ARENA_BUDDY) {
    size_t b = kAlign;
    while (b < need) b <<= 1;
    need = b;
  }
  if (need > S->bytes || L.tiles > kTileCap)
    return fail(FD_ENOMEM, "shot_submit: footprint %zu bytes can never fit the arena (%zu)",
                need, S->bytes);
  if (S->stopping) return fail(FD_ECANCELED, "shot_submit: server is shut down");
  S->submitted = true;
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
    memcpy(traces_host, s->host,
           4 * std::min(cap, (size_t)s->d.nt * (size_t)std::max(s->d.nrec, 0)));
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
  for (auto& kv : S->shots) {
    give_pinned(S, kv.second->host, kv.second->host_cap);
    kv.second->host = nullptr;
    give_pinned(S, kv.second->stage, kv.second->stage_cap);
    kv.second->stage = nullptr;
  }
  for (auto& pb : S->pinned_pool) (void)hipHostFree(pb.second);
  for (int i = 0; i < 2; ++i) {
    if (S->h_shots[i]) (void)hipHostFree(S->h_shots[i]);
    if (S->h_tiles[i]) (void)hipHostFree(S->h_tiles[i]);
    if (S->h_slots[i]) (void)hipHostFree(S->h_slots[i]);
    if (S->table_ev[i]) (void)hipEventDestroy(S->table_ev[i]);
  }
  for (int i = 0; i < kInflight; ++i)
    if (S->step_ev[i]) (void)hipEventDestroy(S->step_ev[i]);
  S->pool.reset();  // synchronises and destroys the admission streams
  if (S->own_cs) (void)hipStreamDestroy(S->cs);
  if (S->own_xs) (void)hipStreamDestroy(S->xs);
  delete S;
  return FD_OK;
}

}  // extern "C"
