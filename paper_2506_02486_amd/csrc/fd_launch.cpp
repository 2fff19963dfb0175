// fd_launch.cpp -- launch shape of the z-marching stencil kernels (host only).
//
// A stencil block owns one x-y tile and marches through a chunk of kc z planes,
// so a launch over a grid has tiles_x * tiles_y * ceil(nz / kc) blocks.  The
// chunk trades blocks (bandwidth needs enough of them in flight, and a small
// last round of blocks runs nearly alone) against the z halo each chunk reads
// again.  choose_kchunk takes the chunk of least modelled time.
#include <algorithm>
#include <atomic>

#include "fd_internal.h"

namespace fd {
namespace {

std::atomic<int> g_kchunk_override{0};
std::atomic<int> g_tile_override{0};

// Up to about 100^3 points the 64 x 32 tile leaves CUs idle even with one-plane
// chunks (64^3: 128 blocks); 64 x 16 tiles double the blocks (64^3: 6.4 us per
// step against 7.2, 96^3: 10.4 against 11.1, 128^3 the same).
constexpr long long kSmallGridPoints = 1LL << 20;

// Relative time of a launch of B blocks that each stream kc planes (+1 for the
// z halo, which mostly hits L2), when R blocks fit on the chip at once.  Below one
// round the blocks cannot pull the full bandwidth; a little above it the second
// round runs nearly alone.  Fitted to stencil times of cubes 128..512 over z chunks
// of 4..128 planes; with the three wavefields rotating as in real stepping, its
// choice was the fastest of 17 chunks tried at every one of those sizes (e.g.
// 384^3: 576 blocks 235 us, 432 blocks 185 us, the chosen 504 blocks 175 us).
double launch_cost(long long B, int kc, long long R) {
  const double x = (double)B / (double)R;
  const double e = x <= 1.0 ? 0.55 + 0.3 * x : std::max(0.9 * x + 0.2, 1.4);
  return (kc + 1.0) * e;
}

}  // namespace

int choose_kchunk(const long long* xy, const int* nz, int n, int waves_per_block, int kc_max,
                  long long max_blocks) {
  // 4096 waves: 16 per CU on 256 CUs
  const long long R = std::max(1, 4096 / std::max(1, waves_per_block));
  int deep = 1;
  for (int i = 0; i < n; ++i) deep = std::max(deep, nz[i]);
  const int top = kc_max > 0 ? std::min(deep, kc_max) : deep;
  // candidates: the shortest chunk that cuts the deepest grid into z pieces, for
  // z = 1, 2, ... (exact for one grid: the time grows with kc at a fixed block
  // count); past eight rounds of blocks shorter chunks only add blocks and halo
  int best = top, prev = -1;
  double best_cost = -1.0;
  for (long long z = (deep + top - 1) / top;; ++z) {
    const int kc = (int)((deep + z - 1) / z);
    if (kc == prev) continue;
    prev = kc;
    long long B = 0;
    for (int i = 0; i < n; ++i) B += xy[i] * ((nz[i] + kc - 1) / kc);
    if (B > max_blocks) break;  // B only grows as kc shrinks
    const double c = launch_cost(B, kc, R);
    if (best_cost < 0.0 || c < best_cost) {  // ties go to the longer chunk
      best_cost = c;
      best = kc;
    }
    if (kc == 1 || B > 8 * R) break;
  }
  return best;
}

LaunchShape stencil_shape(const Geo& g, int tx, int ty, int waves_per_block) {
  LaunchShape s;
  s.tiles_x = (g.nx + tx - 1) / tx;
  s.tiles_y = (g.ny + ty - 1) / ty;
  const long long tiles = (long long)s.tiles_x * s.tiles_y;
  int kc = g_kchunk_override.load(std::memory_order_relaxed);
  if (kc <= 0) {
    // one full round of resident blocks where the x-y tiles allow it (512^3: 128
    // planes, 256^3: 16), several rounds otherwise, one plane for small grids whose
    // arrays sit in cache (64^3: 4.8 us per step at 1 plane, 8.0 at 4).  The last
    // choice is kept per thread.
    thread_local struct { int nx = -1, ny = -1, nz = -1, tx = -1, ty = -1, w = -1, kc = 0; } last;
    if (last.nx == g.nx && last.ny == g.ny && last.nz == g.nz && last.tx == tx && last.ty == ty &&
        last.w == waves_per_block) {
      kc = last.kc;
    } else {
      kc = choose_kchunk(&tiles, &g.nz, 1, waves_per_block, 0, 0x7fffffffLL);
      last = {g.nx, g.ny, g.nz, tx, ty, waves_per_block, kc};
    }
  }
  if (kc > g.nz) kc = std::max(1, g.nz);
  s.kchunk = kc;
  s.zchunks = (g.nz + kc - 1) / kc;
  return s;
}

void set_kchunk_override(int kc) { g_kchunk_override.store(kc, std::memory_order_relaxed); }

double stencil_cost(const Geo& g, int tx, int ty, int waves_per_block) {
  const LaunchShape s = stencil_shape(g, tx, ty, waves_per_block);
  const long long R = std::max(1, 4096 / std::max(1, waves_per_block));
  return launch_cost((long long)s.tiles_x * s.tiles_y * s.zchunks, s.kchunk, R);
}

int tile_override() { return g_tile_override.load(std::memory_order_relaxed); }

bool forward_small_tiles(const Geo& g) {
  const int mode = g_tile_override.load(std::memory_order_relaxed);
  if (mode == 1 || mode == 4 || mode == 5) return false;
  if (mode == 2 || mode == 3) return true;
  return (long long)g.nx * g.ny * g.nz <= kSmallGridPoints;
}

void set_tile_override(int mode) { g_tile_override.store(mode, std::memory_order_relaxed); }

// From about this size on the 16-byte-lane kernel's wider loads, more of them in
// flight, pay (native loop, sponge 16, us per step, 64 x 32 marching kernel / one
// thread per point / 16-byte lanes: 192^3 29.6 / 29.5 / 32.4, 200^3 40.7 / 41.9 /
// 35.5, 256^3 56.4 / 89.1 / 49.8, 384^3 179.0 / 310.3 / 167.2).
constexpr long long kWideGridPoints = 7500000;

bool forward_wide_tiles(const Geo& g) {
  const int mode = g_tile_override.load(std::memory_order_relaxed);
  if (mode == 4 || mode == 5) return true;
  if (mode != 0) return false;
  return (long long)g.nx * g.ny * g.nz >= kWideGridPoints;
}

// Grids small enough to sit in cache run their forward step latency-bound; up to
// about this size the one-thread-per-point kernel finishes first (native loop, 200
// steps, us per step, marching against point: 64^3 4.52 / 3.51, with a sponge 5.16
// / 3.72, 96^3 9.58 / 6.91, 128^3 13.4 / 12.1, 160^3 22.8 / 21.6, 176^3 27.8 /
// 27.6, 192^3 29.4 / 30.0, 256^3 56.1 / 91.6).
constexpr long long kPointGridPoints = 1LL << 22;

bool point_kernel_pays(const Geo& g) {
  const int mode = g_tile_override.load(std::memory_order_relaxed);
  if (mode == 3) return true;
  if (mode == 1 || mode == 2 || mode == 4 || mode == 5) return false;
  return (long long)g.nx * g.ny * g.nz <= kPointGridPoints;
}

// The exchange step (six faces read and written in the same launch) pays off on
// smaller grids only: loopback, sponge 8, x-line receivers, native loop, us per
// step, point against the marching kernel with its pack and unpack launches: 64^3
// 4.96 / 9.74, 96^3 10.5 / 15.1, 128^3 15.5 / 16.7, 160^3 30.1 / 27.3.
constexpr long long kPointExchangePoints = 1LL << 21;

bool point_exchange_pays(const Geo& g) {
  const int mode = g_tile_override.load(std::memory_order_relaxed);
  if (mode == 3) return true;
  if (mode == 1 || mode == 2 || mode == 4 || mode == 5) return false;
  return (long long)g.nx * g.ny * g.nz <= kPointExchangePoints;
}

// The receiver row taken by the stencil launch saves a launch per step but adds a
// dependent map lookup to the blocks of the receiver plane, whose finish sets the
// launch time: a gain where launches dominate (64^3: 6.4 -> 4.7 us per step), a loss
// on bandwidth-bound grids (256^3: +6 us per launch against a 4.8 us receiver launch).
bool receiver_plane_pays(const Geo& g) {
  return (long long)g.nx * g.ny * g.nz <= kSmallGridPoints;
}

}  // namespace fd
