// fd_internal.h -- declarations shared by the host ABI layer and the HIP
// kernel files of libfd (not installed, not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fd.h"

namespace fd {

// In-plane byte offsets are 32-bit unsigned in the stencil kernels.
constexpr long long FD_MAX_ZSTRIDE = (1LL << 29);

// Thread-local error detail; returns `code` so callers can `return fail(...)`.
int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
// Map a HIP error to FD_EDEVICE with detail, or FD_OK.
int check_hip(hipError_t e, const char* what);

// Geometry in the form the kernels take (by value).
struct Geo {
  int nx, ny, nz;
  int sy;          // ystride (elements)
  int sz;          // zstride (elements), <= FD_MAX_ZSTRIDE
  long long org;   // origin (elements)
};

inline Geo make_geo(const fd_grid* g) {
  Geo q;
  q.nx = g->nx;
  q.ny = g->ny;
  q.nz = g->nz;
  q.sy = (int)g->ystride;
  q.sz = (int)g->zstride;
  q.org = g->origin;
  return q;
}

// Stencil weights divided by the squared spacing, rounded to FP32 from FP64:
// cx[m], cy[m], cz[m] for m = 1..4 (index 0 unused) and the merged centre weight.
struct Coef {
  float cx[5], cy[5], cz[5];
  float cc;
};
Coef make_coef(const fd_grid* g);

// One shot of a batched launch (device memory, written by the shot server).
struct BatchShot {
  Geo g;
  Coef c;
  float* arr[3];        // wavefields; u^n lives in arr[n % 3]
  const float* q;       // vdt2
  const float* ex;      // sponge tables (all zeros when the shot has none)
  const float* ey;
  const float* ez;
  int si, sj, sk;       // source point
  int kchunk;           // z planes per tile-table entry
  const int64_t* rec;   // receiver offsets
  float* traces;        // nt x nrec
  int nrec;
  int rk;               // receiver plane of rmap
  const int32_t* rmap;  // receivers on one plane: [ny][nx] receiver index or -1; the
                        // batched kernel writes their rows (NULL: batched_record does)
};

constexpr int MAX_BATCH_SLOTS = 64;

// Per-step arguments of a batched launch (by value).
struct BatchStep {
  int n[MAX_BATCH_SLOTS];    // steps done so far by the shot in each slot
  float w[MAX_BATCH_SLOTS];  // its source amplitude for this step
};

// Receivers that all lie on one z plane k: map[j * nx + i] is the index of the
// receiver at (i, j, k) or -1 (device, nx * ny), row the trace row they fill.
struct RecPlane {
  const int32_t* map;
  int k;
  float* row;
  bool add = false;  // row is added at the points, scaled by vdt2 / (1+eta) (adjoint)
};

// ------------------------------------------------------------ launchers
// All validate nothing (the ABI layer has) and return a HIP error code.
// src may be NULL (no fused source term); rp (optional) has the forward kernel
// write the receiver row of un itself (or, with rp->add, add that row to un)
hipError_t launch_step(const Geo& g, const Coef& c, const float* up, const float* u,
                       float* un, const float* q, const float* ex, const float* ey,
                       const float* ez, const fd_source* src, hipStream_t s,
                       const RecPlane* rp = nullptr);
// The same forward step by the one-thread-per-point kernel (small grids; same
// bits); rp as for launch_step (rp->add not in the exchange form).  With rin and
// sout (all twelve non-NULL; every axis at least 4 long) the whole exchange step:
// u's halos read from rin, the faces of un written to sout (halo_unpack /
// halo_pack layouts).
hipError_t launch_step_point(const Geo& g, const Coef& c, const float* up, const float* u,
                             float* un, const float* q, const float* ex, const float* ey,
                             const float* ez, const fd_source* src, const RecPlane* rp,
                             hipStream_t s, const float* const rin[6] = nullptr,
                             float* const sout[6] = nullptr);
// Whether forward steps over g without faces in the kernel take the point kernel:
// grids of at most kPointGridPoints points, or as forced by set_tile_override
// (3: always, 1 or 2: never).
bool point_kernel_pays(const Geo& g);
// The same for the exchange step with all six faces in the launch (at most
// kPointExchangePoints points, or as forced).
bool point_exchange_pays(const Geo& g);
// Planes per block (z chunk) for one launch over n grids, grid i with xy[i] x-y
// tiles and nz[i] planes, with the least modelled time; at most kc_max planes
// (0: no limit) and at most max_blocks blocks (the longest chunk is the fallback).
int choose_kchunk(const long long* xy, const int* nz, int n, int waves_per_block, int kc_max,
                  long long max_blocks);
struct LaunchShape {
  int tiles_x, tiles_y, kchunk, zchunks;
};
// Blocks of a stencil kernel with tx x ty tiles over g: the z chunk set by
// set_kchunk_override (> 0), else choose_kchunk's.
LaunchShape stencil_shape(const Geo& g, int tx, int ty, int waves_per_block);
// Process-wide z chunk for every stencil launch (0: automatic).
void set_kchunk_override(int kc);
// Modelled time (arbitrary units) of the launch stencil_shape picks for tx x ty
// tiles over g.
double stencil_cost(const Geo& g, int tx, int ty, int waves_per_block);
// The process-wide tile mode of set_tile_override.
int tile_override();
// Whether the 16-byte-lane forward update and gradient pass over g (not the
// exchange form) take 64 x 64 tiles instead of 128 x 32 (tile mode 5: always; 4:
// never; else where the launch model prefers them by a tenth).
bool wide_narrow_tiles(const Geo& g);
// Whether g's tiles in a launch shared with other grids (launch_wide_multi) are
// 64 x 64 (modes 5 and 4 as above; else where they cover the plane with a tenth
// fewer points than 128 x 32).
bool wide_narrow_in_multi(const Geo& g);
// Forward launches over g use 64 x 16 tiles instead of 64 x 32: small grids (at
// most kSmallGridPoints interior points), or as forced by set_tile_override
// (0: automatic, 1: always 64 x 32, 2: always 64 x 16).
bool forward_small_tiles(const Geo& g);
void set_tile_override(int mode);
// Forward updates (and gradient passes) over g take the 16-byte-lane
// kernel of fd_stencil4.hip: bandwidth-bound grids (more than kWideGridPoints
// interior points), or as forced by set_tile_override (4, 5: wherever it fits; 1,
// 2, 3: never).
bool forward_wide_tiles(const Geo& g);
// Whether the 16-byte-lane kernel can take a step over g: rows, strides and origin
// multiples of 4 floats, the four volume arrays (u_prev, u, u_next, vdt2) 16-byte
// aligned; with faces (-x in, +x in, -x out, +x out; NULL: no exchange) nx a multiple
// of its tile width and the four buffers 16-byte aligned.
bool wide_forward_fits(const Geo& g, const float* const arrays[4], const float* const faces[4]);
// tiles_x, tiles_y, kchunk, zchunks of the 16-byte-lane kernel's launch over g
void wide_forward_shape(const Geo& g, int out[4]);
// The forward step (launch_step, or with rin/sout launch_step_exchange) by the
// 16-byte-lane kernel; same bits.  rp (optional): the kernel writes the receiver
// row of un itself, or with rp->add adds the row scaled by vdt2 / (1+eta), as
// launch_step does.
hipError_t launch_forward_wide(const Geo& g, const Coef& c, const float* up, const float* u,
                               float* un, const float* q, const float* ex, const float* ey,
                               const float* ez, const fd_source* src, const float* const rin[2],
                               float* const sout[2], hipStream_t s,
                               const RecPlane* rp = nullptr);
// Whether launch_step over g with these arrays (u_prev, u, u_next, vdt2) takes the
// 16-byte-lane kernel.
bool wide_takes_step(const Geo& g, const float* const arrays[4]);
// launch_grad by the 16-byte-lane kernel (same bits); gq is read and written in
// place.  The caller checks wide_forward_fits for {an1, u, gq, gq}.
hipError_t launch_grad_wide(const Geo& g, const Coef& c, const float* u, const float* an1,
                            float* gq, const float* ex, const float* ey, const float* ez,
                            const fd_source* src, hipStream_t s);
// Whether a z-marching step over g takes its receiver row in the stencil launch
// (small grids, whose launches are short) rather than in a launch of its own.
bool receiver_plane_pays(const Geo& g);
// tiles_x, tiles_y, kchunk, zchunks of the forward stencil launch over g
void forward_launch_shape(const Geo& g, int out[4]);
// Tile size (x, y) of the batched kernel; returns threads per block.
int batch_tile_shape(int* tx, int* ty);
// Tile size (x, y) of the batched kernel of 16-byte lanes; returns the waves of a
// CU's residency one block takes (for choose_kchunk).
int batch4_tile_shape(int* tx, int* ty);
// One step of up to kWideMulti grids in one launch of the 16-byte-lane kernel, their
// parameters passed in the kernel arguments (each grid as fd_step_fused with its source
// term steps it; same bits; one z chunk for all from the launch model).
constexpr int kWideMulti = 8;
struct WideStep {
  Geo g;
  Coef c;
  const float* up;
  const float* u;
  float* un;
  const float* q;
  const float* ex;
  const float* ey;
  const float* ez;
  fd_source src;
  RecPlane rec{nullptr, -1, nullptr};  // receiver row written by the launch (map NULL: none)
};
hipError_t launch_wide_multi(const WideStep* steps, int n, hipStream_t s);
// One time step of every shot listed in the tile table, by the 16-byte-lane kernel
// (same bits as the other kernels; no receiver row in the kernel).
hipError_t launch_batched4(const BatchShot* shots, const int4* tiles, int ntiles,
                           const BatchStep& a, hipStream_t s);
// One time step of every shot listed in the tile table (entries: slot, bx, by, bz).
hipError_t launch_batched(const BatchShot* shots, const int4* tiles, int ntiles,
                          const BatchStep& a, hipStream_t s);
// trace[n][r] = u^{n+1}[rec[r]] for every active slot (slots[i], i < nslots).
hipError_t launch_batched_record(const BatchShot* shots, const int* slots, int nslots,
                                 int max_nrec, const BatchStep& a, hipStream_t s);
// vdt2 = (v dt)^2 on the padded box of g from a strided velocity view (element
// (i,j,k) at v[k*vsz + j*vsy + i], interior only read); faces wrap, edges 0.
hipError_t launch_prepare_vdt2_view(const Geo& g, const float* v, long long vsy, long long vsz,
                                    float* q, double dt, hipStream_t s);
// max and min of a strided velocity view's interior into out[0], out[1] (float bits)
hipError_t launch_vmax_view(int nx, int ny, int nz, const float* v, long long vsy,
                            long long vsz, int32_t* out, hipStream_t s);
// dst[i] = 0 for i < n
hipError_t launch_zero(float* dst, long long n, hipStream_t s);
// Device address of the calling thread's current device's copy of the library's
// static max(v) result slots (kCflScratchInts int32, of which launch_vmax uses 2);
// looked up once per device.
constexpr int kCflScratchInts = 64;
hipError_t cfl_scratch(int32_t** out);

// The forward step with the x faces exchanged inside the stencil kernel: u's
// x-face halos are read from rin[0] (-x) and rin[1] (+x) (halo_unpack layout
// [nz][ny][4]), the x faces of un are written to sout[0], sout[1] (halo_pack
// layout), the source is added when src is given.  All four buffers non-NULL;
// only where exchange_fits (nx a multiple of the tile width).
bool exchange_fits(const Geo& g);
hipError_t launch_step_exchange(const Geo& g, const Coef& c, const float* up, const float* u,
                                float* un, const float* q, const float* ex, const float* ey,
                                const float* ez, const fd_source* src, const float* const rin[2],
                                float* const sout[2], hipStream_t s);
hipError_t launch_adjoint(const Geo& g, const Coef& c, const float* ann, const float* an1,
                          float* aout, const float* q, const float* ex, const float* ey,
                          const float* ez, hipStream_t s);
hipError_t launch_grad(const Geo& g, const Coef& c, const float* u, const float* an1,
                       float* gq, const float* ex, const float* ey, const float* ez,
                       const fd_source* src, hipStream_t s);
hipError_t launch_inject(const Geo& g, float* un, const float* q, const float* ex,
                         const float* ey, const float* ez, int i, int j, int k, float w,
                         hipStream_t s);
hipError_t launch_record(const float* u, const int64_t* off, int n, float* out,
                         hipStream_t s);
hipError_t launch_scatter_add(float* a, const int64_t* off, const float* vals, int n,
                              hipStream_t s);
hipError_t launch_pack(const Geo& g, const float* u, float* const face[6], hipStream_t s);
// launch_pack and launch_record(u, off, n, out) in one launch where the faces
// take the 16-byte form, else the two launches
hipError_t launch_pack_record(const Geo& g, const float* u, float* const face[6],
                              const int64_t* off, int n, float* out, hipStream_t s);
hipError_t launch_unpack(const Geo& g, float* u, const float* const face[6], hipStream_t s);
// from_m: the input is squared slowness m and vdt2 = dt^2/m; else velocity v and
// vdt2 = (v dt)^2
hipError_t launch_prepare_vdt2(const Geo& g, const float* v, float* q, double dt, bool from_m,
                               hipStream_t s);
hipError_t launch_vmax(const Geo& g, const float* v, int32_t* out, hipStream_t s);
// scaled: gq accumulates b (L u + f) with b = Q D lambda (grad_m = -gq Q / dt^2);
// else gq = g_vdt2 (grad_m = -gq Q^2 / dt^2)
hipError_t launch_grad_finalize(const Geo& g, const float* gq, const float* q, double dt,
                                bool scaled, float* gm, hipStream_t s);
// a[off[r]] += vals[r] * q / (1 + eta) at each (interior) offset
hipError_t launch_scatter_add_scaled(const Geo& g, float* a, const int64_t* off,
                                     const float* vals, const float* q, const float* ex,
                                     const float* ey, const float* ez, int n, hipStream_t s);

}  // namespace fd
