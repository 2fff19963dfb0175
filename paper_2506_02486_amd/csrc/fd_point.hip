// fd_point.hip -- the forward update of small grids, one thread per point.
//
// A grid of up to about a million points sits in the L2 and MALL caches between
// steps, so its step is bound by latency, not bandwidth: the z-marching kernel's
// blocks spend most of their life filling the nine-plane register queue of a short
// chunk.  Here every thread reads its 25 stencil values directly (cache hits after
// the first step) and writes its point, so the whole grid is in flight at once.
// The arithmetic is that of the marching kernel, term for term and in the same
// order (centre, x pairs, y pairs, z pairs; the damped form only where eta != 0;
// the source and receiver epilogues), so both give the same bits.
#include "fd_internal.h"

namespace fd {
namespace {

constexpr int PX = 64, PY = 4;

template <bool SPONGE, bool REC>
__global__ void __launch_bounds__(PX * PY)
    point_kernel(Geo g, Coef c, const float* up, const float* __restrict__ u, float* un,
                 const float* __restrict__ q, const float* __restrict__ ex,
                 const float* __restrict__ ey, const float* __restrict__ ez, int si, int sj, int sk,
                 float sw, const int32_t* __restrict__ rmap, int rk, float* __restrict__ rrow) {
  // up and un may be one array (two-array stepping): each thread reads its point of
  // up before it writes the same point of un, and touches no other point of either
  const int x = blockIdx.x * PX + threadIdx.x;
  const int y = blockIdx.y * PY + threadIdx.y;
  const int k = blockIdx.z;
  if (x >= g.nx || y >= g.ny) return;
  const long long o = g.org + (long long)k * g.sz + (long long)y * g.sy + x;
  const float* c0 = u + o;
  const float uc = c0[0];
  float lap = c.cc * uc;
#pragma unroll
  for (int m = 1; m <= 4; ++m) lap += c.cx[m] * (c0[m] + c0[-m]);
#pragma unroll
  for (int m = 1; m <= 4; ++m) lap += c.cy[m] * (c0[(long long)m * g.sy] + c0[-(long long)m * g.sy]);
#pragma unroll
  for (int m = 1; m <= 4; ++m) lap += c.cz[m] * (c0[(long long)m * g.sz] + c0[-(long long)m * g.sz]);
  const float pa = up[o], pb = q[o];
  float eta = 0.f;
  if (SPONGE) eta = ex[x] + ey[y] + ez[k];
  float v = 2.f * uc - pa + pb * lap;
  if (SPONGE && eta != 0.f) v = (v + eta * pa) * __builtin_amdgcn_rcpf(1.f + eta);
  if (k == sk && x == si && y == sj) {
    // rounds as inject_source: no contraction
#pragma clang fp contract(off)
    v += pb * sw / (1.f + eta);
  }
  un[o] = v;  // a plain store: the next step reads it from cache
  if (REC && k == rk) {
    const int rr = rmap[y * g.nx + x];
    if (rr >= 0) rrow[rr] = v;
  }
}

}  // namespace

hipError_t launch_step_point(const Geo& g, const Coef& c, const float* up, const float* u,
                             float* un, const float* q, const float* ex, const float* ey,
                             const float* ez, const fd_source* src, const RecPlane* rp,
                             hipStream_t s) {
  if (rp && rp->map && rp->add) return hipErrorInvalidValue;  // the forward step only records
  const dim3 grid((unsigned)((g.nx + PX - 1) / PX), (unsigned)((g.ny + PY - 1) / PY),
                  (unsigned)g.nz);
  const int si = src ? src->i : -1, sj = src ? src->j : -1, sk = src ? src->k : -1;
  const float sw = src ? src->w : 0.f;
  const bool rec = rp && rp->map;
  const int32_t* map = rec ? rp->map : nullptr;
  const int rk = rec ? rp->k : -1;
  float* row = rec ? rp->row : nullptr;
  if (ex && rec)
    hipLaunchKernelGGL((point_kernel<true, true>), grid, dim3(PX, PY), 0, s, g, c, up, u, un, q,
                       ex, ey, ez, si, sj, sk, sw, map, rk, row);
  else if (ex)
    hipLaunchKernelGGL((point_kernel<true, false>), grid, dim3(PX, PY), 0, s, g, c, up, u, un, q,
                       ex, ey, ez, si, sj, sk, sw, map, rk, row);
  else if (rec)
    hipLaunchKernelGGL((point_kernel<false, true>), grid, dim3(PX, PY), 0, s, g, c, up, u, un, q,
                       ex, ey, ez, si, sj, sk, sw, map, rk, row);
  else
    hipLaunchKernelGGL((point_kernel<false, false>), grid, dim3(PX, PY), 0, s, g, c, up, u, un,
                       q, ex, ey, ez, si, sj, sk, sw, map, rk, row);
  return hipGetLastError();
}

}  // namespace fd
