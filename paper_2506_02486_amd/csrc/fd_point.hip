// fd_point.hip -- the forward update of small grids, one thread per point.
//
// A grid of up to a few million points (the limits are in fd_launch.cpp) sits in
// the L2 and MALL caches between steps, so its step is bound by latency rather than
// bandwidth: the z-marching kernel's
// blocks spend most of their life filling the nine-plane register queue of a short
// chunk.  Here every thread reads its 25 stencil values directly (cache hits after
// the first step) and writes its point, so the whole grid is in flight at once.
// The arithmetic is that of the marching kernel, term for term and in the same
// order (centre, x pairs, y pairs, z pairs; the damped form only where eta != 0;
// the source and receiver epilogues), so both give the same bits.
// Exchange form (XCH): a neighbour outside the interior is read from the receive
// buffer of its face instead of u's halo, and a point within 4 of a face is also
// written to that face's send buffer (halo_unpack / halo_pack layouts), so the
// whole exchange step is this one launch.
#include "fd_internal.h"

namespace fd {
namespace {

constexpr int PX = 64, PY = 4;

struct PFaces {
  const float* in[6];
  float* out[6];
};

// REC: 1 writes the receiver row of plane rk, 2 adds the row scaled by
// vdt2 / (1+eta) there (the scaled adjoint's residual), as the marching kernel does
template <bool SPONGE, int REC, bool XCH>
__global__ void __launch_bounds__(PX * PY)
    point_kernel(Geo g, Coef c, const float* up, const float* __restrict__ u, float* un,
                 const float* __restrict__ q, const float* __restrict__ ex,
                 const float* __restrict__ ey, const float* __restrict__ ez, int si, int sj, int sk,
                 float sw, const int32_t* __restrict__ rmap, int rk, float* __restrict__ rrow,
                 PFaces fc) {
  // up and un may be one array (two-array stepping): each thread reads its point of
  // up before it writes the same point of un, and touches no other point of either
  const int x = blockIdx.x * PX + threadIdx.x;
  const int y = blockIdx.y * PY + threadIdx.y;
  const int k = blockIdx.z;
  if (x >= g.nx || y >= g.ny) return;
  const long long o = g.org + (long long)k * g.sz + (long long)y * g.sy + x;
  const float* c0 = u + o;
  const unsigned nx = (unsigned)g.nx, ny = (unsigned)g.ny, nz = (unsigned)g.nz;
  // neighbour at x + d (y + d, k + d): u itself, or in the exchange form, outside
  // the interior, the receive buffer of that face (indexes fit 32 bits: a face
  // holds at most INT32_MAX elements)
  auto xn = [&](int d) -> float {
    const int xm = x + d;
    if (XCH && xm < 0) return fc.in[0][((unsigned)k * ny + (unsigned)y) * 4u + (unsigned)(xm + 4)];
    if (XCH && xm >= g.nx)
      return fc.in[1][((unsigned)k * ny + (unsigned)y) * 4u + (unsigned)(xm - g.nx)];
    return c0[d];
  };
  auto yn = [&](int d) -> float {
    const int ym = y + d;
    if (XCH && ym < 0) return fc.in[2][((unsigned)k * 4u + (unsigned)(ym + 4)) * nx + (unsigned)x];
    if (XCH && ym >= g.ny)
      return fc.in[3][((unsigned)k * 4u + (unsigned)(ym - g.ny)) * nx + (unsigned)x];
    return c0[(long long)d * g.sy];
  };
  auto zn = [&](int d) -> float {
    const int zm = k + d;
    if (XCH && zm < 0) return fc.in[4][((unsigned)(zm + 4) * ny + (unsigned)y) * nx + (unsigned)x];
    if (XCH && zm >= g.nz)
      return fc.in[5][((unsigned)(zm - g.nz) * ny + (unsigned)y) * nx + (unsigned)x];
    return c0[(long long)d * g.sz];
  };
  const float uc = c0[0];
  float lap = c.cc * uc;
#pragma unroll
  for (int m = 1; m <= 4; ++m) lap += c.cx[m] * (xn(m) + xn(-m));
#pragma unroll
  for (int m = 1; m <= 4; ++m) lap += c.cy[m] * (yn(m) + yn(-m));
#pragma unroll
  for (int m = 1; m <= 4; ++m) lap += c.cz[m] * (zn(m) + zn(-m));
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
  if (REC == 2 && k == rk) {
    const int rr = rmap[y * g.nx + x];
    if (rr >= 0) {
      // rounds as fd_scatter_add_scaled: the row value times vdt2 / (1+eta)
#pragma clang fp contract(off)
      v += rrow[rr] * (pb / (1.f + eta));
    }
  }
  un[o] = v;  // a plain store: the next step reads it from cache
  if (XCH) {  // the faces of the result that hold this point
    const unsigned ux = (unsigned)x, uy = (unsigned)y, uk = (unsigned)k;
    if (x < 4) fc.out[0][(uk * ny + uy) * 4u + ux] = v;
    if (x >= g.nx - 4) fc.out[1][(uk * ny + uy) * 4u + (ux - (nx - 4u))] = v;
    if (y < 4) fc.out[2][(uk * 4u + uy) * nx + ux] = v;
    if (y >= g.ny - 4) fc.out[3][(uk * 4u + (uy - (ny - 4u))) * nx + ux] = v;
    if (k < 4) fc.out[4][(uk * ny + uy) * nx + ux] = v;
    if (k >= g.nz - 4) fc.out[5][((uk - (nz - 4u)) * ny + uy) * nx + ux] = v;
  }
  if (REC == 1 && k == rk) {
    const int rr = rmap[y * g.nx + x];
    if (rr >= 0) rrow[rr] = v;
  }
}

}  // namespace

hipError_t launch_step_point(const Geo& g, const Coef& c, const float* up, const float* u,
                             float* un, const float* q, const float* ex, const float* ey,
                             const float* ez, const fd_source* src, const RecPlane* rp,
                             hipStream_t s, const float* const rin[6], float* const sout[6]) {
  const bool xch = rin != nullptr;
  if (xch && rp && rp->map && rp->add) return hipErrorInvalidValue;  // exchange: records only
  PFaces fc{};
  if (xch) {
    if (!sout || g.nx < 4 || g.ny < 4 || g.nz < 4) return hipErrorInvalidValue;
    for (int f = 0; f < 6; ++f) {
      if (!rin[f] || !sout[f]) return hipErrorInvalidValue;
      fc.in[f] = rin[f];
      fc.out[f] = sout[f];
    }
  }
  const dim3 grid((unsigned)((g.nx + PX - 1) / PX), (unsigned)((g.ny + PY - 1) / PY),
                  (unsigned)g.nz);
  const int si = src ? src->i : -1, sj = src ? src->j : -1, sk = src ? src->k : -1;
  const float sw = src ? src->w : 0.f;
  const bool rec = rp && rp->map;
  const int32_t* map = rec ? rp->map : nullptr;
  const int rk = rec ? rp->k : -1;
  float* row = rec ? rp->row : nullptr;
  const int recm = rec ? (rp->add ? 2 : 1) : 0;
  const int variant = (ex ? 8 : 0) | (recm << 1) | (xch ? 1 : 0);
#define FD_POINT(SP, RC, XC)                                                                   \
  hipLaunchKernelGGL((point_kernel<SP, RC, XC>), grid, dim3(PX, PY), 0, s, g, c, up, u, un, q, \
                     ex, ey, ez, si, sj, sk, sw, map, rk, row, fc)
  switch (variant) {
    case 8 | 2 | 1: FD_POINT(true, 1, true); break;
    case 8 | 2: FD_POINT(true, 1, false); break;
    case 8 | 4: FD_POINT(true, 2, false); break;
    case 8 | 1: FD_POINT(true, 0, true); break;
    case 8: FD_POINT(true, 0, false); break;
    case 2 | 1: FD_POINT(false, 1, true); break;
    case 2: FD_POINT(false, 1, false); break;
    case 4: FD_POINT(false, 2, false); break;
    case 1: FD_POINT(false, 0, true); break;
    default: FD_POINT(false, 0, false); break;
  }
#undef FD_POINT
  return hipGetLastError();
}

}  // namespace fd
