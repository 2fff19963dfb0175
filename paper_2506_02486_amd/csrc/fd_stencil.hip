// fd_stencil.hip -- the 25-point 8th-order star stencil on gfx950.
//
// One z-marching engine serves three operations:
//   FWD  : u_next = (2u - (1-eta) u_prev + vdt2 * L u) / (1+eta)      (fd_step)
//          optionally + the source term (FUSE)
//   ADJ  : a_out  = 2 D c + L(vdt2 D c) - E D a_nn,  D = 1/(1+eta),
//          E = 1-eta, c = a^{n+1}                                  (fd_adjoint_step)
//   GRAD : g     += D c (L u + f)                                  (fused gradient)
//
// Work decomposition (2.5-D blocking).  A block of TXT x NY threads owns an
// x-y tile of TXT x (NY*RY) points and marches along z through a chunk of
// `kchunk` planes.  threadIdx.x = x (each wave loads a 256-byte coalesced row
// segment); each thread row owns RY consecutive y rows.  Per plane:
//   * the stencil field of the current plane (tile + 4-wide x and y halos) is
//     staged in LDS (double buffered, so one barrier per plane);
//   * x neighbours come from LDS; y neighbours from the thread's own registers
//     when the row is its own, else from LDS;
//   * z neighbours come from a 9-deep register queue per row, so every plane of
//     the field is read from global memory once per block (plus the 8-plane
//     z halo of each chunk); the queue is a ring renamed by unrolling the z loop
//     nine times, so advancing a plane moves no registers;
//   * the next plane of every operand is prefetched one iteration ahead;
//   * pointwise operands (u_prev, vdt2, ...) are streamed with non-temporal
//     loads and the result with non-temporal stores, leaving L2 to the field
//     whose x/y halos neighbouring tiles re-read.
// Addressing: every load is a 32-bit unsigned byte offset from a block-uniform
// plane base (the padded corner (-4,-4) of plane k), so the address of each
// load is one scalar base plus one 32-bit register.
// Sponge: a block whose x-y tile lies outside the damping layer takes the
// undamped update on planes where eta_z is zero too (a uniform branch), and
// inside such tiles the damped form applies only where eta != 0, so a point's
// bits never depend on its tile.
// Blocks are renumbered so that each of the 8 XCDs (each with its own L2) gets
// one contiguous run of tiles: hardware dispatches block b to XCD b % 8.
// Exchange form (XCH, fd_step_exchange): the -x/+x halos are read from receive
// buffers and the x faces of the result written to send buffers by the lanes
// that own them, instead of a separate unpack/pack over 16-byte row pieces.
// Receiver plane (REC): when the receivers share one z plane, the forward
// kernel writes their trace row at that plane from a per-point index map.
// Tile shapes: 64 x 32 (8 waves, 4 rows per thread); 64 x 16 (2 rows per
// thread) for small grids, where it doubles the blocks.
#include <type_traits>

#include "fd_internal.h"

namespace fd {
namespace {

enum Mode { FWD = 0, ADJ = 1, GRAD = 2 };

struct Params {
  Geo g;
  Coef c;
  // stencil field: FWD/GRAD read f; ADJ forms vdt2 * D * f from f = a^{n+1} and fq = vdt2
  const float* f;
  const float* fq;
  // pointwise operands
  const float* pa;  // FWD: u_prev   ADJ: a_nn (may be null)  GRAD: a^{n+1}
  const float* pb;  // FWD: vdt2     ADJ: -                   GRAD: -
  float* out;       // FWD: u_next   ADJ: a_out               GRAD: g (read-modify-write)
  const float* ex;
  const float* ey;
  const float* ez;
  int tiles_x, tiles_y, kchunk;
  int si, sj, sk;   // source point (si < 0: none): FWD adds its term, GRAD its f
  float sw;         // source amplitude
  // exchange form (XCH): the x-face halos of f are read from rin[0], rin[1]
  // instead of f's own halo, and the x faces of out are written to sout[0],
  // sout[1] (halo_unpack / halo_pack layouts [nz][ny][4]; all four non-NULL)
  const float* rin[2];
  float* sout[2];
  // FWD: receivers on plane rk: rmap[j * nx + i] is the receiver index of point
  // (i, j, rk) or -1, and rrow[r] takes u_next there (rmap NULL: none)
  const int32_t* rmap;
  int rk;
  float* rrow;
  bool radd;  // rrow is a row to add (scaled by vdt2 / (1+eta)) instead of to write
};

__device__ __forceinline__ int remap_block(int bid, int nb) {
  const int per = nb >> 3;
  if (bid < (per << 3)) return (bid & 7) * per + (bid >> 3);
  return bid;
}

__device__ __forceinline__ int wrapi(int i, int n) {
  while (i < 0) i += n;
  while (i >= n) i -= n;
  return i;
}

__device__ __forceinline__ float ld(const char* base, unsigned boff) {
  return *reinterpret_cast<const float*>(base + boff);
}
__device__ __forceinline__ float ld_nt(const char* base, unsigned boff) {
  return __builtin_nontemporal_load(reinterpret_cast<const float*>(base + boff));
}

// The per-block work of every stencil kernel: tile (bx, by) of the x-y plane,
// z-chunk bz, of the grid and operands described by p.
template <int TXT, int NY, int RY, int MODE, bool SPONGE, bool FUSE, bool EARLY, bool XCH,
          int REC = 0>
__device__ __forceinline__ void stencil_block(const Params& p, const int bx, const int by,
                                              const int bz) {
  constexpr int TX = TXT;
  constexpr int TY = NY * RY;
  constexpr int LX = TX + 8;
  constexpr int LY = TY + 8;
  constexpr int HPT = 8 / NY;  // y-halo rows each thread row loads per plane
  static_assert(NY == 1 || NY == 2 || NY == 4 || NY == 8, "NY must divide 8");
  static_assert(8 * RY <= TXT, "x-halo cells must fit in one thread row");
  static_assert(!EARLY || MODE == FWD, "the halo ring needs the unrolled forward z loop");
  static_assert(!XCH || EARLY, "the exchange form is a forward kernel");

  __shared__ float sm[2][LY * LX];

  const int lane = threadIdx.x;
  // a wave is one thread row when TXT is a multiple of 64: w is wave-uniform
  const int w = TXT % 64 == 0 ? __builtin_amdgcn_readfirstlane((int)threadIdx.y) : (int)threadIdx.y;
  const int nx = p.g.nx, ny = p.g.ny, nz = p.g.nz;
  const int sy = p.g.sy;
  const long long szb = 4LL * p.g.sz;  // plane stride in bytes
  const int x0 = bx * TX;
  const int y0 = by * TY;
  const int kb = bz * p.kchunk;
  const int ke = min(kb + p.kchunk, nz);
  const int x = x0 + lane;
  const int yr = y0 + w * RY;

  // byte offset of (x, y) inside a plane, from the padded corner (-4, -4)
  auto boff = [&](int xx, int yy) -> unsigned {
    return 4u * (unsigned)((yy + 4) * sy + (xx + 4));
  };

  // ---- per-thread geometry of the cells it loads every plane
  unsigned cb[RY];
  bool cld[RY], act[RY];
#pragma unroll
  for (int r = 0; r < RY; ++r) {
    const int yy = yr + r;
    cb[r] = boff(x, yy);
    cld[r] = (x < nx + 4) && (yy < ny + 4);
    act[r] = (x < nx) && (yy < ny);
  }
  // y-halo rows: thread row w loads halo rows hr = w + h*NY (h < HPT) at column
  // x; hr < 4 are the rows above the tile, hr >= 4 the rows below
  int hy_y[HPT], hy_lds[HPT];
  unsigned hyb[HPT];
  bool hy_ld[HPT];
#pragma unroll
  for (int h = 0; h < HPT; ++h) {
    const int hr = w + h * NY;
    hy_y[h] = hr < 4 ? y0 - 4 + hr : y0 + TY + (hr - 4);
    hyb[h] = boff(x, hy_y[h]);
    hy_lds[h] = (hr < 4 ? hr : TY + hr) * LX + 4 + lane;
    hy_ld[h] = (x < nx + 4) && (hy_y[h] < ny + 4);
  }
  // x-halo columns: lanes < 8*RY of each thread row load (row yr + lane/8, column c = lane%8)
  const int hx_r = lane >> 3;
  const int hx_c = lane & 7;
  const int hx_x = hx_c < 4 ? x0 - 4 + hx_c : x0 + TX + (hx_c - 4);
  const int hx_y = yr + hx_r;
  const bool hx_on = lane < 8 * RY;
  const bool hx_ld = hx_on && (hx_x < nx + 4) && (hx_y < ny + 4);
  const unsigned hxb = boff(hx_on ? hx_x : 0, hx_on ? hx_y : 0);
  const int hx_lds = (4 + w * RY + hx_r) * LX + (hx_c < 4 ? hx_c : TX + hx_c);

  // ---- sponge factors that are constant along z for this thread
  float ex_c = 0.f, ex_h = 0.f, ey_r[RY], ey_hy[HPT], ey_h = 0.f;
#pragma unroll
  for (int r = 0; r < RY; ++r) ey_r[r] = 0.f;
#pragma unroll
  for (int h = 0; h < HPT; ++h) ey_hy[h] = 0.f;
  bool tile_sponge = false;  // block-uniform: some point of the x-y tile is damped
  if (SPONGE) {
    if (MODE == ADJ) {  // halo cells take eta of their periodic image
      if (x < nx + 4) ex_c = p.ex[wrapi(x, nx)];
      if (hx_ld) ex_h = p.ex[wrapi(hx_x, nx)];
      if (hx_ld) ey_h = p.ey[wrapi(hx_y, ny)];
#pragma unroll
      for (int h = 0; h < HPT; ++h)
        if (hy_y[h] < ny + 4) ey_hy[h] = p.ey[wrapi(hy_y[h], ny)];
#pragma unroll
      for (int r = 0; r < RY; ++r)
        if (yr + r < ny + 4) ey_r[r] = p.ey[wrapi(yr + r, ny)];
    } else {
      if (x < nx) ex_c = p.ex[x];
      int any = 0;
#pragma unroll
      for (int r = 0; r < RY; ++r) {
        if (yr + r < ny) ey_r[r] = p.ey[yr + r];
        any |= act[r] && (ex_c != 0.f || ey_r[r] != 0.f);
      }
      tile_sponge = __syncthreads_or(any) != 0;
    }
  }

  // block-uniform: the source point lies in this block's tile and z chunk
  const bool src_tile = p.si >= x0 && p.si < x0 + TX && p.sj >= y0 && p.sj < y0 + TY &&
                        p.sk >= kb && p.sk < ke;

  const long long org_c = p.g.org - 4LL * sy - 4;  // element offset of the padded corner
  const char* F0 = reinterpret_cast<const char*>(p.f + org_c);
  const char* Q0 = reinterpret_cast<const char*>(p.fq + org_c);
  const char* A0 = reinterpret_cast<const char*>(p.pa ? p.pa + org_c : p.f + org_c);
  const char* B0 = reinterpret_cast<const char*>(p.pb ? p.pb + org_c : p.f + org_c);
  char* O0 = reinterpret_cast<char*>(p.out + org_c);

  // Field value at byte offset b of plane k (k in [-4, nz+4)).  ADJ forms
  // vdt2 * c / (1 + eta) with eta of the periodic image.
  auto fld = [&](const char* fk, const char* qk, unsigned b, bool ok, float exv, float eyv,
                 float ezv) -> float {
    if (!ok) return 0.f;
    if (MODE == ADJ) {
      float v = ld(qk, b) * ld(fk, b);
      if (SPONGE) v *= __builtin_amdgcn_rcpf(1.f + (exv + eyv + ezv));
      return v;
    } else {
      return ld(fk, b);
    }
  };
  // XCH: the x-face halos come from the receive buffers and the x faces of the
  // result go to the send buffers.  Both are 16-byte pieces of rows whose cache
  // lines otherwise hold interior points, so a separate pack/unpack, and the
  // stencil's own x-halo loads, fetch and write whole lines for them; here each
  // lane keeps a pointer and a per-plane step for its x-halo cell (interior
  // tiles: u itself) and edge lanes a pointer into the x face they own.  nx is a
  // multiple of TX, so only lanes hx_c < 4 of the first tile column and hx_c >= 4
  // of the last read x halos; rows hx_y >= ny of a ragged last tile row are
  // corner cells no point uses, left on u's halo (in bounds).
  const char* hxp = F0 + hxb;
  unsigned hxs = (unsigned)szb;
  float* sx_ptr = nullptr;
  bool xedge = false;  // block-uniform: the tile holds x-face points
  if (XCH) {
    if (hx_on && hx_y < ny && hx_c < 4 && bx == 0) {
      hxp = reinterpret_cast<const char*>(p.rin[0]) + 4ull * ((unsigned)hx_y * 4u + (unsigned)hx_c);
      hxs = 16u * (unsigned)ny;
    } else if (hx_on && hx_y < ny && hx_c >= 4 && x0 + TX == nx) {
      hxp = reinterpret_cast<const char*>(p.rin[1]) +
            4ull * ((unsigned)hx_y * 4u + (unsigned)(hx_c - 4));
      hxs = 16u * (unsigned)ny;
    }
    if (x < 4) sx_ptr = p.sout[0] + x;
    else if (x >= nx - 4) sx_ptr = p.sout[1] + (x - (nx - 4));
    xedge = bx == 0 || x0 + TX == nx;
  }
  auto xload = [&](int k) -> float {
    return hx_ld ? *reinterpret_cast<const float*>(hxp + (unsigned long long)k * hxs) : 0.f;
  };

  auto ezw = [&](int k) -> float {
    if (!SPONGE) return 0.f;
    if (MODE == ADJ) return p.ez[wrapi(k, nz)];
    return (k >= 0 && k < nz) ? p.ez[k] : 0.f;
  };

  // ---- prologue: z queue for planes kb-4 .. kb+4, halos of plane kb
  float zq[9][RY];
  float cq[5][RY];  // ADJ: a^{n+1} of planes k .. k+4 (centre column)
#pragma unroll
  for (int s = 0; s < 9; ++s) {
    const int k = kb - 4 + s;
    const float ezv = ezw(k);
    const char* fk = F0 + (long long)k * szb;
    const char* qk = Q0 + (long long)k * szb;
#pragma unroll
    for (int r = 0; r < RY; ++r) {
      zq[s][r] = fld(fk, qk, cb[r], cld[r], ex_c, ey_r[r], ezv);
      if (MODE == ADJ && s >= 4) cq[s - 4][r] = cld[r] ? ld(fk, cb[r]) : 0.f;
    }
  }
  // x-y halos of the field.  EARLY: a ring like the z queue (slot (P + s) % 9
  // holds plane k - 4 + s; planes k .. k + 4 are live), filled in the same
  // iteration as the centre column of the plane, so that a neighbouring tile's
  // re-read of those cells follows its own load closely enough to hit in L2.
  // Otherwise: the halos of plane k only, loaded one plane ahead.
  float hy[HPT], hx;
  float hq[9][HPT], xq[9];  // the early form's rings (unused, and removed, otherwise)
  if constexpr (EARLY) {
#pragma unroll
    for (int s = 4; s < 9; ++s) {
      const int k = kb - 4 + s;
      const char* fk = F0 + (long long)k * szb;
#pragma unroll
      for (int h = 0; h < HPT; ++h)
        hq[s][h] = k < ke ? fld(fk, fk, hyb[h], hy_ld[h], 0.f, 0.f, 0.f) : 0.f;
      xq[s] = k < ke ? (XCH ? xload(k) : fld(fk, fk, hxb, hx_ld, 0.f, 0.f, 0.f)) : 0.f;
    }
  } else {
    const float ezv = ezw(kb);
    const char* fk = F0 + (long long)kb * szb;
    const char* qk = Q0 + (long long)kb * szb;
#pragma unroll
    for (int h = 0; h < HPT; ++h) hy[h] = fld(fk, qk, hyb[h], hy_ld[h], ex_c, ey_hy[h], ezv);
    hx = fld(fk, qk, hxb, hx_ld, ex_h, ey_h, ezv);
  }
  float pa[RY], pb[RY];
  {
    const char* ak = A0 + (long long)kb * szb;
    const char* bk = B0 + (long long)kb * szb;
    const char* ok = O0 + (long long)kb * szb;
#pragma unroll
    for (int r = 0; r < RY; ++r) {
      pa[r] = 0.f;
      pb[r] = 0.f;
      if (act[r] && kb < ke) {
        if (MODE == FWD) {
          pa[r] = ld_nt(ak, cb[r]);
          pb[r] = ld_nt(bk, cb[r]);
        } else if (MODE == ADJ) {
          if (p.pa) pa[r] = ld_nt(ak, cb[r]);
        } else {
          pa[r] = ld_nt(ak, cb[r]);
          pb[r] = ld(ok, cb[r]);
        }
      }
    }
  }

  // One z-plane.  The 9-plane queue is a ring: with ring position P (the
  // plane's index since kb, mod 9) slot (P + s) % 9 holds plane k - 4 + s, so
  // advancing a plane renames registers instead of moving them (the loop below
  // is unrolled 9 times with a compile-time P).
  auto iter = [&](auto pos, const int k) {
    constexpr int P = decltype(pos)::value;
    const int buf = (k - kb) & 1;
    // ---- prefetch for the next iteration
    float nzq[RY], ncq[RY], npa[RY], npb[RY], nhy[HPT];
    float nhx = 0.f;
#pragma unroll
    for (int h = 0; h < HPT; ++h) nhy[h] = 0.f;
    {
      const int kn = k + 5;
      const bool need = kn < ke + 4;
      const float ezv = ezw(kn);
      const char* fk = F0 + (long long)kn * szb;
      const char* qk = Q0 + (long long)kn * szb;
#pragma unroll
      for (int r = 0; r < RY; ++r) {
        nzq[r] = need ? fld(fk, qk, cb[r], cld[r], ex_c, ey_r[r], ezv) : 0.f;
        if (MODE == ADJ) ncq[r] = (need && cld[r]) ? ld(fk, cb[r]) : 0.f;
      }
    }
    const bool more = k + 1 < ke;
    if (EARLY) {
      const int kn = k + 5;
      if (kn < ke) {
        const char* fk = F0 + (long long)kn * szb;
#pragma unroll
        for (int h = 0; h < HPT; ++h)
          nhy[h] = fld(fk, fk, hyb[h], hy_ld[h], 0.f, 0.f, 0.f);
        nhx = XCH ? xload(kn) : fld(fk, fk, hxb, hx_ld, 0.f, 0.f, 0.f);
      }
    } else if (more) {
      const float ezv = ezw(k + 1);
      const char* fk = F0 + (long long)(k + 1) * szb;
      const char* qk = Q0 + (long long)(k + 1) * szb;
#pragma unroll
      for (int h = 0; h < HPT; ++h) nhy[h] = fld(fk, qk, hyb[h], hy_ld[h], ex_c, ey_hy[h], ezv);
      nhx = fld(fk, qk, hxb, hx_ld, ex_h, ey_h, ezv);
    }
    {
      const char* ak = A0 + (long long)(k + 1) * szb;
      const char* bk = B0 + (long long)(k + 1) * szb;
      const char* ok = O0 + (long long)(k + 1) * szb;
#pragma unroll
      for (int r = 0; r < RY; ++r) {
        npa[r] = 0.f;
        npb[r] = 0.f;
        if (more && act[r]) {
          if (MODE == FWD) {
            npa[r] = ld_nt(ak, cb[r]);
            npb[r] = ld_nt(bk, cb[r]);
          } else if (MODE == ADJ) {
            if (p.pa) npa[r] = ld_nt(ak, cb[r]);
          } else {
            npa[r] = ld_nt(ak, cb[r]);
            npb[r] = ld(ok, cb[r]);
          }
        }
      }
    }

    // ---- stage plane k of the field in LDS
    float* s = sm[buf];
#pragma unroll
    for (int r = 0; r < RY; ++r) s[(4 + w * RY + r) * LX + 4 + lane] = zq[(P + 4) % 9][r];
#pragma unroll
    for (int h = 0; h < HPT; ++h) s[hy_lds[h]] = EARLY ? hq[(P + 4) % 9][h] : hy[h];
    if (hx_on) s[hx_lds] = EARLY ? xq[(P + 4) % 9] : hx;
    __syncthreads();

    // ---- compute
    const float ezk = SPONGE ? p.ez[k] : 0.f;
    // block-uniform: does any point of this tile-plane carry damping?
    const bool damped = SPONGE && (MODE == ADJ || tile_sponge || ezk != 0.f);
    // block-uniform: the source point lies in this tile-plane
    const bool src_plane = src_tile && k == p.sk;
    // block-uniform: this plane holds the receivers (REC: a separate instantiation,
    // so the kernels without it keep their registers; 1 writes their trace row,
    // 2 adds a row scaled by vdt2 / (1+eta) as fd_scatter_add_scaled would)
    const bool rec_plane = REC != 0 && MODE == FWD && k == p.rk;
    char* ok = O0 + (long long)k * szb;
#pragma unroll
    for (int r = 0; r < RY; ++r) {
      const float* row = s + (4 + w * RY + r) * LX + 4 + lane;
      const float uc = zq[(P + 4) % 9][r];
      float lap = p.c.cc * uc;
#pragma unroll
      for (int m = 1; m <= 4; ++m) lap += p.c.cx[m] * (row[m] + row[-m]);
#pragma unroll
      for (int m = 1; m <= 4; ++m) {
        const float up_ = (r + m < RY) ? zq[(P + 4) % 9][(r + m) % RY] : row[m * LX];
        const float dn_ = (r - m >= 0) ? zq[(P + 4) % 9][(r - m + RY) % RY] : row[-m * LX];
        lap += p.c.cy[m] * (up_ + dn_);
      }
#pragma unroll
      for (int m = 1; m <= 4; ++m) lap += p.c.cz[m] * (zq[(P + 4 + m) % 9][r] + zq[(P + 4 - m) % 9][r]);

      if (act[r]) {
        float eta = 0.f;
        if (damped) eta = ex_c + ey_r[r] + ezk;
        float* dst = reinterpret_cast<float*>(ok + cb[r]);
        if (MODE == FWD) {
          // undamped update; the damped one, (2u - (1-eta) u_prev + q L u)/(1+eta),
          // is that value plus eta u_prev over 1+eta, taken only where eta != 0 (with
          // eta == 0 it would still turn a -0 into +0), so a point's bits do not
          // depend on whether its tile holds damped points
          float v = 2.f * uc - pa[r] + pb[r] * lap;
          if (damped && eta != 0.f) v = (v + eta * pa[r]) * __builtin_amdgcn_rcpf(1.f + eta);
          if (FUSE && src_plane) {
            // no contraction: the product, quotient and sum round exactly as in
            // inject_source, whether or not eta is known to be 0 here
#pragma clang fp contract(off)
            if (x == p.si && yr + r == p.sj) v += pb[r] * p.sw / (1.f + eta);
          }
          if constexpr (REC == 2) {
            if (rec_plane) {
              const int rr = p.rmap[(yr + r) * nx + x];
              if (rr >= 0) {
                // rounds as fd_scatter_add_scaled: the row value times vdt2 / (1+eta)
#pragma clang fp contract(off)
                v += p.rrow[rr] * (pb[r] / (1.f + eta));
              }
            }
          }
          __builtin_nontemporal_store(v, dst);
          if (XCH && xedge && sx_ptr) sx_ptr[((unsigned)k * (unsigned)ny + (unsigned)(yr + r)) * 4u] = v;
          if constexpr (REC == 1) {
            if (rec_plane) {
              const int rr = p.rmap[(yr + r) * nx + x];
              if (rr >= 0) p.rrow[rr] = v;
            }
          }
        } else if (MODE == ADJ) {
          const float c = cq[0][r];
          float v;
          if (damped && eta != 0.f) {
            const float D = __builtin_amdgcn_rcpf(1.f + eta);
            v = 2.f * D * c + lap - (1.f - eta) * D * pa[r];
          } else {
            v = 2.f * c + lap - pa[r];
          }
          __builtin_nontemporal_store(v, dst);
        } else {
          float src = 0.f;
          if (src_plane && x == p.si && yr + r == p.sj) src = p.sw;
          float D = 1.f;
          if (damped && eta != 0.f) D = __builtin_amdgcn_rcpf(1.f + eta);
          *dst = pb[r] + D * pa[r] * (lap + src);
        }
      }
    }

    // ---- rotate queues
#pragma unroll
    for (int r = 0; r < RY; ++r) {
      zq[P][r] = nzq[r];  // plane k + 5 replaces plane k - 4
      if (MODE == ADJ) {
#pragma unroll
        for (int t = 0; t < 4; ++t) cq[t][r] = cq[t + 1][r];
        cq[4][r] = ncq[r];
      }
      pa[r] = npa[r];
      pb[r] = npb[r];
    }
#pragma unroll
    for (int h = 0; h < HPT; ++h) {
      if constexpr (EARLY) hq[P][h] = nhy[h];  // plane k + 5
      else hy[h] = nhy[h];
    }
    if constexpr (EARLY) xq[P] = nhx;
    else hx = nhx;
  };
  using std::integral_constant;
  if (MODE != FWD) {  // the adjoint kernels keep the queue in place (fewer scalar registers)
    for (int k = kb; k < ke; ++k) {
      iter(integral_constant<int, 0>{}, k);
#pragma unroll
      for (int r = 0; r < RY; ++r) {  // rotate: slot 0 now holds plane k + 5
        const float t = zq[0][r];
#pragma unroll
        for (int s2 = 0; s2 < 8; ++s2) zq[s2][r] = zq[s2 + 1][r];
        zq[8][r] = t;
      }
    }
    return;
  }
  for (int k = kb; k < ke; k += 9) {
    iter(integral_constant<int, 0>{}, k);
    if (k + 1 >= ke) break;
    iter(integral_constant<int, 1>{}, k + 1);
    if (k + 2 >= ke) break;
    iter(integral_constant<int, 2>{}, k + 2);
    if (k + 3 >= ke) break;
    iter(integral_constant<int, 3>{}, k + 3);
    if (k + 4 >= ke) break;
    iter(integral_constant<int, 4>{}, k + 4);
    if (k + 5 >= ke) break;
    iter(integral_constant<int, 5>{}, k + 5);
    if (k + 6 >= ke) break;
    iter(integral_constant<int, 6>{}, k + 6);
    if (k + 7 >= ke) break;
    iter(integral_constant<int, 7>{}, k + 7);
    if (k + 8 >= ke) break;
    iter(integral_constant<int, 8>{}, k + 8);
  }
}

template <int TXT, int NY, int RY, int MODE, bool SPONGE, bool FUSE, bool EARLY = (MODE == FWD),
          bool XCH = false, int REC = 0>
__global__ void __launch_bounds__(TXT * NY) stencil_kernel(Params p) {
  const int logical = remap_block(blockIdx.x, gridDim.x);
  const int bx = logical % p.tiles_x;
  const int rest = logical / p.tiles_x;
  stencil_block<TXT, NY, RY, MODE, SPONGE, FUSE, EARLY, XCH, REC>(p, bx, rest % p.tiles_y,
                                                             rest / p.tiles_y);
}

// Many grids in one launch: block b runs tile tiles[remap(b)] = (slot, bx, by, bz)
// of shot `slot`, whose step is a.n[slot] (u^n in arr[n % 3]) and source
// amplitude a.w[slot].  Every point runs exactly the code of stencil_kernel; a shot
// whose receivers share one plane has its trace row written here too.
template <int TXT, int NY, int RY>
__global__ void __launch_bounds__(TXT * NY) batched_kernel(const BatchShot* __restrict__ shots,
                                                           const int4* __restrict__ tiles,
                                                           BatchStep a) {
  const int4 t = tiles[remap_block(blockIdx.x, gridDim.x)];
  const BatchShot& b = shots[t.x];
  const int n = a.n[t.x];
  Params p;
  p.g = b.g;
  p.c = b.c;
  p.f = b.arr[n % 3];
  p.fq = p.f;
  p.pa = b.arr[(n + 2) % 3];
  p.pb = b.q;
  p.out = b.arr[(n + 1) % 3];
  p.ex = b.ex;
  p.ey = b.ey;
  p.ez = b.ez;
  p.tiles_x = 0;
  p.tiles_y = 0;
  p.kchunk = b.kchunk;
  p.si = b.si;
  p.sj = b.sj;
  p.sk = b.sk;
  p.sw = a.w[t.x];
  p.rmap = b.rmap;
  p.rk = b.rmap ? b.rk : -1;  // no plane: the receiver epilogue never runs
  p.rrow = b.traces + (size_t)n * (size_t)b.nrec;
  p.radd = false;
  stencil_block<TXT, NY, RY, FWD, true, true, true, false, 1>(p, t.y, t.z, t.w);
}

template <int TXT, int NY, int RY, int MODE, bool SPONGE, bool FUSE = false,
          bool EARLY = (MODE == FWD), bool XCH = false, int REC = 0>
hipError_t launch_mode(Params p, hipStream_t st) {
  const LaunchShape sh = stencil_shape(p.g, TXT, NY * RY, (TXT * NY + 63) / 64);
  p.tiles_x = sh.tiles_x;
  p.tiles_y = sh.tiles_y;
  p.kchunk = sh.kchunk;
  const long long nb = (long long)sh.tiles_x * sh.tiles_y * sh.zchunks;
  if (nb <= 0 || nb > 0x7fffffffLL) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL((stencil_kernel<TXT, NY, RY, MODE, SPONGE, FUSE, EARLY, XCH, REC>), dim3((unsigned)nb),
                     dim3(TXT, NY), 0, st, p);
  return hipGetLastError();
}

Params base_params(const Geo& g, const Coef& c, const float* ex, const float* ey,
                   const float* ez) {
  Params p{};
  p.g = g;
  p.c = c;
  p.ex = ex;
  p.ey = ey;
  p.ez = ez;
  p.si = -1;
  p.sj = -1;
  p.sk = -1;
  p.sw = 0.f;
  p.rmap = nullptr;
  p.rk = -1;
  p.rrow = nullptr;
  p.radd = false;
  return p;
}

// tile shapes (threads in x, thread rows, y rows per thread)
#define FWD_SHAPE 64, 8, 4
#define FWD_SMALL_SHAPE 64, 8, 2  // grids small enough to leave CUs idle with 64 x 32 tiles
#define ADJ_SHAPE 64, 4, 2
constexpr int BATCH_TX = 64;      // tile width of the batched kernel (FWD_SHAPE)
constexpr int BATCH_TY = 8 * 4;   // tile height of the batched kernel (FWD_SHAPE)

// The forward kernel in one tile shape: x faces exchanged inside (always with the
// source epilogue, a negative source index meaning none), or the source and the
// receiver row fused, or the source fused, or the plain update.
template <int TXT, int NY, int RY>
hipError_t launch_forward(const Params& p, bool sponge, bool fuse, bool xch, hipStream_t s) {
  if (p.rmap && !xch && !p.radd) {  // the receiver row written by the kernel
    if (sponge) return launch_mode<TXT, NY, RY, FWD, true, true, true, false, 1>(p, s);
    return launch_mode<TXT, NY, RY, FWD, false, true, true, false, 1>(p, s);
  }
  if (p.rmap && !xch) {  // a scaled row added at the receiver points
    if (sponge) return launch_mode<TXT, NY, RY, FWD, true, true, true, false, 2>(p, s);
    return launch_mode<TXT, NY, RY, FWD, false, true, true, false, 2>(p, s);
  }
  if (xch) {
    if (sponge) return launch_mode<TXT, NY, RY, FWD, true, true, true, true>(p, s);
    return launch_mode<TXT, NY, RY, FWD, false, true, true, true>(p, s);
  }
  if (fuse) {
    if (sponge) return launch_mode<TXT, NY, RY, FWD, true, true>(p, s);
    return launch_mode<TXT, NY, RY, FWD, false, true>(p, s);
  }
  if (sponge) return launch_mode<TXT, NY, RY, FWD, true>(p, s);
  return launch_mode<TXT, NY, RY, FWD, false>(p, s);
}

hipError_t launch_forward(const Params& p, bool sponge, bool fuse, bool xch, hipStream_t s) {
  if (forward_small_tiles(p.g)) return launch_forward<FWD_SMALL_SHAPE>(p, sponge, fuse, xch, s);
  return launch_forward<FWD_SHAPE>(p, sponge, fuse, xch, s);
}

}  // namespace

void forward_launch_shape(const Geo& g, int out[4]) {
  // FWD_SHAPE or FWD_SMALL_SHAPE: 64-wide tiles of 8 waves, 4 or 2 rows per thread
  const int ty = forward_small_tiles(g) ? 8 * 2 : 8 * 4;
  const LaunchShape sh = stencil_shape(g, 64, ty, 8);
  out[0] = sh.tiles_x;
  out[1] = sh.tiles_y;
  out[2] = sh.kchunk;
  out[3] = sh.zchunks;
}

int batch_tile_shape(int* tx, int* ty) {
  *tx = BATCH_TX;
  *ty = BATCH_TY;
  return BATCH_TX * 8;
}

hipError_t launch_batched(const BatchShot* shots, const int4* tiles, int ntiles,
                          const BatchStep& a, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  hipLaunchKernelGGL((batched_kernel<FWD_SHAPE>), dim3((unsigned)ntiles), dim3(BATCH_TX, 8), 0, s,
                     shots, tiles, a);
  return hipGetLastError();
}

hipError_t launch_step(const Geo& g, const Coef& c, const float* up, const float* u,
                       float* un, const float* q, const float* ex, const float* ey,
                       const float* ez, const fd_source* src, hipStream_t s,
                       const RecPlane* rp) {
  {
    const float* const arr[4] = {up, u, un, q};
    if (wide_takes_step(g, arr))
      return launch_forward_wide(g, c, up, u, un, q, ex, ey, ez, src, nullptr, nullptr, s, rp);
  }
  Params p = base_params(g, c, ex, ey, ez);
  if (rp && rp->map) {
    p.rmap = rp->map;
    p.rk = rp->k;
    p.rrow = rp->row;
    p.radd = rp->add;
  }
  p.f = u;
  p.fq = u;
  p.pa = up;
  p.pb = q;
  p.out = un;
  if (src) {
    p.si = src->i;
    p.sj = src->j;
    p.sk = src->k;
    p.sw = src->w;
  }
  // the receiver plane needs the fused epilogue (a negative source index: none)
  return launch_forward(p, ex != nullptr, src != nullptr || p.rmap != nullptr, false, s);
}

bool exchange_fits(const Geo& g) { return g.nx % BATCH_TX == 0; }

hipError_t launch_step_exchange(const Geo& g, const Coef& c, const float* up, const float* u,
                                float* un, const float* q, const float* ex, const float* ey,
                                const float* ez, const fd_source* src, const float* const rin[2],
                                float* const sout[2], hipStream_t s) {
  if (!exchange_fits(g)) return hipErrorInvalidValue;
  if (forward_wide_tiles(g)) {
    const float* const arr[4] = {up, u, un, q};
    const float* const fc[4] = {rin[0], rin[1], sout[0], sout[1]};
    if (wide_forward_fits(g, arr, fc))
      return launch_forward_wide(g, c, up, u, un, q, ex, ey, ez, src, rin, sout, s);
  }
  Params p = base_params(g, c, ex, ey, ez);
  p.f = u;
  p.fq = u;
  p.pa = up;
  p.pb = q;
  p.out = un;
  if (src) {
    p.si = src->i;
    p.sj = src->j;
    p.sk = src->k;
    p.sw = src->w;
  }
  if (!rin[0] || !rin[1] || !sout[0] || !sout[1]) return hipErrorInvalidValue;
  for (int f = 0; f < 2; ++f) {
    p.rin[f] = rin[f];
    p.sout[f] = sout[f];
  }
  return launch_forward(p, ex != nullptr, true, true, s);
}

hipError_t launch_adjoint(const Geo& g, const Coef& c, const float* ann, const float* an1,
                          float* aout, const float* q, const float* ex, const float* ey,
                          const float* ez, hipStream_t s) {
  Params p = base_params(g, c, ex, ey, ez);
  p.f = an1;
  p.fq = q;
  p.pa = ann;
  p.pb = nullptr;
  p.out = aout;
  if (ex) return launch_mode<ADJ_SHAPE, ADJ, true>(p, s);
  return launch_mode<ADJ_SHAPE, ADJ, false>(p, s);
}

hipError_t launch_grad(const Geo& g, const Coef& c, const float* u, const float* an1,
                       float* gq, const float* ex, const float* ey, const float* ez,
                       const fd_source* src, hipStream_t s) {
  if (forward_wide_tiles(g)) {
    const float* const arr[4] = {an1, u, gq, gq};
    if (wide_forward_fits(g, arr, nullptr))
      return launch_grad_wide(g, c, u, an1, gq, ex, ey, ez, src, s);
  }
  Params p = base_params(g, c, ex, ey, ez);
  p.f = u;
  p.fq = u;
  p.pa = an1;
  p.pb = nullptr;
  p.out = gq;
  if (src) {
    p.si = src->i;
    p.sj = src->j;
    p.sk = src->k;
    p.sw = src->w;
  }
  if (ex) return launch_mode<FWD_SHAPE, GRAD, true>(p, s);
  return launch_mode<FWD_SHAPE, GRAD, false>(p, s);
}

}  // namespace fd
