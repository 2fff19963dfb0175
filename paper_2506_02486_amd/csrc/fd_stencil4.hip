// fd_stencil4.hip -- the forward stencil update with 16-byte lanes (gfx950).
//
// The same leapfrog update as the z-marching forward kernel of fd_stencil.hip
// (same arithmetic, in the same order, so the same bits), for bandwidth-bound
// grids.  What differs is how a block
// streams HBM: each lane owns 4 consecutive x points (16-byte loads and
// stores), a row of 32 lanes covers 128 x points (512 bytes), and each thread
// owns 2 consecutive y rows, so a thread has 6 independent 16-byte loads in
// flight per plane (u^n, u^{n-1}, vdt2 of both rows).  With 64 x 32 tiles of
// one float per lane the operands of one plane stream at 5.2 TB/s on MI355X;
// as 128 x 32 tiles of 16-byte lanes with two rows per thread they stream at
// 5.85 TB/s (3 reads + 1 write of a 512^3 volume, 256 blocks of 512 threads).
// Those loads only overlap the work of the planes before them if the compiler
// never has to wait for all of them: every load is unconditional (clamped
// addresses), lands in a register of its own (rings one slot longer than what
// is live) and is issued one plane before its use, and no value is loaded just
// before it is needed (eta_z travels with the pointwise operands).
//
// Block: 32 x 16 threads (8 waves; a wave holds two thread rows), tile
// 128 x 32 points, marching along z through a chunk of planes (or 16 x 32 threads,
// tile 64 x 64 points, where the x extent leaves a 128-wide tile column mostly
// empty: 320 points take 3 columns of 128 or 5 of 64; the launch takes the shape
// whose modelled cost is lower by 10%):
//   * z neighbours: a 9-deep queue of float4 per row in registers, a ring of 10
//     slots renamed by unrolling the z loop ten times;
//   * the plane (tile + 4-wide x/y halos) is staged in double-buffered LDS;
//     x neighbours are the lane's own float4 and the two float4 beside it,
//     y neighbours come from the thread's other row or from LDS;
//   * each thread of the first 8 thread rows loads one float4 of the y halo
//     (8 rows x 32 float4; 8 x 16 with 64 x 64 tiles), 64 (128) threads of the
//     others one float4 of the x halo (32 (64) rows x 2 sides); these are loaded in the same iteration as the plane
//     they belong to is loaded by the neighbouring tile as its interior (five
//     planes ahead, kept in a ring), so those re-reads hit in L2;
//   * u^{n-1} and vdt2 are prefetched one plane ahead and streamed, like the
//     result, with non-temporal accesses.
// Exchange form (XCH): the -x/+x halos of the first and last tile column are
// read from the receive buffers ([nz][ny][4]: one float4 per row) and the x
// faces of the result written to the send buffers by the lanes that own them.
// One block per CU (more than 128 VGPRs per lane): 256 blocks fill the chip.
#include <stdint.h>

#include <algorithm>
#include <type_traits>

#include "fd_internal.h"

namespace fd {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

// Tile shapes: 32 lanes x 16 thread rows (128 x 32 points), or 16 lanes x 32 thread
// rows (64 x 64 points), for grids whose x extent leaves a 128-wide tile column
// mostly empty.  Both are 512 threads; a wave is 2 or 4 thread rows.
struct Wide128 {
  static constexpr int LANES = 32;  // lanes per thread row
  static constexpr int TROWS = 16;  // thread rows per block
};
struct Wide64 {
  static constexpr int LANES = 16;
  static constexpr int TROWS = 32;
};
constexpr int RY = 2;                   // y rows per thread
constexpr int LANES = Wide128::LANES;   // the shape of the exchange, tile-table and
constexpr int TROWS = Wide128::TROWS;   // multi-grid launches
constexpr int TX = 4 * LANES;           // 128 x points per tile
constexpr int TY = TROWS * RY;          // 32 y rows per tile

struct P4 {
  Geo g;
  Coef c;
  const float* u;   // u^n (stencil field)
  const float* up;  // u^{n-1}
  const float* q;   // vdt2
  float* un;        // u^{n+1}; may alias up
  const float* ex;
  const float* ey;
  const float* ez;
  int tiles_x, tiles_y, kchunk;
  int si, sj, sk;  // source point (si < 0: none)
  float sw;
  const float* rin[2];  // XCH: -x / +x receive buffers
  float* sout[2];       // XCH: -x / +x send buffers
  // FUSE, not XCH: receivers on plane rk (rk < 0: none): rmap[j * nx + i] is the receiver
  // index of point (i, j, rk) or -1, and rrow[r] takes u^{n+1} there
  const int32_t* rmap;
  int rk;
  float* rrow;
  bool radd;    // rrow is a row to add at the receivers, scaled by vdt2 / (1+eta)
  bool narrow;  // multi-grid launch: this grid's tiles are 64 x 64 (tiles_x, tiles_y so)
};

__device__ __forceinline__ int remap_block4(int bid, int nb) {
  const int per = nb >> 3;
  if (bid < (per << 3)) return (bid & 7) * per + (bid >> 3);
  return bid;
}

__device__ __forceinline__ f4 ld4(const char* base, unsigned boff) {
  return *reinterpret_cast<const f4*>(base + boff);
}
__device__ __forceinline__ f4 ld4_nt(const char* base, unsigned boff) {
  return __builtin_nontemporal_load(reinterpret_cast<const f4*>(base + boff));
}

// The work of one block: tile (bx, by) of the x-y plane, z chunk bz, of the grid
// and operands p describes; the thread is lane lx of thread row tr (SH's shape).
template <class SH, bool SPONGE, bool FUSE, bool XCH, bool GRAD = false>
__device__ __forceinline__ void stencil4_block(const P4& p, const int bx, const int by,
                                               const int bz, const int lx, const int tr) {
  constexpr int LANES = SH::LANES;
  constexpr int TX = 4 * LANES;           // x points per tile
  constexpr int TY = SH::TROWS * RY;      // y rows per tile
  constexpr int LX = TX + 8;              // LDS row pitch (floats)
  constexpr int LY = TY + 8;              // LDS rows
  constexpr int XH = 2 * TY / LANES;      // thread rows that load the x halo
  __shared__ __attribute__((aligned(16))) float sm[2][LY * LX];

  const int nx = p.g.nx, ny = p.g.ny, nz = p.g.nz;
  const int sy = p.g.sy;
  const long long szb = 4LL * p.g.sz;
  const int x0 = bx * TX;
  const int y0 = by * TY;
  const int kb = bz * p.kchunk;
  const int ke = min(kb + p.kchunk, nz);
  const int x = x0 + 4 * lx;  // first of the lane's 4 points
  const int yr = y0 + RY * tr;

  auto boff = [&](int xx, int yy) -> unsigned {
    return 4u * (unsigned)((yy + 4) * sy + (xx + 4));
  };

  // Rows need not be a multiple of 4 floats: the float4 that holds the last
  // interior points of a row may also hold +x halo cells, and the one after it the
  // rest of the halo and up to 3 cells past it (in the row's padding, or the next
  // row's).  Loads whose float4 would hold nothing needed are clamped to the last
  // float4 that holds a needed cell: in a y-halo row (whose +x halo cells are
  // corners, never used) the one that ends at or before the halo's end, so that the
  // last row of the last plane is never read past the array.
  const int xcl_in = (nx + 3) & ~3;  // interior rows: the float4 holding cell nx + 3
  const int xcl_halo = nx & ~3;      // y-halo rows
  auto xcl = [&](int yy) { return yy < ny ? xcl_in : xcl_halo; };
  // ---- the thread's own rows
  unsigned cb[RY];
  bool act[RY], full[RY];
#pragma unroll
  for (int r = 0; r < RY; ++r) {
    cb[r] = boff(x, yr + r);
    act[r] = (x < nx) && (yr + r < ny);  // some point of the float4 is stored
    full[r] = (x + 4 <= nx) && (yr + r < ny);
  }
  // ---- the halo float4 this thread loads per plane.  Waves 0-3 (thread rows 0-7)
  // load the y halo (row tr of the 8: 4 above the tile, 4 below), wave 4 (thread
  // rows 8-9) the x halo (32 rows x 2 sides), waves 5-7 nothing of use: they load
  // their own row's cell of the same plane instead, so that every wave issues the
  // same loads (a load that some waves skip makes the compiler wait for the
  // youngest loads of every wave).
  bool h_on = false;
  int h_lds = 0;
  int h_x = x, h_y = yr, h_side = 0;
  if (tr < 8) {
    h_on = true;
    h_y = tr < 4 ? y0 - 4 + tr : y0 + TY + (tr - 4);
    h_lds = (tr < 4 ? tr : TY + tr) * LX + 4 + 4 * lx;
  } else if (tr < 8 + XH) {
    const int idx = (tr - 8) * LANES + lx;
    h_on = true;
    h_side = idx & 1;
    h_x = h_side ? x0 + TX : x0 - 4;
    h_y = y0 + (idx >> 1);
    h_lds = (4 + (idx >> 1)) * LX + (h_side ? 4 + TX : 0);
  }
  // a halo cell past the grid's halo is only read by points that are not stored:
  // load a clamped one instead
  const unsigned h_off = boff(min(h_x, xcl(min(h_y, ny + 3))), min(h_y, ny + 3));

  const bool src_tile = p.si >= x0 && p.si < x0 + TX && p.sj >= y0 && p.sj < y0 + TY &&
                        p.sk >= kb && p.sk < ke;

  const long long org_c = p.g.org - 4LL * sy - 4;
  const char* F0 = reinterpret_cast<const char*>(p.u + org_c);
  const char* A0 = reinterpret_cast<const char*>(p.up + org_c);
  const char* B0 = reinterpret_cast<const char*>(p.q + org_c);
  char* O0 = reinterpret_cast<char*>(p.un + org_c);

  // halo source: u's own halo, or (XCH, first / last tile column) the receive
  // buffer of that face, whose rows are one float4 each
  // halo address: a scalar plane base and a 32-bit in-plane offset for u's own
  // halo; for a cell of a receive buffer (XCH) the buffer's base per lane and a
  // 32-bit offset (a face is at most 2^32 bytes: nz * ny * 16 < 2^32 is checked on
  // the host)
  const char* hrb = nullptr;  // XCH receive buffer of this lane, or NULL
  unsigned hro = 0;
  float* sx_ptr = nullptr;
  if (XCH) {
    if (h_on && tr >= 8 && h_y < ny) {  // rows past ny: corner cells no point uses
      if (h_side == 0 && bx == 0) hrb = reinterpret_cast<const char*>(p.rin[0]);
      else if (h_side == 1 && x0 + TX == nx) hrb = reinterpret_cast<const char*>(p.rin[1]);
      hro = 16u * (unsigned)h_y;
    }
    if (x == 0) sx_ptr = p.sout[0];
    else if (x == nx - 4) sx_ptr = p.sout[1];
  }
  // Every load below is unconditional (a predicated load makes the compiler wait
  // for all outstanding loads where its value is merged): a lane whose cell lies
  // outside what it must load reads a clamped cell instead, whose value only ever
  // reaches points that are not stored.
  auto hload = [&](int k) -> f4 {
    const int kk = min(k, nz - 1);
    if (XCH && hrb)
      return *reinterpret_cast<const f4*>(hrb + (hro + (unsigned)kk * (16u * (unsigned)ny)));
    return ld4(F0 + (long long)kk * szb, h_off);
  };
  unsigned cbz[RY], cbp[RY];  // clamped: field (interior + halo), pointwise (interior)
#pragma unroll
  for (int r = 0; r < RY; ++r) {
    const int yz = min(yr + r, ny + 3);
    cbz[r] = boff(min(x, xcl(yz)), yz);
    cbp[r] = boff(min(x, (nx - 1) & ~3), min(yr + r, ny - 1));
  }
  auto zload = [&](int k, int r) -> f4 {
    return ld4(F0 + (long long)min(k, nz + 3) * szb, cbz[r]);
  };

  // ---- rings, one slot larger than what is live, so that each load lands in a
  // dead slot and advancing a plane moves no registers (the z loop is unrolled 10
  // times): at ring position P (plane k), slot (P + s) % 10 of zq holds plane
  // k - 4 + s (s < 9) and hq the halo of the same plane (s >= 4); slot (P + 9) % 10
  // receives plane k + 5.  pa/pb[P % 2] hold u^{n-1} and vdt2 of plane k,
  // [(P + 1) % 2] receive plane k + 1.
  f4 zq[10][RY];
  f4 hq[10];
  f4 pa[2][RY], pb[2][RY];
  // eta_z of plane k, loaded with plane k's pointwise operands: a load issued just
  // before its use would make the compiler wait for every older load as well
  float ezq[2] = {0.f, 0.f};
  if (SPONGE) ezq[0] = p.ez[kb];
#pragma unroll
  for (int s = 0; s < 9; ++s) {
#pragma unroll
    for (int r = 0; r < RY; ++r) zq[s][r] = zload(kb - 4 + s, r);
    if (s >= 4) hq[s] = hload(kb - 4 + s);
  }
#pragma unroll
  for (int r = 0; r < RY; ++r) {
    pa[0][r] = ld4_nt(A0 + (long long)kb * szb, cbp[r]);
    pb[0][r] = ld4_nt(B0 + (long long)kb * szb, cbp[r]);
  }

  // ---- sponge factors constant along z (after the prologue's loads are issued, so
  // that their round trip overlaps the one of these tables)
  float exc[4] = {0.f, 0.f, 0.f, 0.f};
  float eyr[RY];
#pragma unroll
  for (int r = 0; r < RY; ++r) eyr[r] = 0.f;
  bool tile_sponge = false;
  if (SPONGE) {
#pragma unroll
    for (int e = 0; e < 4; ++e)
      if (x + e < nx) exc[e] = p.ex[x + e];
    int any = 0;
#pragma unroll
    for (int r = 0; r < RY; ++r) {
      if (yr + r < ny) eyr[r] = p.ey[yr + r];
#pragma unroll
      for (int e = 0; e < 4; ++e)
        any |= (x + e < nx) && (yr + r < ny) && (exc[e] != 0.f || eyr[r] != 0.f);
    }
    tile_sponge = __syncthreads_or(any) != 0;
  }
  // ---- receiver indices of the thread's points, if the chunk holds the receiver
  // plane (loaded here, long before that plane is stored, so that its stores wait
  // for nothing).  Not in the exchange form, whose receiver row is taken where the
  // faces are packed.
  const bool rec_chunk = FUSE && !XCH && !GRAD && p.rk >= kb && p.rk < ke;
  int rix[RY][4];
#pragma unroll
  for (int r = 0; r < RY; ++r)
#pragma unroll
    for (int e = 0; e < 4; ++e) rix[r][e] = -1;
  float rval[RY][4];  // radd: the row values to add there
#pragma unroll
  for (int r = 0; r < RY; ++r)
#pragma unroll
    for (int e = 0; e < 4; ++e) rval[r][e] = 0.f;
  if (rec_chunk) {
#pragma unroll
    for (int r = 0; r < RY; ++r)
#pragma unroll
      for (int e = 0; e < 4; ++e)
        if (x + e < nx && yr + r < ny) rix[r][e] = p.rmap[(long long)(yr + r) * nx + x + e];
    if (p.radd) {
#pragma unroll
      for (int r = 0; r < RY; ++r)
#pragma unroll
        for (int e = 0; e < 4; ++e)
          if (rix[r][e] >= 0) rval[r][e] = p.rrow[rix[r][e]];
    }
  }
  const Coef& c = p.c;
  auto iter = [&](auto pos, const int k) {
    constexpr int P = decltype(pos)::value;
    constexpr int C = (P + 4) % 10;  // slot of plane k
    constexpr int L = (P + 9) % 10;  // landing slot of plane k + 5
    constexpr int Q = P % 2;         // u^{n-1} and vdt2 of plane k
    const int buf = (k - kb) & 1;
    // ---- prefetch: plane k + 5 of the field and its halo, plane k + 1 of u^{n-1}
    // and vdt2 (clamped to the last plane: unused past the chunk)
#pragma unroll
    for (int r = 0; r < RY; ++r) zq[L][r] = zload(k + 5, r);
    hq[L] = hload(k + 5);
    {
      const long long kp = min(k + 1, nz - 1);
#pragma unroll
      for (int r = 0; r < RY; ++r) {
        pa[Q ^ 1][r] = ld4_nt(A0 + kp * szb, cbp[r]);
        pb[Q ^ 1][r] = ld4_nt(B0 + kp * szb, cbp[r]);
      }
      if (SPONGE) ezq[Q ^ 1] = p.ez[kp];
    }
    // ---- stage plane k in LDS
    float* s = sm[buf];
#pragma unroll
    for (int r = 0; r < RY; ++r)
      *reinterpret_cast<f4*>(s + (4 + RY * tr + r) * LX + 4 + 4 * lx) = zq[C][r];
    if (h_on) *reinterpret_cast<f4*>(s + h_lds) = hq[C];
    __syncthreads();

    // ---- compute
    const float ezk = SPONGE ? ezq[Q] : 0.f;
    const bool damped = SPONGE && (tile_sponge || ezk != 0.f);
    const bool src_plane = src_tile && k == p.sk;
    // rows -4..-1 and +2..+5 around the thread's first row, from LDS
    f4 yv[10];
#pragma unroll
    for (int d = -4; d <= 5; ++d) {
      if (d == 0 || d == 1) continue;
      yv[d + 4] = *reinterpret_cast<const f4*>(s + (4 + RY * tr + d) * LX + 4 + 4 * lx);
    }
    yv[4] = zq[C][0];
    yv[5] = zq[C][1];
    char* ok = O0 + (long long)k * szb;
#pragma unroll
    for (int r = 0; r < RY; ++r) {
      const float* row = s + (4 + RY * tr + r) * LX + 4 + 4 * lx;
      const f4 lf = *reinterpret_cast<const f4*>(row - 4);
      const f4 rt = *reinterpret_cast<const f4*>(row + 4);
      const f4 uc = zq[C][r];
      const f4 ua = pa[Q][r];
      const f4 ub = pb[Q][r];
      f4 v4;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        // x neighbour at offset o (-4..4) of element e
        auto X = [&](int o) -> float {
          const int j = e + o;
          return j < 0 ? lf[j + 4] : (j > 3 ? rt[j - 4] : uc[j]);
        };
        const float u0 = uc[e];
        float lap = c.cc * u0;
#pragma unroll
        for (int m = 1; m <= 4; ++m) lap += c.cx[m] * (X(m) + X(-m));
#pragma unroll
        for (int m = 1; m <= 4; ++m) lap += c.cy[m] * (yv[r + m + 4][e] + yv[r - m + 4][e]);
#pragma unroll
        for (int m = 1; m <= 4; ++m)
          lap += c.cz[m] * (zq[(C + m) % 10][r][e] + zq[(C + 10 - m) % 10][r][e]);
        float eta = 0.f;
        if (damped) eta = exc[e] + eyr[r] + ezk;
        float v;
        if constexpr (GRAD) {
          // g += D a (L u + f): ua is a^{n+1}, ub the accumulator (as the gradient
          // mode of the marching kernel, same rounding)
          float src = 0.f;
          if (src_plane && x + e == p.si && yr + r == p.sj) src = p.sw;
          float D = 1.f;
          if (damped && eta != 0.f) D = __builtin_amdgcn_rcpf(1.f + eta);
          v = ub[e] + D * ua[e] * (lap + src);
        } else {
          v = 2.f * u0 - ua[e] + ub[e] * lap;
          if (damped && eta != 0.f) v = (v + eta * ua[e]) * __builtin_amdgcn_rcpf(1.f + eta);
          if (FUSE && src_plane) {
            // no contraction: rounds exactly as inject_source
#pragma clang fp contract(off)
            if (x + e == p.si && yr + r == p.sj) v += ub[e] * p.sw / (1.f + eta);
          }
          if (rec_chunk && p.radd && k == p.rk && rix[r][e] >= 0) {
            // rounds as fd_scatter_add_scaled: the row value times vdt2 / (1+eta)
#pragma clang fp contract(off)
            v += rval[r][e] * (ub[e] / (1.f + eta));
          }
        }
        v4[e] = v;
      }
      if (rec_chunk && !p.radd && k == p.rk) {
#pragma unroll
        for (int e = 0; e < 4; ++e)
          if (rix[r][e] >= 0) p.rrow[rix[r][e]] = v4[e];
      }
      if (full[r]) {
        __builtin_nontemporal_store(v4, reinterpret_cast<f4*>(ok + cb[r]));
        if (XCH && sx_ptr)
          *reinterpret_cast<f4*>(sx_ptr + ((size_t)k * (size_t)ny + (size_t)(yr + r)) * 4) = v4;
      } else if (act[r]) {  // the row's last points: x < nx < x + 4
        float* d = reinterpret_cast<float*>(ok + cb[r]);
#pragma unroll
        for (int e = 0; e < 3; ++e)
          if (x + e < nx) __builtin_nontemporal_store(v4[e], d + e);
      }
    }
  };
  using std::integral_constant;
  for (int k = kb; k < ke; k += 10) {
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
    if (k + 9 >= ke) break;
    iter(integral_constant<int, 9>{}, k + 9);
  }
}

template <class SH, bool SPONGE, bool FUSE, bool XCH, bool GRAD = false>
__global__ void __launch_bounds__(SH::LANES * SH::TROWS) stencil4_kernel(P4 p) {
  const int logical = remap_block4(blockIdx.x, gridDim.x);
  const int bx = logical % p.tiles_x;
  const int rest = logical / p.tiles_x;
  stencil4_block<SH, SPONGE, FUSE, XCH, GRAD>(p, bx, rest % p.tiles_y, rest / p.tiles_y,
                                              threadIdx.x, threadIdx.y);
}

// Many grids in one launch: block b runs tile tiles[remap(b)] = (slot, bx, by, bz) of
// shot `slot` at its own step a.n[slot] (u^n in arr[n % 3]) with source amplitude
// a.w[slot]; every point runs exactly the code of stencil4_kernel.
__global__ void __launch_bounds__(LANES * TROWS) batched4_kernel(const BatchShot* __restrict__ shots,
                                                                 const int4* __restrict__ tiles,
                                                                 BatchStep a) {
  const int4 t = tiles[remap_block4(blockIdx.x, gridDim.x)];
  const BatchShot& b = shots[t.x];
  const int n = a.n[t.x];
  P4 p;
  p.g = b.g;
  p.c = b.c;
  p.u = b.arr[n % 3];
  p.up = b.arr[(n + 2) % 3];
  p.q = b.q;
  p.un = b.arr[(n + 1) % 3];
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
  p.rin[0] = p.rin[1] = nullptr;
  p.sout[0] = p.sout[1] = nullptr;
  p.rmap = b.rmap;
  p.rk = b.rmap ? b.rk : -1;
  p.rrow = b.traces + (size_t)n * (size_t)b.nrec;
  p.radd = false;  // the trace row is written, not added to
  p.narrow = false;
  stencil4_block<Wide128, true, true, false>(p, t.y, t.z, t.w, threadIdx.x, threadIdx.y);
}

// Up to kWideMulti grids in one launch, their parameters in the kernel arguments:
// grid i owns blocks [start[i], start[i+1]) (tiles in the order of stencil4_kernel);
// a block finds its grid by comparing uniform values, with no memory look-up before
// its first loads.  Each grid has its own tile shape: the block's 512 threads are
// 32 x 16 for 128 x 32 tiles and, renumbered in the same order, 16 x 32 for 64 x 64
// (the branch is uniform over the block; both shapes compute the same bits).
struct MultiArgs {
  int n;
  int start[kWideMulti + 1];
  P4 grid[kWideMulti];
};

__global__ void __launch_bounds__(LANES * TROWS) multi4_kernel(MultiArgs A) {
  const int b = remap_block4(blockIdx.x, gridDim.x);
  int i = 0;
  while (i + 1 < A.n && b >= A.start[i + 1]) ++i;
  const P4& p = A.grid[i];
  const int t = b - A.start[i];
  const int bx = t % p.tiles_x;
  const int rest = t / p.tiles_x;
  if (p.narrow) {
    const int lin = threadIdx.x + LANES * threadIdx.y;
    stencil4_block<Wide64, true, true, false>(p, bx, rest % p.tiles_y, rest / p.tiles_y,
                                              lin % Wide64::LANES, lin / Wide64::LANES);
  } else {
    stencil4_block<Wide128, true, true, false>(p, bx, rest % p.tiles_y, rest / p.tiles_y,
                                               threadIdx.x, threadIdx.y);
  }
}

template <class SH, bool SPONGE, bool FUSE, bool XCH, bool GRAD = false>
hipError_t launch4(P4 p, hipStream_t st) {
  // one block per CU: its 8 waves take a CU's share of 16 (more than 128 VGPRs)
  const LaunchShape sh = stencil_shape(p.g, 4 * SH::LANES, SH::TROWS * RY, 16);
  p.tiles_x = sh.tiles_x;
  p.tiles_y = sh.tiles_y;
  p.kchunk = sh.kchunk;
  const long long nb = (long long)sh.tiles_x * sh.tiles_y * sh.zchunks;
  if (nb <= 0 || nb > 0x7fffffffLL) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL((stencil4_kernel<SH, SPONGE, FUSE, XCH, GRAD>), dim3((unsigned)nb),
                     dim3(SH::LANES, SH::TROWS), 0, st, p);
  return hipGetLastError();
}

bool aligned16(const void* ptr) { return ((uintptr_t)ptr & 15u) == 0; }

}  // namespace

bool wide_forward_fits(const Geo& g, const float* const arrays[4], const float* const faces[4]) {
  // (a row's last float4 may end up to 3 cells past its +x halo: in the next row,
  // which exists, since y-halo rows clamp theirs to end within the halo)
  if (g.sy % 4 || g.sz % 4 || g.org % 4) return false;
  for (int i = 0; i < 4; ++i)
    if (!arrays[i] || !aligned16(arrays[i])) return false;
  if (faces) {
    // x faces are one float4 per row; a receive buffer cell is addressed by a
    // 32-bit byte offset
    if (g.nx % TX || (long long)g.ny * g.nz * 16 >= (1LL << 32)) return false;
    for (int i = 0; i < 4; ++i)
      if (!faces[i] || !aligned16(faces[i])) return false;
  }
  return true;
}

bool wide_takes_step(const Geo& g, const float* const arrays[4]) {
  return forward_wide_tiles(g) && wide_forward_fits(g, arrays, nullptr);
}

int batch4_tile_shape(int* tx, int* ty) {
  *tx = TX;
  *ty = TY;
  return 16;  // one block per CU: a CU's share of 16 waves
}

hipError_t launch_batched4(const BatchShot* shots, const int4* tiles, int ntiles,
                           const BatchStep& a, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(batched4_kernel, dim3((unsigned)ntiles), dim3(LANES, TROWS), 0, s, shots,
                     tiles, a);
  return hipGetLastError();
}

hipError_t launch_wide_multi(const WideStep* steps, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (n > kWideMulti) return hipErrorInvalidValue;
  // each grid's tile shape, then one z chunk for all the grids, from the launch
  // model over them
  long long xy[kWideMulti];
  int nz[kWideMulti];
  bool narrow[kWideMulti];
  for (int i = 0; i < n; ++i) {
    narrow[i] = wide_narrow_in_multi(steps[i].g);
    const int tx = narrow[i] ? 64 : TX, ty = narrow[i] ? 64 : TY;
    xy[i] = (long long)((steps[i].g.nx + tx - 1) / tx) * ((steps[i].g.ny + ty - 1) / ty);
    nz[i] = steps[i].g.nz;
  }
  const int kc = choose_kchunk(xy, nz, n, 16, 0, 0x7fffffffLL);
  MultiArgs A;
  A.n = n;
  A.start[0] = 0;
  for (int i = 0; i < n; ++i) {
    const WideStep& w = steps[i];
    P4& p = A.grid[i];
    p = P4{};
    p.g = w.g;
    p.c = w.c;
    p.u = w.u;
    p.up = w.up;
    p.q = w.q;
    p.un = w.un;
    p.ex = w.ex;
    p.ey = w.ey;
    p.ez = w.ez;
    p.narrow = narrow[i];
    p.tiles_x = (w.g.nx + (narrow[i] ? 64 : TX) - 1) / (narrow[i] ? 64 : TX);
    p.tiles_y = (w.g.ny + (narrow[i] ? 64 : TY) - 1) / (narrow[i] ? 64 : TY);
    p.kchunk = std::min(kc, w.g.nz);
    p.si = w.src.i;
    p.sj = w.src.j;
    p.sk = w.src.k;
    p.sw = w.src.w;
    p.rmap = w.rec.map;
    p.rk = w.rec.map ? w.rec.k : -1;
    p.rrow = w.rec.row;
    const long long blocks =
        (long long)p.tiles_x * p.tiles_y * ((w.g.nz + p.kchunk - 1) / p.kchunk);
    if ((long long)A.start[i] + blocks > 0x7fffffffLL) return hipErrorInvalidConfiguration;
    A.start[i + 1] = A.start[i] + (int)blocks;
  }
  for (int i = n + 1; i <= kWideMulti; ++i) A.start[i] = A.start[n];
  hipLaunchKernelGGL(multi4_kernel, dim3((unsigned)A.start[n]), dim3(LANES, TROWS), 0, s, A);
  return hipGetLastError();
}

hipError_t launch_grad_wide(const Geo& g, const Coef& c, const float* u, const float* an1,
                            float* gq, const float* ex, const float* ey, const float* ez,
                            const fd_source* src, hipStream_t s) {
  P4 p{};
  p.g = g;
  p.c = c;
  p.u = u;
  p.up = an1;
  p.q = gq;
  p.un = gq;
  p.ex = ex;
  p.ey = ey;
  p.ez = ez;
  p.si = p.sj = p.sk = -1;
  p.sw = 0.f;
  p.rk = -1;
  if (src) {
    p.si = src->i;
    p.sj = src->j;
    p.sk = src->k;
    p.sw = src->w;
  }
  if (wide_narrow_tiles(g)) {
    if (ex) return launch4<Wide64, true, false, false, true>(p, s);
    return launch4<Wide64, false, false, false, true>(p, s);
  }
  if (ex) return launch4<Wide128, true, false, false, true>(p, s);
  return launch4<Wide128, false, false, false, true>(p, s);
}

bool wide_narrow_tiles(const Geo& g) {
  const int mode = tile_override();
  if (mode == 5) return true;
  if (mode == 4) return false;
  // 64 x 64 where they cut the modelled launch time by a tenth: where a 128-wide
  // tile column would be mostly empty (nx = 257: 3 columns of 128, 5 of 64)
  return stencil_cost(g, 64, 64, 16) < 0.9 * stencil_cost(g, TX, TY, 16);
}

bool wide_narrow_in_multi(const Geo& g) {
  const int mode = tile_override();
  if (mode == 5) return true;
  if (mode == 4) return false;
  // in a launch shared with other grids only the tiles' area counts: 64 x 64 where
  // it covers the plane with a tenth fewer points than 128 x 32
  const long long a128 = (long long)((g.nx + TX - 1) / TX) * TX * (((g.ny + TY - 1) / TY) * TY);
  const long long a64 = (long long)((g.nx + 63) / 64) * 64 * (((g.ny + 63) / 64) * 64);
  return 10 * a64 < 9 * a128;
}

void wide_forward_shape(const Geo& g, int out[4]) {
  const bool narrow = wide_narrow_tiles(g);
  const LaunchShape sh = stencil_shape(g, narrow ? 64 : TX, narrow ? 64 : TY, 16);
  out[0] = sh.tiles_x;
  out[1] = sh.tiles_y;
  out[2] = sh.kchunk;
  out[3] = sh.zchunks;
}

hipError_t launch_forward_wide(const Geo& g, const Coef& c, const float* up, const float* u,
                               float* un, const float* q, const float* ex, const float* ey,
                               const float* ez, const fd_source* src, const float* const rin[2],
                               float* const sout[2], hipStream_t s, const RecPlane* rp) {
  P4 p{};
  p.g = g;
  p.c = c;
  p.u = u;
  p.up = up;
  p.q = q;
  p.un = un;
  p.ex = ex;
  p.ey = ey;
  p.ez = ez;
  p.si = p.sj = p.sk = -1;
  p.sw = 0.f;
  p.rk = -1;
  if (rp && rp->map) {
    p.rmap = rp->map;
    p.rk = rp->k;
    p.rrow = rp->row;
    p.radd = rp->add;
  }
  if (src) {
    p.si = src->i;
    p.sj = src->j;
    p.sk = src->k;
    p.sw = src->w;
  }
  const bool xch = rin != nullptr;
  if (xch) {
    for (int f = 0; f < 2; ++f) {
      p.rin[f] = rin[f];
      p.sout[f] = sout[f];
    }
  }
  const bool sponge = ex != nullptr;
  if (xch) {
    if (sponge) return launch4<Wide128, true, true, true>(p, s);
    return launch4<Wide128, false, true, true>(p, s);
  }
  const bool fuse = src || p.rmap;
  if (wide_narrow_tiles(g)) {
    if (fuse) {
      if (sponge) return launch4<Wide64, true, true, false>(p, s);
      return launch4<Wide64, false, true, false>(p, s);
    }
    if (sponge) return launch4<Wide64, true, false, false>(p, s);
    return launch4<Wide64, false, false, false>(p, s);
  }
  if (fuse) {
    if (sponge) return launch4<Wide128, true, true, false>(p, s);
    return launch4<Wide128, false, true, false>(p, s);
  }
  if (sponge) return launch4<Wide128, true, false, false>(p, s);
  return launch4<Wide128, false, false, false>(p, s);
}

}  // namespace fd
