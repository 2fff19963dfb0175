// fd_gemm.hip -- the local block product of Cannon's matrix multiply on gfx950.
//
// In Cannon's algorithm each of P ranks holds row stripes of Ns = N/P rows and, at
// each of its P steps, multiplies an Ns x Ns block of its A stripe with the B
// stripe it holds, adding the N * Ns * Ns multiply-adds into its C stripe
// (Sec. 4.4).  That step is C = C + A B, a dense contraction, so it runs on the
// FP64 matrix cores (v_mfma_f64_16x16x4f64): the paper states no element type,
// and FP64 is the precision of the oracle that defines the product.
//
// Block: 1024 threads (16 waves), a 256 x 128 tile of C; each wave owns a 32 x 64
// piece as 2 x 4 MFMA tiles of 16 x 16 (8 independent accumulators of 4 doubles per
// lane), so that four waves share each SIMD and one's LDS and barrier phases hide
// behind the others' MFMAs.  The K loop takes 16 columns of A and 16 rows of B per stage, staged in
// double-buffered LDS; the next stage is loaded into registers while the MFMAs of the
// current one run.
// Operands of any shape and leading dimension: K is split into a first stage of
// 1..16 columns, whose loads past K read 0, and whole stages, whose loads need no
// bounds arithmetic (a pointer per thread plus the stage's offset); rows past m and
// columns past n are read clamped and their results not stored.  Blocks sharing a B
// panel (a column of tiles) run on one XCD in succession, so that the panel is read
// from HBM about once.
#include <stdint.h>

#include <algorithm>

#include "fd.h"
#include "fd_internal.h"

namespace fd {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int BM = 256;          // tile rows (M)
constexpr int BN = 128;          // tile columns (N)
constexpr int BK = 16;           // K per stage
constexpr int WTM = 32;          // wave tile rows
constexpr int WTN = 64;          // wave tile columns
constexpr int WAVES_N = BN / WTN;
constexpr int GT = 64 * (BM / WTM) * WAVES_N;  // threads per block
constexpr int FM = WTM / 16;     // MFMA tiles per wave, rows
constexpr int FN = WTN / 16;     // MFMA tiles per wave, columns
// LDS pitches (doubles), chosen so that the 64 lanes of a fragment read (16 rows or
// columns x 4 k) fall on distinct banks in each half-wave: A is kept row-major [m][k]
// with pitch 18 (36 fr + 2 fk distinct mod 64 dwords), B as [k][n] with pitch 144
// (consecutive k 32 banks apart).
constexpr int SA = BK + 2;
constexpr int SB = BN + 16;
// waves per SIMD the register budget must allow (the second __launch_bounds__
// argument): one block of 16 waves per CU (LDS 110.6 KB of 160 KB), at most 128
// VGPRs per lane
constexpr int WAVES_PER_SIMD = 4;
constexpr int A_PER = BM * BK / GT;  // A elements a thread loads per stage
constexpr int B_PER = BK * BN / GT;  // B elements a thread loads per stage

struct GemmArgs {
  int64_t m, n, k;
  const double* a;
  int64_t lda;
  const double* b;
  int64_t ldb;
  double* c;
  int64_t ldc;
  int tiles_m;
  int accumulate;
};

// Blocks b, b+8, b+16, ... run on one XCD; give each XCD a contiguous run of
// logical tiles (row tiles fastest: the tiles of one B panel).
__device__ __forceinline__ int remap_gemm(int bid, int nb) {
  const int per = nb >> 3;
  if (bid < (per << 3)) return (bid & 7) * per + (bid >> 3);
  return bid;
}

__global__ void __launch_bounds__(GT, WAVES_PER_SIMD) gemm_f64_kernel(GemmArgs g) {
  __shared__ double sa[2][BM * SA];
  __shared__ double sb[2][BK * SB];

  const int logical = remap_gemm(blockIdx.x, gridDim.x);
  const int64_t m0 = (int64_t)(logical % g.tiles_m) * BM;
  const int64_t n0 = (int64_t)(logical / g.tiles_m) * BN;
  const int t = threadIdx.x;
  const int lane = t & 63;
  const int w = t >> 6;
  const int wm = (w / WAVES_N) * WTM;
  const int wn = (w % WAVES_N) * WTN;

  // stage loads: A as BK consecutive k of rows t / BK + (GT / BK) i; B as BN
  // consecutive columns of rows t / BN + (GT / BN) i (each instruction: 4 rows of 128
  // bytes of A, 512 contiguous bytes of B)
  const int ak = t % BK;
  const int ar = t / BK;
  const int bc = t % BN;
  const int br = t / BN;
  // K is taken as a first stage of kt = k - (stages - 1) BK columns (1..BK), then
  // whole stages of BK.  Rows of A past m and columns of B past n are read clamped and
  // not cleared: they only reach rows and columns of the tile that are not stored.
  // Only the first stage clears what lies past its kt columns (in both operands: 0 x
  // Inf would be NaN).  So a load of a whole stage is a per-thread pointer plus the
  // stage's uniform offset, with no bounds arithmetic, and every load is unconditional
  // (a load under a branch would make the compiler wait for it where the branch joins).
  const int64_t stages = (g.k + BK - 1) / BK;
  const int64_t kt = g.k - (stages - 1) * BK;
  const double* pa[A_PER];
  const double* pb[B_PER];
  const int64_t bcol = std::min(n0 + bc, g.n - 1);
#pragma unroll
  for (int i = 0; i < A_PER; ++i)  // (k < BK: a single stage, read clamped in K)
    pa[i] = g.a + std::min(m0 + ar + (GT / BK) * i, g.m - 1) * g.lda +
            std::min<int64_t>(ak, g.k - 1);
#pragma unroll
  for (int i = 0; i < B_PER; ++i)
    pb[i] = g.b + std::min<int64_t>(br + (GT / BN) * i, g.k - 1) * g.ldb + bcol;
  double ra[A_PER], rb[B_PER];
  // whole stage at column k0 = kt + (s - 1) BK of A, row k0 of B (s >= 1)
  auto load_stage = [&](int64_t k0) {
    const int64_t boff = k0 * g.ldb;
#pragma unroll
    for (int i = 0; i < A_PER; ++i) ra[i] = pa[i][k0];
#pragma unroll
    for (int i = 0; i < B_PER; ++i) rb[i] = pb[i][boff];
  };
  auto store_stage = [&](int buf) {
#pragma unroll
    for (int i = 0; i < A_PER; ++i) sa[buf][(ar + (GT / BK) * i) * SA + ak] = ra[i];
#pragma unroll
    for (int i = 0; i < B_PER; ++i) sb[buf][(br + (GT / BN) * i) * SB + bc] = rb[i];
  };

  d4 acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};

  if (stages > 0) {
    // the first stage: columns 0 .. kt-1 of A and rows 0 .. kt-1 of B, the rest 0
    // (a cleared element reads the stage's last valid one, in bounds)
#pragma unroll
    for (int i = 0; i < A_PER; ++i) {
      const double x = g.a[std::min(m0 + ar + (GT / BK) * i, g.m - 1) * g.lda +
                           std::min<int64_t>(ak, kt - 1)];
      ra[i] = ak < kt ? x : 0.0;
    }
#pragma unroll
    for (int i = 0; i < B_PER; ++i) {
      const int64_t row = br + (GT / BN) * i;
      const double x = g.b[std::min(row, kt - 1) * g.ldb + bcol];
      rb[i] = row < kt ? x : 0.0;
    }
    store_stage(0);
  }
  __syncthreads();
  // fragment lanes: A rows / B columns lane % 16 of a 16-wide tile, k = lane / 16
  const int fr = lane & 15;
  const int fk = lane >> 4;
  for (int64_t s = 0; s < stages; ++s) {
    const int buf = (int)(s & 1);
    // the next stage's loads, unconditional (the last iteration reloads its own
    // stage into the buffer nobody reads again): a load under a branch would make
    // the compiler wait for it where the branch joins, before the MFMAs
    load_stage(std::max<int64_t>(kt + (std::min(s + 1, stages - 1) - 1) * BK, 0));
    const double* A = sa[buf];
    const double* B = sb[buf];
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      double af[FM], bf[FN];
#pragma unroll
      for (int i = 0; i < FM; ++i) af[i] = A[(wm + 16 * i + fr) * SA + kk + fk];
#pragma unroll
      for (int j = 0; j < FN; ++j) bf[j] = B[(kk + fk) * SB + wn + 16 * j + fr];
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i], bf[j], acc[i][j], 0, 0, 0);
    }
    store_stage(buf ^ 1);
    __syncthreads();
  }

  // accumulator element v of lane l holds row l / 16 + 4 v, column l % 16 of its
  // 16 x 16 tile (the lane layout of v_mfma_f64_16x16x4f64, checked with one-hot
  // operands on the device)
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      const int64_t col = n0 + wn + 16 * j + fr;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t row = m0 + wm + 16 * i + fk + 4 * v;
        if (row < g.m && col < g.n) {
          double* p = g.c + row * g.ldc + col;
          *p = g.accumulate ? *p + acc[i][j][v] : acc[i][j][v];
        }
      }
    }
}

// Last byte (exclusive) a row-major rows x cols operand with leading dimension ld
// occupies, from its first element.
int64_t extent_bytes(int64_t rows, int64_t cols, int64_t ld) {
  if (rows <= 0 || cols <= 0) return 0;
  return 8 * ((rows - 1) * ld + cols);
}

bool ranges_overlap(const void* p, int64_t pn, const void* q, int64_t qn) {
  if (pn <= 0 || qn <= 0) return false;
  const char* a = static_cast<const char*>(p);
  const char* b = static_cast<const char*>(q);
  return a < b + qn && b < a + pn;
}

}  // namespace
}  // namespace fd

using namespace fd;

extern "C" int fd_block_gemm_f64(int64_t m, int64_t n, int64_t k, const double* a, int64_t lda,
                                 const double* b, int64_t ldb, double* c, int64_t ldc,
                                 int32_t accumulate, void* stream) {
  if (m < 0 || n < 0 || k < 0) return fail(FD_EINVAL, "fd_block_gemm_f64: negative extent");
  if (m == 0 || n == 0) return FD_OK;
  if (!c) return fail(FD_EINVAL, "fd_block_gemm_f64: c is NULL");
  if (ldc < n) return fail(FD_EINVAL, "fd_block_gemm_f64: ldc < n");
  if (k > 0) {
    if (!a || !b) return fail(FD_EINVAL, "fd_block_gemm_f64: a or b is NULL");
    if (lda < k || ldb < n) return fail(FD_EINVAL, "fd_block_gemm_f64: lda < k or ldb < n");
    const int64_t cb = extent_bytes(m, n, ldc);
    if (ranges_overlap(c, cb, a, extent_bytes(m, k, lda)) ||
        ranges_overlap(c, cb, b, extent_bytes(k, n, ldb)))
      return fail(FD_EINVAL, "fd_block_gemm_f64: c overlaps a or b");
  }
  const int64_t tm = (m + BM - 1) / BM;
  const int64_t tn = (n + BN - 1) / BN;
  if (tm * tn > 0x7fffffffLL || tm > 0x7fffffffLL)
    return fail(FD_EINVAL, "fd_block_gemm_f64: too many tiles");
  GemmArgs g;
  g.m = m;
  g.n = n;
  g.k = k;
  g.a = a;
  g.lda = lda;
  g.b = b;
  g.ldb = ldb;
  g.c = c;
  g.ldc = ldc;
  g.tiles_m = (int)tm;
  g.accumulate = accumulate ? 1 : 0;
  hipLaunchKernelGGL(gemm_f64_kernel, dim3((unsigned)(tm * tn)), dim3(GT), 0,
                     reinterpret_cast<hipStream_t>(stream), g);
  return check_hip(hipGetLastError(), "fd_block_gemm_f64 launch");
}
