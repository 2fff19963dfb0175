// fd_aux.hip -- the small kernels around the stencil: halo face pack/unpack,
// source injection, receiver sampling, adjoint residual scatter, model prep
// (vdt2 and max velocity) and the gradient's change of variable.
#include <algorithm>
#include <mutex>

#include "fd_internal.h"

namespace fd {
namespace {

constexpr int BS = 256;

struct Faces {
  float* p[6];
};
struct CFaces {
  const float* p[6];
};

__device__ __forceinline__ long long face_count(const Geo& g, int face) {
  if (face < 2) return 4LL * g.ny * g.nz;
  if (face < 4) return 4LL * g.nx * g.nz;
  return 4LL * g.nx * g.ny;
}

// Interior coordinates (i,j,k) of element e of face buffer `face` in the
// layouts of halo_pack; `q` in 0..3 counts planes from the lower index.
__device__ __forceinline__ void face_coord(const Geo& g, int face, unsigned e, int& q, int& a,
                                           int& b) {
  if (face < 2) {  // [nz][ny][4]: a = j, b = k
    q = e & 3u;
    const unsigned t = e >> 2;
    a = t % (unsigned)g.ny;
    b = t / (unsigned)g.ny;
  } else if (face < 4) {  // [nz][4][nx]: a = i, b = k
    a = e % (unsigned)g.nx;
    const unsigned t = e / (unsigned)g.nx;
    q = t & 3u;
    b = t >> 2;
  } else {  // [4][ny][nx]: a = i, b = j
    a = e % (unsigned)g.nx;
    const unsigned t = e / (unsigned)g.nx;
    b = t % (unsigned)g.ny;
    q = t / (unsigned)g.ny;
  }
}

__device__ __forceinline__ long long at(const Geo& g, int i, int j, int k) {
  return g.org + (long long)k * g.sz + (long long)j * g.sy + i;
}

__global__ void __launch_bounds__(BS) pack_kernel(Geo g, const float* __restrict__ u, Faces f) {
  const int face = blockIdx.y;
  float* __restrict__ dst = f.p[face];
  if (!dst) return;
  const unsigned n = (unsigned)face_count(g, face);
  for (unsigned e = blockIdx.x * BS + threadIdx.x; e < n; e += gridDim.x * BS) {
    int q, a, b;
    face_coord(g, face, e, q, a, b);
    long long src;
    switch (face) {
      case 0: src = at(g, q, a, b); break;
      case 1: src = at(g, g.nx - 4 + q, a, b); break;
      case 2: src = at(g, a, q, b); break;
      case 3: src = at(g, a, g.ny - 4 + q, b); break;
      case 4: src = at(g, a, b, q); break;
      default: src = at(g, a, b, g.nz - 4 + q); break;
    }
    dst[e] = u[src];
  }
}

__global__ void __launch_bounds__(BS) unpack_kernel(Geo g, float* __restrict__ u, CFaces f) {
  const int face = blockIdx.y;
  const float* __restrict__ src = f.p[face];
  if (!src) return;
  const unsigned n = (unsigned)face_count(g, face);
  for (unsigned e = blockIdx.x * BS + threadIdx.x; e < n; e += gridDim.x * BS) {
    int q, a, b;
    face_coord(g, face, e, q, a, b);
    long long dst;
    switch (face) {
      case 0: dst = at(g, q - 4, a, b); break;
      case 1: dst = at(g, g.nx + q, a, b); break;
      case 2: dst = at(g, a, q - 4, b); break;
      case 3: dst = at(g, a, g.ny + q, b); break;
      case 4: dst = at(g, a, b, q - 4); break;
      default: dst = at(g, a, b, g.nz + q); break;
    }
    u[dst] = src[e];
  }
}

// 16-byte form of pack/unpack for the default layout (origin, strides and nx
// multiples of 4 floats): each thread moves four consecutive x points.  Element
// offset in u of the first of the four points that float4 e4 of `face` covers;
// `halo` selects the unpack destination (the halo) instead of the pack source.
__device__ __forceinline__ long long face4_at(const Geo& g, int face, unsigned e4, bool halo) {
  const unsigned nx4 = (unsigned)g.nx >> 2;
  int i, j, k;
  if (face < 2) {  // [nz][ny][4]: one float4 per (j, k)
    j = e4 % (unsigned)g.ny;
    k = e4 / (unsigned)g.ny;
    i = face == 0 ? (halo ? -4 : 0) : (halo ? g.nx : g.nx - 4);
  } else if (face < 4) {  // [nz][4][nx]
    const unsigned t = e4 / nx4;
    const int q = t & 3u;
    i = 4 * (int)(e4 % nx4);
    k = t >> 2;
    j = face == 2 ? (halo ? q - 4 : q) : (halo ? g.ny + q : g.ny - 4 + q);
  } else {  // [4][ny][nx]
    const unsigned t = e4 / nx4;
    const int q = t / (unsigned)g.ny;
    i = 4 * (int)(e4 % nx4);
    j = t % (unsigned)g.ny;
    k = face == 4 ? (halo ? q - 4 : q) : (halo ? g.nz + q : g.nz - 4 + q);
  }
  return at(g, i, j, k);
}

__global__ void __launch_bounds__(BS) pack4_kernel(Geo g, const float* __restrict__ u, Faces f) {
  const int face = blockIdx.y;
  float4* __restrict__ dst = reinterpret_cast<float4*>(f.p[face]);
  if (!dst) return;
  const unsigned n4 = (unsigned)(face_count(g, face) >> 2);
  for (unsigned e = blockIdx.x * BS + threadIdx.x; e < n4; e += gridDim.x * BS)
    dst[e] = *reinterpret_cast<const float4*>(u + face4_at(g, face, e, false));
}

// pack4_kernel with a seventh row of blocks that samples the receivers
// (out[r] = u[off[r]]), so a step's pack and receiver row take one launch.
__global__ void __launch_bounds__(BS) pack4_record_kernel(Geo g, const float* __restrict__ u,
                                                          Faces f,
                                                          const int64_t* __restrict__ off,
                                                          int n, float* __restrict__ out) {
  const int face = blockIdx.y;
  if (face == 6) {
    for (int r = blockIdx.x * BS + threadIdx.x; r < n; r += gridDim.x * BS) out[r] = u[off[r]];
    return;
  }
  float4* __restrict__ dst = reinterpret_cast<float4*>(f.p[face]);
  if (!dst) return;
  const unsigned n4 = (unsigned)(face_count(g, face) >> 2);
  for (unsigned e = blockIdx.x * BS + threadIdx.x; e < n4; e += gridDim.x * BS)
    dst[e] = *reinterpret_cast<const float4*>(u + face4_at(g, face, e, false));
}

__global__ void __launch_bounds__(BS) unpack4_kernel(Geo g, float* __restrict__ u, CFaces f) {
  const int face = blockIdx.y;
  const float4* __restrict__ src = reinterpret_cast<const float4*>(f.p[face]);
  if (!src) return;
  const unsigned n4 = (unsigned)(face_count(g, face) >> 2);
  for (unsigned e = blockIdx.x * BS + threadIdx.x; e < n4; e += gridDim.x * BS)
    *reinterpret_cast<float4*>(u + face4_at(g, face, e, true)) = src[e];
}

bool vec4_ok(const Geo& g, const void* u, const void* const* face) {
  if ((g.org | g.sy | g.sz | g.nx) & 3) return false;
  if (reinterpret_cast<uintptr_t>(u) & 15) return false;
  for (int i = 0; i < 6; ++i)
    if (reinterpret_cast<uintptr_t>(face[i]) & 15) return false;
  return true;
}

__global__ void inject_kernel(float* un, const float* q, const float* ex, const float* ey,
                              const float* ez, long long o, int i, int j, int k, float w) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  {
#pragma clang fp contract(off)  // rounds as the source term fused into the stencil
    float eta = 0.f;
    if (ex) eta = ex[i] + ey[j] + ez[k];
    un[o] += q[o] * w / (1.f + eta);
  }
}

__global__ void __launch_bounds__(BS) record_kernel(const float* __restrict__ u,
                                                    const int64_t* __restrict__ off, int n,
                                                    float* __restrict__ out) {
  const int r = blockIdx.x * BS + threadIdx.x;
  if (r < n) out[r] = u[off[r]];
}

// a[off[r]] += vals[r] * Q / (1 + eta) at the point, eta from its interior
// coordinates (recovered from the offset; an offset outside the interior takes
// eta = 0).
__global__ void __launch_bounds__(BS) scatter_add_scaled_kernel(Geo g, float* a,
                                                                const int64_t* __restrict__ off,
                                                                const float* __restrict__ vals,
                                                                const float* __restrict__ q,
                                                                const float* ex, const float* ey,
                                                                const float* ez, int n) {
  const int r = blockIdx.x * BS + threadIdx.x;
  if (r >= n) return;
  const long long o = off[r];
  float w = q[o];
  if (ex) {
    const long long t = o - g.org;
    if (t >= 0) {
      const long long k = t / g.sz;
      const long long rem = t - k * g.sz;
      const long long j = rem / g.sy;
      const long long i = rem - j * g.sy;
      if (k < g.nz && j < g.ny && i < g.nx) w = w / (1.f + (ex[i] + ey[j] + ez[k]));
    }
  }
  atomicAdd(a + o, vals[r] * w);
}

__global__ void __launch_bounds__(BS) scatter_add_kernel(float* a, const int64_t* __restrict__ off,
                                                         const float* __restrict__ vals, int n) {
  const int r = blockIdx.x * BS + threadIdx.x;
  if (r < n) atomicAdd(a + off[r], vals[r]);
}

// One thread per element of the padded box [-4,n+4)^3 in each of PREP_K planes,
// one block row per (j, k-group): interior from v, face halo from the periodic image,
// edges 0.  v0 points at interior (0,0,0) of the input, which has its own strides.
// The PREP_K planes' loads are issued before any store, so that a thread keeps
// several loads in flight (one per thread left the 224 MB read of a 384^3 model
// latency-bound at about 3 TB/s).
constexpr int PREP_K = 4;

__device__ __forceinline__ int wrap_index(int a, int n) {
  int c = a < 0 ? a + n : (a >= n ? a - n : a);
  // a face halo wider than the axis wraps more than once
  while (c < 0) c += n;
  while (c >= n) c -= n;
  return c;
}

__global__ void __launch_bounds__(BS) prep_vdt2_kernel(Geo g, const float* __restrict__ v0,
                                                       long long vsy, long long vsz,
                                                       float* __restrict__ q, double dt,
                                                       bool from_m) {
  const int jj = blockIdx.y - 4;                  // j in [-4, ny+4)
  const int k0 = (int)blockIdx.z * PREP_K - 4;    // first k of the group, in [-4, nz+4)
  const int oj = (jj < 0) + (jj >= g.ny);
  const int cj = wrap_index(jj, g.ny);
  for (int ii = (int)(blockIdx.x * BS + threadIdx.x) - 4; ii < g.nx + 4; ii += gridDim.x * BS) {
    const int oi = (ii < 0) + (ii >= g.nx);
    const int ci = wrap_index(ii, g.nx);
    float vin[PREP_K];
    bool use[PREP_K];
#pragma unroll
    for (int t = 0; t < PREP_K; ++t) {
      const int kk = k0 + t;
      const int ok = (kk < 0) + (kk >= g.nz);
      use[t] = kk < g.nz + 4 && oi + oj + ok <= 1;
      vin[t] = use[t] ? v0[(long long)wrap_index(kk, g.nz) * vsz + (long long)cj * vsy + ci] : 0.f;
    }
#pragma unroll
    for (int t = 0; t < PREP_K; ++t) {
      const int kk = k0 + t;
      if (kk >= g.nz + 4) break;
      float val = 0.f;
      if (use[t]) {
        if (from_m) {
          val = (float)(dt * dt / (double)vin[t]);
        } else {
          const double vv = (double)vin[t] * dt;
          val = (float)(vv * vv);
        }
      }
      q[at(g, ii, jj, kk)] = val;
    }
  }
}

__global__ void vmax_init_kernel(int32_t* out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    out[0] = 0;           // max of the float bit patterns (positive floats order as ints)
    out[1] = 0x7f800000;  // min, starting at +inf
  }
}

__device__ __forceinline__ int wave_max(int v) {
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
  return v;
}
__device__ __forceinline__ int wave_min(int v) {
  for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o));
  return v;
}

// max and min of v (as float bit patterns: positive floats order as integers) over
// an nx x ny x nz view.  A block takes VMAX_LINES x-lines at a time (their row bases
// are uniform: no per-element division), so that a thread has VMAX_LINES loads in
// flight; lines past the last repeat the last one (no effect on max or min).  One
// atomic pair per block.
constexpr int VMAX_LINES = 8;

__global__ void __launch_bounds__(BS) vmax_kernel(int nx, int ny, int nz,
                                                  const float* __restrict__ v0, long long vsy,
                                                  long long vsz, int32_t* out) {
  const long long nline = (long long)ny * nz;
  int mx = 0, mn = 0x7f800000;
  for (long long l0 = (long long)blockIdx.x * VMAX_LINES; l0 < nline;
       l0 += (long long)gridDim.x * VMAX_LINES) {
    const float* row[VMAX_LINES];
#pragma unroll
    for (int u = 0; u < VMAX_LINES; ++u) {
      const long long line = min(l0 + u, nline - 1);
      const long long k = line / ny;
      row[u] = v0 + k * vsz + (line - k * ny) * vsy;
    }
    for (int i = threadIdx.x; i < nx; i += BS) {
      int bits[VMAX_LINES];
#pragma unroll
      for (int u = 0; u < VMAX_LINES; ++u) bits[u] = __float_as_int(row[u][i]);
#pragma unroll
      for (int u = 0; u < VMAX_LINES; ++u) {
        mx = max(mx, bits[u]);
        mn = min(mn, bits[u]);
      }
    }
  }
  mx = wave_max(mx);
  mn = wave_min(mn);
  __shared__ int red[2][BS / 64];
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    red[0][w] = mx;
    red[1][w] = mn;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < BS / 64; ++i) {
      mx = max(mx, red[0][i]);
      mn = min(mn, red[1][i]);
    }
    atomicMax(out, mx);
    atomicMin(out + 1, mn);
  }
}

// scaled: the accumulator holds sum b (L u + f) with b = Q D lambda, so that
// g_vdt2 = acc / Q and grad_m = -acc Q / dt^2; else acc = g_vdt2 and
// grad_m = -acc Q^2 / dt^2.  gm may be gq itself (in place: each thread reads and
// then writes its own element), so neither carries __restrict__.
__global__ void __launch_bounds__(BS) grad_finalize_kernel(Geo g, const float* gq,
                                                           const float* __restrict__ q, float s,
                                                           bool scaled, float* gm) {
  const int j = blockIdx.y;
  const int k = blockIdx.z;
  for (int i = blockIdx.x * BS + threadIdx.x; i < g.nx; i += gridDim.x * BS) {
    const long long o = at(g, i, j, k);
    const float qq = q[o];
    gm[o] = scaled ? -gq[o] * qq * s : -gq[o] * qq * qq * s;
  }
}

__global__ void __launch_bounds__(BS) zero_kernel(float* __restrict__ dst, long long n) {
  for (long long i = blockIdx.x * (long long)BS + threadIdx.x; i < n; i += (long long)gridDim.x * BS)
    dst[i] = 0.f;
}

// blockIdx.y = position in the active-slot list; x covers that shot's receivers.
// Runs after the batched step of the same BatchStep: u^{n+1} is in arr[(n+1) % 3].
__global__ void __launch_bounds__(BS) batched_record_kernel(const BatchShot* __restrict__ shots,
                                                            const int* __restrict__ slots,
                                                            BatchStep a) {
  const int slot = slots[blockIdx.y];
  const BatchShot& b = shots[slot];
  const int r = blockIdx.x * BS + threadIdx.x;
  if (r >= b.nrec) return;
  const int n = a.n[slot];
  b.traces[(long long)n * b.nrec + r] = b.arr[(n + 1) % 3][b.rec[r]];
}

unsigned blocks_for(long long n, unsigned cap) {
  long long b = (n + BS - 1) / BS;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return (unsigned)b;
}

}  // namespace

hipError_t launch_pack(const Geo& g, const float* u, float* const face[6], hipStream_t s) {
  Faces f;
  long long mx = 0;
  for (int i = 0; i < 6; ++i) {
    f.p[i] = face[i];
    const long long c = i < 2 ? 4LL * g.ny * g.nz : (i < 4 ? 4LL * g.nx * g.nz : 4LL * g.nx * g.ny);
    if (face[i] && c > mx) mx = c;
  }
  if (mx == 0) return hipSuccess;
  if (vec4_ok(g, u, reinterpret_cast<const void* const*>(face)))
    hipLaunchKernelGGL(pack4_kernel, dim3(blocks_for(mx / 4, 4096), 6), dim3(BS), 0, s, g, u, f);
  else
    hipLaunchKernelGGL(pack_kernel, dim3(blocks_for(mx, 4096), 6), dim3(BS), 0, s, g, u, f);
  return hipGetLastError();
}

hipError_t launch_pack_record(const Geo& g, const float* u, float* const face[6],
                              const int64_t* off, int n, float* out, hipStream_t s) {
  if (n <= 0) return launch_pack(g, u, face, s);
  long long mx = 0;
  Faces f;
  for (int i = 0; i < 6; ++i) {
    f.p[i] = face[i];
    const long long c = i < 2 ? 4LL * g.ny * g.nz : (i < 4 ? 4LL * g.nx * g.nz : 4LL * g.nx * g.ny);
    if (face[i] && c > mx) mx = c;
  }
  if (mx == 0 || !vec4_ok(g, u, reinterpret_cast<const void* const*>(face))) {
    const hipError_t e = launch_pack(g, u, face, s);
    return e == hipSuccess ? launch_record(u, off, n, out, s) : e;
  }
  const unsigned bx = std::max(blocks_for(mx / 4, 4096), (unsigned)((n + BS - 1) / BS));
  hipLaunchKernelGGL(pack4_record_kernel, dim3(bx, 7), dim3(BS), 0, s, g, u, f, off, n, out);
  return hipGetLastError();
}

hipError_t launch_unpack(const Geo& g, float* u, const float* const face[6], hipStream_t s) {
  CFaces f;
  long long mx = 0;
  for (int i = 0; i < 6; ++i) {
    f.p[i] = face[i];
    const long long c = i < 2 ? 4LL * g.ny * g.nz : (i < 4 ? 4LL * g.nx * g.nz : 4LL * g.nx * g.ny);
    if (face[i] && c > mx) mx = c;
  }
  if (mx == 0) return hipSuccess;
  if (vec4_ok(g, u, reinterpret_cast<const void* const*>(face)))
    hipLaunchKernelGGL(unpack4_kernel, dim3(blocks_for(mx / 4, 4096), 6), dim3(BS), 0, s, g, u,
                       f);
  else
    hipLaunchKernelGGL(unpack_kernel, dim3(blocks_for(mx, 4096), 6), dim3(BS), 0, s, g, u, f);
  return hipGetLastError();
}

hipError_t launch_inject(const Geo& g, float* un, const float* q, const float* ex,
                         const float* ey, const float* ez, int i, int j, int k, float w,
                         hipStream_t s) {
  const long long o = g.org + (long long)k * g.sz + (long long)j * g.sy + i;
  hipLaunchKernelGGL(inject_kernel, dim3(1), dim3(64), 0, s, un, q, ex, ey, ez, o, i, j, k, w);
  return hipGetLastError();
}

hipError_t launch_record(const float* u, const int64_t* off, int n, float* out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(record_kernel, dim3((n + BS - 1) / BS), dim3(BS), 0, s, u, off, n, out);
  return hipGetLastError();
}

hipError_t launch_scatter_add(float* a, const int64_t* off, const float* vals, int n,
                              hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(scatter_add_kernel, dim3((n + BS - 1) / BS), dim3(BS), 0, s, a, off, vals,
                     n);
  return hipGetLastError();
}

hipError_t launch_prepare_vdt2(const Geo& g, const float* v, float* q, double dt, bool from_m,
                               hipStream_t s) {
  const unsigned bx = blocks_for(g.nx + 8, 64);
  hipLaunchKernelGGL(prep_vdt2_kernel, dim3(bx, g.ny + 8, (g.nz + 8 + PREP_K - 1) / PREP_K),
                     dim3(BS), 0, s, g, v + g.org, (long long)g.sy, (long long)g.sz, q, dt,
                     from_m);
  return hipGetLastError();
}

hipError_t launch_prepare_vdt2_view(const Geo& g, const float* v, long long vsy, long long vsz,
                                    float* q, double dt, hipStream_t s) {
  const unsigned bx = blocks_for(g.nx + 8, 64);
  hipLaunchKernelGGL(prep_vdt2_kernel, dim3(bx, g.ny + 8, (g.nz + 8 + PREP_K - 1) / PREP_K),
                     dim3(BS), 0, s, g, v, vsy, vsz, q, dt, false);
  return hipGetLastError();
}

hipError_t launch_zero(float* dst, long long n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(zero_kernel, dim3(blocks_for(n, 8192)), dim3(BS), 0, s, dst, n);
  return hipGetLastError();
}

hipError_t launch_batched_record(const BatchShot* shots, const int* slots, int nslots,
                                 int max_nrec, const BatchStep& a, hipStream_t s) {
  if (nslots <= 0 || max_nrec <= 0) return hipSuccess;
  hipLaunchKernelGGL(batched_record_kernel, dim3((max_nrec + BS - 1) / BS, nslots), dim3(BS), 0,
                     s, shots, slots, a);
  return hipGetLastError();
}

hipError_t launch_vmax_view(int nx, int ny, int nz, const float* v, long long vsy,
                            long long vsz, int32_t* out, hipStream_t s) {
  hipLaunchKernelGGL(vmax_init_kernel, dim3(1), dim3(64), 0, s, out);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const long long groups = ((long long)ny * nz + VMAX_LINES - 1) / VMAX_LINES;
  const unsigned nb = (unsigned)std::min<long long>(std::max<long long>(groups, 1), 1024);
  hipLaunchKernelGGL(vmax_kernel, dim3(nb), dim3(BS), 0, s, nx, ny, nz, v, vsy, vsz, out);
  return hipGetLastError();
}

hipError_t launch_vmax(const Geo& g, const float* v, int32_t* out, hipStream_t s) {
  return launch_vmax_view(g.nx, g.ny, g.nz, v + g.org, g.sy, g.sz, out, s);
}

hipError_t launch_grad_finalize(const Geo& g, const float* gq, const float* q, double dt,
                                bool scaled, float* gm, hipStream_t s) {
  const float sc = (float)(1.0 / (dt * dt));
  hipLaunchKernelGGL(grad_finalize_kernel, dim3(blocks_for(g.nx, 64), g.ny, g.nz), dim3(BS), 0,
                     s, g, gq, q, sc, scaled, gm);
  return hipGetLastError();
}

hipError_t launch_scatter_add_scaled(const Geo& g, float* a, const int64_t* off,
                                     const float* vals, const float* q, const float* ex,
                                     const float* ey, const float* ez, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(scatter_add_scaled_kernel, dim3((n + BS - 1) / BS), dim3(BS), 0, s, g, a,
                     off, vals, q, ex, ey, ez, n);
  return hipGetLastError();
}

// ---- allocation-free max(v): the result slots live in a file-scope device array.
// Each device that runs the library holds its own copy until the process ends; its
// address is looked up once per device (hipGetSymbolAddress, with that device
// current) and only that address is handed to kernels and copies.  Every call on a
// device shares its copy: calls that overlap in time on one device race.
namespace {
static __device__ __align__(256) int32_t scratch[kCflScratchInts];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
int32_t* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t cfl_scratch(int32_t** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = static_cast<int32_t*>(ptr);
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

}  // namespace fd
