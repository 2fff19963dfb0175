// fd_abi.cpp -- the C ABI of libfd: argument validation, error reporting,
// geometry and the small host-side set-up helpers.  Every entry point checks
// its arguments before enqueuing anything and converts HIP errors to
// FD_EDEVICE; no C++ exception escapes.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <limits>
#include <new>

#include "fd_internal.h"

namespace fd {

static thread_local char t_err[512];

int fail(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(t_err, sizeof(t_err), fmt, ap);
  va_end(ap);
  return code;
}

int check_hip(hipError_t e, const char* what) {
  if (e == hipSuccess) return FD_OK;
  return fail(FD_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

// 8th-order weights (exact rationals) of the second derivative on unit spacing.
static const double kC[5] = {-205.0 / 72.0, 8.0 / 5.0, -1.0 / 5.0, 8.0 / 315.0, -1.0 / 560.0};

Coef make_coef(const fd_grid* g) {
  Coef c;
  const double ix = 1.0 / (g->dx * g->dx), iy = 1.0 / (g->dy * g->dy), iz = 1.0 / (g->dz * g->dz);
  c.cx[0] = c.cy[0] = c.cz[0] = 0.f;
  for (int m = 1; m <= 4; ++m) {
    c.cx[m] = (float)(kC[m] * ix);
    c.cy[m] = (float)(kC[m] * iy);
    c.cz[m] = (float)(kC[m] * iz);
  }
  c.cc = (float)(kC[0] * (ix + iy + iz));
  return c;
}

}  // namespace fd

using namespace fd;

namespace {

bool finite_pos(double d) { return isfinite(d) && d > 0.0; }

int check_grid(const fd_grid* g) {
  if (!g) return fail(FD_EINVAL, "grid is NULL");
  if (g->nx < 1 || g->ny < 1 || g->nz < 1)
    return fail(FD_EINVAL, "interior extent %d x %d x %d: each must be >= 1", g->nx, g->ny, g->nz);
  if (g->nx > (1 << 24) || g->ny > 65000 || g->nz > 65000)
    return fail(FD_EINVAL, "interior extent %d x %d x %d too large", g->nx, g->ny, g->nz);
  if (g->halo != FD_HALO) return fail(FD_EINVAL, "halo is %d, must be %d", g->halo, FD_HALO);
  if (g->ystride < (int64_t)g->nx + 8)
    return fail(FD_EINVAL, "ystride %lld < nx+8", (long long)g->ystride);
  if (g->zstride < g->ystride * ((int64_t)g->ny + 8))
    return fail(FD_EINVAL, "zstride %lld < ystride*(ny+8)", (long long)g->zstride);
  if (g->zstride > FD_MAX_ZSTRIDE)
    return fail(FD_EINVAL, "zstride %lld exceeds 2^29", (long long)g->zstride);
  if (g->origin < 4 * g->zstride + 4 * g->ystride + 4)
    return fail(FD_EINVAL, "origin %lld leaves no room for the halo", (long long)g->origin);
  if (!finite_pos(g->dx) || !finite_pos(g->dy) || !finite_pos(g->dz))
    return fail(FD_EINVAL, "grid spacing must be finite and > 0");
  return FD_OK;
}

int check_sponge(const fd_sponge* sp, const float** ex, const float** ey, const float** ez) {
  *ex = *ey = *ez = nullptr;
  if (!sp) return FD_OK;
  const int n = (sp->eta_x != nullptr) + (sp->eta_y != nullptr) + (sp->eta_z != nullptr);
  if (n == 0) return FD_OK;
  if (n != 3) return fail(FD_EINVAL, "sponge: give all three eta tables or none");
  *ex = sp->eta_x;
  *ey = sp->eta_y;
  *ez = sp->eta_z;
  return FD_OK;
}

int64_t last_elem(const fd_grid* g) {
  return g->origin + (int64_t)(g->nz + 3) * g->zstride + (int64_t)(g->ny + 3) * g->ystride +
         g->nx + 3;
}

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

// Two volume arrays of one grid overlap iff their padded extents intersect.
bool overlaps(const fd_grid* g, const float* a, const float* b) {
  if (!a || !b) return false;
  const int64_t n = last_elem(g) + 1;
  return a < b + n && b < a + n;
}

// The forward update with no faces inside the kernel: the one-thread-per-point
// kernel on grids small enough to stay in cache, else the z-marching kernel (the
// same bits either way).
hipError_t forward_update(const Geo& geo, const Coef& c, const float* up, const float* u,
                          float* un, const float* q, const float* ex, const float* ey,
                          const float* ez, const fd_source* src, hipStream_t s,
                          const RecPlane* rp = nullptr) {
  if (point_kernel_pays(geo)) return launch_step_point(geo, c, up, u, un, q, ex, ey, ez, src, rp, s);
  return launch_step(geo, c, up, u, un, q, ex, ey, ez, src, s, rp);
}

}  // namespace

extern "C" {

const char* fd_strerror(int code) {
  switch (code) {
    case FD_OK: return "success";
    case FD_ENOTFOUND: return "not found";
    case FD_EDEVICE: return "device (HIP) error";
    case FD_EAGAIN: return "not finished yet";
    case FD_ENOMEM: return "out of memory";
    case FD_EINVAL: return "invalid argument";
    case FD_ECANCELED: return "cancelled";
    default: return "unknown error code";
  }
}

const char* fd_last_error(void) { return t_err; }

int fd_version(void) { return 10200; }

int fd_grid_init(fd_grid* g, int32_t nx, int32_t ny, int32_t nz, double dx, double dy,
                 double dz) {
  if (!g) return fail(FD_EINVAL, "grid is NULL");
  fd_grid t;
  t.nx = nx;
  t.ny = ny;
  t.nz = nz;
  t.halo = FD_HALO;
  t.dx = dx;
  t.dy = dy;
  t.dz = dz;
  if (nx < 1 || ny < 1 || nz < 1) return fail(FD_EINVAL, "interior extent must be >= 1");
  const int64_t pad = 32;  // left padding: 128 bytes, the last 4 floats are the x halo
  const int64_t row = ((pad + nx + 4) + 31) / 32 * 32;
  t.ystride = row;
  t.zstride = row * ((int64_t)ny + 8);
  t.origin = 4 * t.zstride + 4 * t.ystride + pad;
  const int rc = check_grid(&t);
  if (rc != FD_OK) return rc;
  *g = t;
  return FD_OK;
}

int64_t fd_grid_elems(const fd_grid* g) {
  if (check_grid(g) != FD_OK) return -1;
  return last_elem(g) + 1;
}

int64_t fd_face_elems(const fd_grid* g, int32_t face) {
  if (check_grid(g) != FD_OK) return -1;
  switch (face) {
    case 0: case 1: return 4LL * g->ny * g->nz;
    case 2: case 3: return 4LL * g->nx * g->nz;
    case 4: case 5: return 4LL * g->nx * g->ny;
    default: fail(FD_EINVAL, "face %d not in 0..5", face); return -1;
  }
}

int64_t fd_offset(const fd_grid* g, int32_t i, int32_t j, int32_t k) {
  if (check_grid(g) != FD_OK) return -1;
  if (i < -4 || i >= g->nx + 4 || j < -4 || j >= g->ny + 4 || k < -4 || k >= g->nz + 4) {
    fail(FD_EINVAL, "point (%d,%d,%d) outside the padded box", i, j, k);
    return -1;
  }
  return g->origin + (int64_t)k * g->zstride + (int64_t)j * g->ystride + i;
}

int fd_set_kchunk(int32_t kchunk) {
  if (kchunk < 0) return fail(FD_EINVAL, "kchunk must be >= 0 (0 = automatic)");
  set_kchunk_override(kchunk);
  return FD_OK;
}

int fd_set_tiles(int32_t mode) {
  if (mode < 0 || mode > 5)
    return fail(FD_EINVAL,
                "tile mode %d: 0 (automatic), 1 (64 x 32), 2 (64 x 16), 3 (one thread per point), "
                "4 (128 x 32, 16-byte lanes) or 5 (64 x 64, 16-byte lanes)",
                mode);
  set_tile_override(mode);
  return FD_OK;
}

int fd_step_launch(const fd_grid* g, int32_t out[4]) {
  int rc = check_grid(g);
  if (rc) return rc;
  if (!out) return fail(FD_EINVAL, "fd_step_launch: out is NULL");
  int o[4];
  forward_launch_shape(make_geo(g), o);
  for (int i = 0; i < 4; ++i) out[i] = o[i];
  return FD_OK;
}

int fd_step_kernel(const fd_grid* g, int32_t with_faces, int32_t out[6]) {
  int rc = check_grid(g);
  if (rc) return rc;
  if (!out) return fail(FD_EINVAL, "fd_step_kernel: out is NULL");
  const Geo geo = make_geo(g);
  int kind, o[4] = {0, 0, 0, 0}, tx = 1, ty = 1;
  // the same choices as fd_step_exchange (all twelve faces) and fd_step_fused, with
  // arrays and face buffers 16-byte aligned
  const bool wide_ok = geo.sy % 4 == 0 && geo.sz % 4 == 0 && geo.org % 4 == 0;
  // with faces: the x faces go inside the marching kernels where nx is a multiple of
  // 64 (of 128 for 16-byte lanes); otherwise unpack, the update without faces, pack
  const bool x_inside = with_faces && exchange_fits(geo);
  const bool point = with_faces && point_exchange_pays(geo) ? true
                     : x_inside                             ? false
                                                            : point_kernel_pays(geo);
  const bool wide_fits = wide_ok && (!x_inside || (geo.nx % 128 == 0 &&
                                                   (long long)geo.ny * geo.nz * 16 < (1LL << 32)));
  if (point) {
    kind = FD_KERNEL_POINT;
  } else if (forward_wide_tiles(geo) && wide_fits) {
    // the exchange form keeps 128 x 32 tiles (its x faces are whole tile columns)
    const bool narrow = !x_inside && wide_narrow_tiles(geo);
    kind = narrow ? FD_KERNEL_WIDE_64x64 : FD_KERNEL_WIDE;
    if (narrow) {
      wide_forward_shape(geo, o);
    } else {
      const LaunchShape sh = stencil_shape(geo, 128, 32, 16);
      o[0] = sh.tiles_x;
      o[1] = sh.tiles_y;
      o[2] = sh.kchunk;
      o[3] = sh.zchunks;
    }
    tx = narrow ? 64 : 128;
    ty = narrow ? 64 : 32;
  } else {
    const bool small = forward_small_tiles(geo);
    kind = small ? FD_KERNEL_MARCH_64x16 : FD_KERNEL_MARCH_64x32;
    forward_launch_shape(geo, o);
    tx = 64;
    ty = small ? 16 : 32;
  }
  out[0] = kind;
  out[1] = tx;
  out[2] = ty;
  if (kind == FD_KERNEL_POINT) {
    out[3] = out[4] = 1;
    out[5] = -1;
  } else {
    out[3] = o[2];  // planes per block
    out[4] = o[3];  // z chunks
    out[5] = o[0] * o[1] * o[3];
  }
  return FD_OK;
}

namespace {
// fd_cfl_dt with its result slots at scratch_dev (two int32 of device memory)
int cfl_dt_with(const fd_grid* g, const float* v, double courant, int32_t* scratch_dev,
                double* vmax_host, double* dt_out, void* stream) {
  int rc = FD_OK;
  hipStream_t s = as_stream(stream);
  rc = check_hip(launch_vmax(make_geo(g), v, scratch_dev, s), "vmax launch");
  if (rc) return rc;
  int32_t host[2];
  rc = check_hip(hipMemcpyAsync(host, scratch_dev, sizeof(host), hipMemcpyDeviceToHost, s),
                 "vmax copy");
  if (rc) return rc;
  rc = check_hip(hipStreamSynchronize(s), "vmax sync");
  if (rc) return rc;
  float vmax, vmin;
  memcpy(&vmax, &host[0], 4);
  memcpy(&vmin, &host[1], 4);
  if (!(isfinite(vmax) && vmax > 0.f) || !(vmin > 0.f))
    return fail(FD_EINVAL, "velocity must be finite and > 0 (max %g, min %g)", vmax, vmin);
  double dmin = g->dx;
  if (g->dy < dmin) dmin = g->dy;
  if (g->dz < dmin) dmin = g->dz;
  if (vmax_host) *vmax_host = vmax;
  if (dt_out) *dt_out = courant * dmin / (double)vmax;
  return FD_OK;
}
}  // namespace

int fd_cfl_dt(const fd_grid* g, const float* v, double courant, int32_t* scratch_dev,
              double* vmax_host, double* dt_out, void* stream) {
  int rc = check_grid(g);
  if (rc) return rc;
  if (!v || !scratch_dev) return fail(FD_EINVAL, "fd_cfl_dt: NULL array");
  if (!finite_pos(courant)) return fail(FD_EINVAL, "fd_cfl_dt: courant must be > 0");
  return cfl_dt_with(g, v, courant, scratch_dev, vmax_host, dt_out, stream);
}

int fd_cfl_dt_static(const fd_grid* g, const float* v, double courant, double* vmax_host,
                     double* dt_out, void* stream) {
  int rc = check_grid(g);
  if (rc) return rc;
  if (!v) return fail(FD_EINVAL, "fd_cfl_dt_static: NULL array");
  if (!finite_pos(courant)) return fail(FD_EINVAL, "fd_cfl_dt_static: courant must be > 0");
  int32_t* slots = nullptr;  // the library's own static slots on the current device
  rc = check_hip(cfl_scratch(&slots), "fd_cfl_dt_static: static scratch lookup");
  if (rc) return rc;
  return cfl_dt_with(g, v, courant, slots, vmax_host, dt_out, stream);
}

int fd_prepare_vdt2(const fd_grid* g, const float* v, float* vdt2, double dt, void* stream) {
  int rc = check_grid(g);
  if (rc) return rc;
  if (!v || !vdt2) return fail(FD_EINVAL, "fd_prepare_vdt2: NULL array");
  if (overlaps(g, v, vdt2)) return fail(FD_EINVAL, "fd_prepare_vdt2: v and vdt2 overlap");
  if (!finite_pos(dt)) return fail(FD_EINVAL, "fd_prepare_vdt2: dt must be > 0");
  return check_hip(launch_prepare_vdt2(make_geo(g), v, vdt2, dt, false, as_stream(stream)),
                   "prepare_vdt2 launch");
}

int fd_prepare_vdt2_m(const fd_grid* g, const float* m, float* vdt2, double dt, void* stream) {
  int rc = check_grid(g);
  if (rc) return rc;
  if (!m || !vdt2) return fail(FD_EINVAL, "fd_prepare_vdt2_m: NULL array");
  if (overlaps(g, m, vdt2)) return fail(FD_EINVAL, "fd_prepare_vdt2_m: m and vdt2 overlap");
  if (!finite_pos(dt)) return fail(FD_EINVAL, "fd_prepare_vdt2_m: dt must be > 0");
  return check_hip(launch_prepare_vdt2(make_geo(g), m, vdt2, dt, true, as_stream(stream)),
                   "prepare_vdt2_m launch");
}

double fd_sponge_eta_max(double vmax, double d, double dt, int32_t width, double R) {
  if (width <= 0) return 0.0;
  if (!finite_pos(vmax) || !finite_pos(d) || !finite_pos(dt) || !(R > 0.0 && R < 1.0))
    return (double)fail(FD_EINVAL, "fd_sponge_eta_max: bad argument");
  const double sigma_max = 3.0 * vmax * log(1.0 / R) / (2.0 * (double)width * d);
  return 0.5 * dt * sigma_max;
}

int fd_sponge_profile(float* host_out, int32_t n, int32_t width, double eta_max) {
  if (!host_out || n < 1) return fail(FD_EINVAL, "fd_sponge_profile: bad output");
  if (!(eta_max >= 0.0) || !isfinite(eta_max))
    return fail(FD_EINVAL, "fd_sponge_profile: eta_max must be finite and >= 0");
  for (int32_t i = 0; i < n; ++i) {
    double e = 0.0;
    if (width > 0) {
      int32_t d = width - i;
      const int32_t d2 = i - (n - 1 - width);
      if (d2 > d) d = d2;
      if (d > 0) {
        const double r = (double)d / (double)width;
        e = eta_max * r * r;
      }
    }
    host_out[i] = (float)e;
  }
  return FD_OK;
}

int fd_ricker(float* host_out, int32_t nt, int32_t n0, double dt, double f0, double t0) {
  if (!host_out || nt < 0) return fail(FD_EINVAL, "fd_ricker: bad output");
  if (!finite_pos(dt) || !finite_pos(f0) || !isfinite(t0))
    return fail(FD_EINVAL, "fd_ricker: bad dt, f0 or t0");
  const double pi = 3.14159265358979323846;
  for (int32_t n = 0; n < nt; ++n) {
    const double t = (double)(n0 + n) * dt - t0;
    const double a = (pi * f0 * t) * (pi * f0 * t);
    host_out[n] = (float)((1.0 - 2.0 * a) * exp(-a));
  }
  return FD_OK;
}

int fd_receiver_offsets(const fd_grid* g, const int32_t* ijk, int32_t nrec, int64_t* off) {
  int rc = check_grid(g);
  if (rc) return rc;
  if (nrec < 0 || (nrec > 0 && (!ijk || !off)))
    return fail(FD_EINVAL, "fd_receiver_offsets: bad arrays");
  for (int32_t r = 0; r < nrec; ++r) {
    const int32_t i = ijk[3 * r], j = ijk[3 * r + 1], k = ijk[3 * r + 2];
    if (i < 0 || i >= g->nx || j < 0 || j >= g->ny || k < 0 || k >= g->nz)
      return fail(FD_EINVAL, "receiver %d at (%d,%d,%d) is outside the interior", r, i, j, k);
    off[r] = g->origin + (int64_t)k * g->zstride + (int64_t)j * g->ystride + i;
  }
  return FD_OK;
}

int fd_step(const fd_grid* g, const float* u_prev, const float* u, float* u_next,
            const float* vdt2, const fd_sponge* sp, void* stream) {
  int rc = check_grid(g);
  if (rc) return rc;
  if (!u_prev || !u || !u_next || !vdt2) return fail(FD_EINVAL, "fd_step: NULL array");
  if (overlaps(g, u, u_next)) return fail(FD_EINVAL, "fd_step: u_next overlaps u");
  if (overlaps(g, vdt2, u_next)) return fail(FD_EINVAL, "fd_step: u_next overlaps vdt2");
  if (u_next != u_prev && overlaps(g, u_prev, u_next))
    return fail(FD_EINVAL, "fd_step: u_next partially overlaps u_prev");
  const float *ex, *ey, *ez;
  rc = check_sponge(sp, &ex, &ey, &ez);
  if (rc) return rc;
  return check_hip(forward_update(make_geo(g), make_coef(g), u_prev, u, u_next, vdt2, ex, ey, ez,
                                  nullptr, as_stream(stream)),
                   "fd_step launch");
}

static int check_faces(const fd_grid* g, const void* const* face, const char* who);

// Overlap checks of six face buffers against the volume arrays of one call.
static int faces_clear_of(const fd_grid* g, const float* const face[6], const float* const* vols,
                          int nvol, const char* who) {
  for (int f = 0; f < 6; ++f) {
    const float* fp = face[f];
    if (!fp) continue;
    const int64_t n = fd_face_elems(g, f);
    for (int v = 0; v < nvol; ++v) {
      const float* a = vols[v];
      if (a && fp < a + last_elem(g) + 1 && a < fp + n)
        return fail(FD_EINVAL, "%s: face %d overlaps a volume array", who, f);
    }
  }
  return FD_OK;
}

int fd_step_fused(const fd_grid* g, const float* u_prev, const float* u, float* u_next,
                  const float* vdt2, const fd_sponge* sp, const fd_source* src,
                  float* const face_out[6], void* stream) {
  int rc = check_grid(g);
  if (rc) return rc;
  if (!u_prev || !u || !u_next || !vdt2) return fail(FD_EINVAL, "fd_step_fused: NULL array");
  if (overlaps(g, u, u_next)) return fail(FD_EINVAL, "fd_step_fused: u_next overlaps u");
  if (overlaps(g, vdt2, u_next)) return fail(FD_EINVAL, "fd_step_fused: u_next overlaps vdt2");
  if (u_next != u_prev && overlaps(g, u_prev, u_next))
    return fail(FD_EINVAL, "fd_step_fused: u_next partially overlaps u_prev");
  if (src && (src->i < 0 || src->i >= g->nx || src->j < 0 || src->j >= g->ny || src->k < 0 ||
              src->k >= g->nz))
    return fail(FD_EINVAL, "fd_step_fused: source outside the interior");
  if (face_out) {
    rc = check_faces(g, (const void* const*)face_out, "fd_step_fused");
    if (rc) return rc;
    const float* vols[4] = {u_prev, u, u_next, vdt2};
    rc = faces_clear_of(g, face_out, vols, 4, "fd_step_fused");
    if (rc) return rc;
  }
  const float *ex, *ey, *ez;
  rc = check_sponge(sp, &ex, &ey, &ez);
  if (rc) return rc;
  const Geo geo = make_geo(g);
  hipStream_t s = as_stream(stream);
  rc = check_hip(forward_update(geo, make_coef(g), u_prev, u, u_next, vdt2, ex, ey, ez, src, s),
                 "fd_step_fused launch");
  if (rc || !face_out) return rc;
  return check_hip(launch_pack(geo, u_next, face_out, s), "fd_step_fused pack launch");
}

static bool face_sets_overlap(const fd_grid* g, const float* const a[6], const float* const b[6]) {
  for (int f = 0; f < 6; ++f) {
    if (!a[f]) continue;
    const int64_t na = fd_face_elems(g, f);
    for (int h = 0; h < 6; ++h) {
      if (!b[h]) continue;
      const int64_t nb = fd_face_elems(g, h);
      if (a[f] < b[h] + nb && b[h] < a[f] + na) return true;
    }
  }
  return false;
}

// One step of the exchange form, arguments already checked; with receivers
// (nrec > 0) the receiver row of un is taken in the launch that packs its faces,
// or, on grids that run one thread per point with all twelve faces, in that one
// launch (with a plane map, rec_map) or one of its own.
static hipError_t step_exchange(const Geo& geo, const Coef& c, const float* up, float* u,
                                float* un, const float* q, const float* ex, const float* ey,
                                const float* ez, const fd_source* src,
                                const float* const face_in[6], float* const face_out[6],
                                hipStream_t s, const int64_t* rec_off = nullptr, int nrec = 0,
                                float* row = nullptr, const int32_t* rec_map = nullptr,
                                int rec_k = -1) {
  hipError_t e = hipSuccess;
  bool all12 = face_in && face_out && point_exchange_pays(geo);
  for (int f = 0; f < 6 && all12; ++f) all12 = face_in[f] && face_out[f];
  if (all12) {  // small grid: the whole step in one launch
    const RecPlane rp{rec_map, rec_k, row};
    const bool in_kernel = rec_map && nrec > 0;
    e = launch_step_point(geo, c, up, u, un, q, ex, ey, ez, src, in_kernel ? &rp : nullptr, s,
                          face_in, face_out);
    if (e == hipSuccess && nrec > 0 && !in_kernel) e = launch_record(un, rec_off, nrec, row, s);
    return e;
  }
  if (exchange_fits(geo) && face_in && face_out && face_in[0] && face_in[1] && face_out[0] &&
      face_out[1]) {
    // x faces inside the stencil kernel; y and z faces (whole rows and planes)
    // by the unpack/pack kernels
    const float* in_yz[6] = {nullptr, nullptr, face_in[2], face_in[3], face_in[4], face_in[5]};
    float* out_yz[6] = {nullptr, nullptr, face_out[2], face_out[3], face_out[4], face_out[5]};
    const float* in_x[2] = {face_in[0], face_in[1]};
    float* out_x[2] = {face_out[0], face_out[1]};
    e = launch_unpack(geo, u, in_yz, s);
    if (e == hipSuccess)
      e = launch_step_exchange(geo, c, up, u, un, q, ex, ey, ez, src, in_x, out_x, s);
    if (e == hipSuccess) e = launch_pack_record(geo, un, out_yz, rec_off, nrec, row, s);
    return e;
  }
  if (face_in) e = launch_unpack(geo, u, face_in, s);
  if (e == hipSuccess) e = forward_update(geo, c, up, u, un, q, ex, ey, ez, src, s);
  if (e == hipSuccess && face_out) e = launch_pack_record(geo, un, face_out, rec_off, nrec, row, s);
  else if (e == hipSuccess && nrec > 0) e = launch_record(un, rec_off, nrec, row, s);
  return e;
}

int fd_step_exchange(const fd_grid* g, const float* u_prev, float* u, float* u_next,
                     const float* vdt2, const fd_sponge* sp, const fd_source* src,
                     const float* const face_in[6], float* const face_out[6], void* stream) {
  int rc = check_grid(g);
  if (rc) return rc;
  if (!u_prev || !u || !u_next || !vdt2) return fail(FD_EINVAL, "fd_step_exchange: NULL array");
  if (overlaps(g, u, u_next)) return fail(FD_EINVAL, "fd_step_exchange: u_next overlaps u");
  if (overlaps(g, vdt2, u_next)) return fail(FD_EINVAL, "fd_step_exchange: u_next overlaps vdt2");
  if (u_next != u_prev && overlaps(g, u_prev, u_next))
    return fail(FD_EINVAL, "fd_step_exchange: u_next partially overlaps u_prev");
  if (src && (src->i < 0 || src->i >= g->nx || src->j < 0 || src->j >= g->ny || src->k < 0 ||
              src->k >= g->nz))
    return fail(FD_EINVAL, "fd_step_exchange: source outside the interior");
  const float* vols[4] = {u_prev, u, u_next, vdt2};
  if (face_in) {
    rc = check_faces(g, (const void* const*)face_in, "fd_step_exchange");
    if (rc) return rc;
    rc = faces_clear_of(g, face_in, vols, 4, "fd_step_exchange (face_in)");
    if (rc) return rc;
  }
  if (face_out) {
    rc = check_faces(g, (const void* const*)face_out, "fd_step_exchange");
    if (rc) return rc;
    rc = faces_clear_of(g, face_out, vols, 4, "fd_step_exchange (face_out)");
    if (rc) return rc;
  }
  if (face_in && face_out && face_sets_overlap(g, face_in, face_out))
    return fail(FD_EINVAL, "fd_step_exchange: a face_in buffer overlaps a face_out buffer");
  const float *ex, *ey, *ez;
  rc = check_sponge(sp, &ex, &ey, &ez);
  if (rc) return rc;
  return check_hip(step_exchange(make_geo(g), make_coef(g), u_prev, u, u_next, vdt2, ex, ey, ez,
                                 src, face_in, face_out, as_stream(stream)),
                   "fd_step_exchange launch");
}

// Argument checks of fd_forward_run (and of the graph that records it): the
// number of face buffers of each set and the sponge tables.
static int forward_checked(const fd_grid* g, const fd_run* run, int* nsend_out, int* nsend2_out,
                           const float** ex_out, const float** ey_out, const float** ez_out) {
  int rc = check_grid(g);
  if (rc) return rc;
  if (!run) return fail(FD_EINVAL, "fd_forward_run: run is NULL");
  const float *up = run->u_prev, *u = run->u, *un = run->u_next;
  if (!up || !u || !un || !run->vdt2) return fail(FD_EINVAL, "fd_forward_run: NULL array");
  if (overlaps(g, up, u) || overlaps(g, u, un) || overlaps(g, up, un))
    return fail(FD_EINVAL, "fd_forward_run: the three wavefields must be distinct");
  if (overlaps(g, run->vdt2, up) || overlaps(g, run->vdt2, u) || overlaps(g, run->vdt2, un))
    return fail(FD_EINVAL, "fd_forward_run: vdt2 overlaps a wavefield");
  if (run->nt < 0) return fail(FD_EINVAL, "fd_forward_run: nt < 0");
  if (run->nrec < 0 || (run->nrec > 0 && run->nt > 0 && (!run->rec_off || !run->traces)))
    return fail(FD_EINVAL, "fd_forward_run: bad receivers");
  if (run->rec_map && (run->rec_k < 0 || run->rec_k >= g->nz))
    return fail(FD_EINVAL, "fd_forward_run: receiver plane %d outside the interior", run->rec_k);
  if (run->wavelet && (run->src[0] < 0 || run->src[0] >= g->nx || run->src[1] < 0 ||
                       run->src[1] >= g->ny || run->src[2] < 0 || run->src[2] >= g->nz))
    return fail(FD_EINVAL, "fd_forward_run: source outside the interior");
  int nsend = 0, nsend2 = 0;
  for (int f = 0; f < 6; ++f) {
    nsend += run->send[f] != nullptr;
    nsend2 += run->send2[f] != nullptr;
  }
  if ((nsend != 0 && nsend != 6) || (nsend2 != 0 && nsend2 != 6))
    return fail(FD_EINVAL, "fd_forward_run: give all six face buffers or none");
  if (nsend2 && !nsend) return fail(FD_EINVAL, "fd_forward_run: send2 needs send");
  const float* vols[4] = {up, u, un, run->vdt2};
  if (nsend) {
    rc = check_faces(g, (const void* const*)run->send, "fd_forward_run");
    if (rc) return rc;
    rc = faces_clear_of(g, run->send, vols, 4, "fd_forward_run (send)");
    if (rc) return rc;
  }
  if (nsend2) {
    rc = check_faces(g, (const void* const*)run->send2, "fd_forward_run");
    if (rc) return rc;
    rc = faces_clear_of(g, run->send2, vols, 4, "fd_forward_run (send2)");
    if (rc) return rc;
    if (face_sets_overlap(g, run->send, run->send2))
      return fail(FD_EINVAL, "fd_forward_run: send and send2 overlap");
  }
  const float *ex, *ey, *ez;
  rc = check_sponge(&run->sponge, &ex, &ey, &ez);
  if (rc) return rc;
  *nsend_out = nsend;
  *nsend2_out = nsend2;
  *ex_out = ex;
  *ey_out = ey;
  *ez_out = ez;
  return FD_OK;
}

// The nt steps of a checked fd_run, enqueued on s; the struct's pointers are
// rotated as the steps go (also when a launch fails part way).
static hipError_t forward_steps(const fd_grid* g, fd_run* run, int nsend, int nsend2,
                                const float* ex, const float* ey, const float* ez,
                                hipStream_t s) {
  float *up = run->u_prev, *u = run->u, *un = run->u_next;
  const Geo geo = make_geo(g);
  const Coef c = make_coef(g);
  float** cur = run->send;   // faces of u
  float** nxt = run->send2;  // ping-pong: faces of u_next
  for (int32_t n = 0; n < run->nt; ++n) {
    hipError_t e = hipSuccess;
    const float* recv[6] = {cur[1], cur[0], cur[3], cur[2], cur[5], cur[4]};
    fd_source src;
    if (run->wavelet) {
      src.i = run->src[0];
      src.j = run->src[1];
      src.k = run->src[2];
      src.w = run->wavelet[n];
    }
    const fd_source* sp_src = run->wavelet ? &src : nullptr;
    // the receiver row of u^{n+1} is taken in the launch that packs its faces, or
    // with a receiver plane map and no faces by the stencil launch itself
    float* row = run->nrec ? run->traces + (int64_t)n * run->nrec : nullptr;
    if (nsend2) {
      e = step_exchange(geo, c, up, u, un, run->vdt2, ex, ey, ez, sp_src, recv, nxt, s,
                        run->rec_off, run->nrec, row, run->rec_map, run->rec_k);
      float** t = cur;
      cur = nxt;
      nxt = t;
    } else {
      const RecPlane rp{run->rec_map, run->rec_k, row};
      // the one-thread-per-point kernel takes the row at the cost of one map load
      // per thread of the plane (128^3, sponge: 12.6 -> 10.1 us per step); the
      // 16-byte-lane kernel loads its map entries before it marches
      const float* const arrs[4] = {up, u, un, run->vdt2};
      const bool in_kernel = run->rec_map && run->nrec > 0 && !nsend &&
                             (receiver_plane_pays(geo) || point_kernel_pays(geo) ||
                              wide_takes_step(geo, arrs));
      if (nsend) e = launch_unpack(geo, u, recv, s);
      if (e == hipSuccess)
        e = forward_update(geo, c, up, u, un, run->vdt2, ex, ey, ez, sp_src, s,
                           in_kernel ? &rp : nullptr);
      if (e == hipSuccess && nsend)
        e = launch_pack_record(geo, un, cur, run->rec_off, run->nrec, row, s);
      else if (e == hipSuccess && run->nrec && !in_kernel)
        e = launch_record(un, run->rec_off, run->nrec, row, s);
    }
    if (e != hipSuccess) {
      run->u_prev = up;
      run->u = u;
      run->u_next = un;
      return e;
    }
    float* t = up;
    up = u;
    u = un;
    un = t;
  }
  run->u_prev = up;
  run->u = u;
  run->u_next = un;
  if (cur != run->send)  // ping-pong: run->send holds the faces of the final u
    for (int f = 0; f < 6; ++f) std::swap(run->send[f], run->send2[f]);
  return hipSuccess;
}

int fd_forward_run(const fd_grid* g, fd_run* run, void* stream) {
  int nsend, nsend2;
  const float *ex, *ey, *ez;
  const int rc = forward_checked(g, run, &nsend, &nsend2, &ex, &ey, &ez);
  if (rc) return rc;
  return check_hip(forward_steps(g, run, nsend, nsend2, ex, ey, ez, as_stream(stream)),
                   "fd_forward_run launch");
}

struct fd_graph {
  hipGraphExec_t exec;
};

int fd_forward_graph(const fd_grid* g, fd_run* run, fd_graph** out) {
  if (!out) return fail(FD_EINVAL, "fd_forward_graph: out is NULL");
  *out = nullptr;
  int nsend, nsend2;
  const float *ex, *ey, *ez;
  int rc = forward_checked(g, run, &nsend, &nsend2, &ex, &ey, &ez);
  if (rc) return rc;
  // recorded on a private stream (capture needs one that is not the null stream);
  // the caller's struct changes only on success
  hipStream_t cs = nullptr;
  rc = check_hip(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking), "fd_forward_graph stream");
  if (rc) return rc;
  fd_run r = *run;
  hipGraphExec_t exec = nullptr;
  hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    // the zero start: u^{n-1}, u^n, u^{n+1} (whose halo is the boundary once it
    // rotates into u^n) and (exchange) the faces of u^n, by fill kernels
    const int64_t n = last_elem(g) + 1;
    hipError_t le = launch_zero(r.u_prev, n, cs);
    if (le == hipSuccess) le = launch_zero(r.u, n, cs);
    if (le == hipSuccess && r.u_next != r.u_prev) le = launch_zero(r.u_next, n, cs);
    for (int f = 0; f < 6 && le == hipSuccess && nsend; ++f)
      le = launch_zero(r.send[f], fd_face_elems(g, f), cs);
    if (le == hipSuccess) le = forward_steps(g, &r, nsend, nsend2, ex, ey, ez, cs);
    hipGraph_t graph = nullptr;
    const hipError_t ee = hipStreamEndCapture(cs, &graph);
    e = le != hipSuccess ? le : ee;
    if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (graph) (void)hipGraphDestroy(graph);
  }
  (void)hipStreamDestroy(cs);
  if (e != hipSuccess) {
    if (exec) (void)hipGraphExecDestroy(exec);
    return check_hip(e, "fd_forward_graph capture");
  }
  *out = new (std::nothrow) fd_graph{exec};
  if (!*out) {
    (void)hipGraphExecDestroy(exec);
    return fail(FD_ENOMEM, "fd_forward_graph: out of host memory");
  }
  *run = r;
  return FD_OK;
}

int fd_graph_launch(fd_graph* graph, void* stream) {
  if (!graph) return fail(FD_EINVAL, "fd_graph_launch: graph is NULL");
  return check_hip(hipGraphLaunch(graph->exec, as_stream(stream)), "fd_graph_launch");
}

int fd_graph_destroy(fd_graph* graph) {
  if (!graph) return FD_OK;
  const int rc = check_hip(hipGraphExecDestroy(graph->exec), "fd_graph_destroy");
  delete graph;
  return rc;
}


int fd_receiver_plane_map(const fd_grid* g, const int32_t* rec_ijk, int32_t nrec, int32_t* map,
                          int32_t* k_out) {
  int rc = check_grid(g);
  if (rc) return rc;
  if (!rec_ijk || !map || !k_out) return fail(FD_EINVAL, "fd_receiver_plane_map: NULL argument");
  if (nrec < 1) return fail(FD_EINVAL, "fd_receiver_plane_map: no receivers");
  const int64_t nxy = (int64_t)g->nx * g->ny;
  for (int64_t q = 0; q < nxy; ++q) map[q] = -1;
  const int32_t k = rec_ijk[2];
  for (int32_t r = 0; r < nrec; ++r) {
    const int32_t i = rec_ijk[3 * r], j = rec_ijk[3 * r + 1], kr = rec_ijk[3 * r + 2];
    if (i < 0 || i >= g->nx || j < 0 || j >= g->ny || kr < 0 || kr >= g->nz)
      return fail(FD_EINVAL, "fd_receiver_plane_map: receiver %d outside the interior", r);
    if (kr != k) return fail(FD_EINVAL, "fd_receiver_plane_map: receivers on more than one plane");
    int32_t& m = map[(int64_t)j * g->nx + i];
    if (m >= 0) return fail(FD_EINVAL, "fd_receiver_plane_map: receivers %d and %d coincide", m, r);
    m = r;
  }
  *k_out = k;
  return FD_OK;
}

int inject_source(const fd_grid* g, float* u_next, const float* vdt2, const fd_sponge* sp,
                  int32_t i, int32_t j, int32_t k, float w, void* stream) {
  int rc = check_grid(g);
  if (rc) return rc;
  if (!u_next || !vdt2) return fail(FD_EINVAL, "inject_source: NULL array");
  if (i < 0 || i >= g->nx || j < 0 || j >= g->ny || k < 0 || k >= g->nz)
    return fail(FD_EINVAL, "inject_source: (%d,%d,%d) outside the interior", i, j, k);
  const float *ex, *ey, *ez;
  rc = check_sponge(sp, &ex, &ey, &ez);
  if (rc) return rc;
  return check_hip(
      launch_inject(make_geo(g), u_next, vdt2, ex, ey, ez, i, j, k, w, as_stream(stream)),
      "inject_source launch");
}

int record_receivers(const fd_grid* g, const float* u, const int64_t* rec_off, int32_t nrec,
                     float* trace_row, void* stream) {
  int rc = check_grid(g);
  if (rc) return rc;
  if (nrec < 0) return fail(FD_EINVAL, "record_receivers: nrec < 0");
  if (nrec == 0) return FD_OK;
  if (!u || !rec_off || !trace_row) return fail(FD_EINVAL, "record_receivers: NULL array");
  return check_hip(launch_record(u, rec_off, nrec, trace_row, as_stream(stream)),
                   "record_receivers launch");
}

static int check_faces(const fd_grid* g, const void* const* face, const char* who) {
  if (!face) return fail(FD_EINVAL, "%s: face array is NULL", who);
  const int n3[3] = {g->nx, g->ny, g->nz};
  for (int f = 0; f < 6; ++f) {
    if (!face[f]) continue;
    if (reinterpret_cast<uintptr_t>(face[f]) & 3)
      return fail(FD_EINVAL, "%s: face %d is not 4-byte aligned", who, f);
    if (n3[f / 2] < 4)
      return fail(FD_EINVAL, "%s: face %d needs at least 4 interior planes on its axis", who, f);
    if (fd_face_elems(g, f) > (int64_t)std::numeric_limits<int32_t>::max())
      return fail(FD_EINVAL, "%s: face %d larger than INT32_MAX elements", who, f);
  }
  return FD_OK;
}

int halo_pack(const fd_grid* g, const float* u, float* const face[6], void* stream) {
  int rc = check_grid(g);
  if (rc) return rc;
  if (!u) return fail(FD_EINVAL, "halo_pack: u is NULL");
  rc = check_faces(g, (const void* const*)face, "halo_pack");
  if (rc) return rc;
  return check_hip(launch_pack(make_geo(g), u, face, as_stream(stream)), "halo_pack launch");
}

int fd_halo_pack_record(const fd_grid* g, const float* u, float* const face[6],
                        const int64_t* rec_off, int32_t nrec, float* trace_row, void* stream) {
  int rc = check_grid(g);
  if (rc) return rc;
  if (!u) return fail(FD_EINVAL, "fd_halo_pack_record: u is NULL");
  rc = check_faces(g, (const void* const*)face, "fd_halo_pack_record");
  if (rc) return rc;
  if (nrec < 0) return fail(FD_EINVAL, "fd_halo_pack_record: nrec < 0");
  if (nrec > 0 && (!rec_off || !trace_row))
    return fail(FD_EINVAL, "fd_halo_pack_record: NULL receiver array");
  return check_hip(launch_pack_record(make_geo(g), u, face, rec_off, nrec, trace_row,
                                      as_stream(stream)),
                   "fd_halo_pack_record launch");
}

int halo_unpack(const fd_grid* g, float* u, const float* const face[6], void* stream) {
  int rc = check_grid(g);
  if (rc) return rc;
  if (!u) return fail(FD_EINVAL, "halo_unpack: u is NULL");
  rc = check_faces(g, (const void* const*)face, "halo_unpack");
  if (rc) return rc;
  return check_hip(launch_unpack(make_geo(g), u, face, as_stream(stream)),
                   "halo_unpack launch");
}

int fd_adjoint_step(const fd_grid* g, const float* a_nn, const float* a_n1, float* a_out,
                    const float* vdt2, const fd_sponge* sp, const float* u_n, float* g_vdt2,
                    const fd_source* src, void* stream) {
  int rc = check_grid(g);
  if (rc) return rc;
  if (!a_n1 || !a_out || !vdt2) return fail(FD_EINVAL, "fd_adjoint_step: NULL array");
  if (overlaps(g, a_n1, a_out)) return fail(FD_EINVAL, "fd_adjoint_step: a_out overlaps a_n1");
  if (overlaps(g, vdt2, a_out)) return fail(FD_EINVAL, "fd_adjoint_step: a_out overlaps vdt2");
  if (a_nn && a_out != a_nn && overlaps(g, a_nn, a_out))
    return fail(FD_EINVAL, "fd_adjoint_step: a_out partially overlaps a_nn");
  if (g_vdt2) {
    if (!u_n) return fail(FD_EINVAL, "fd_adjoint_step: gradient needs u_n");
    if (overlaps(g, g_vdt2, a_out) || overlaps(g, g_vdt2, a_n1) || overlaps(g, g_vdt2, u_n) ||
        overlaps(g, g_vdt2, vdt2) || (a_nn && overlaps(g, g_vdt2, a_nn)))
      return fail(FD_EINVAL, "fd_adjoint_step: g_vdt2 overlaps another array");
    if (src && (src->i < 0 || src->i >= g->nx || src->j < 0 || src->j >= g->ny || src->k < 0 ||
                src->k >= g->nz))
      return fail(FD_EINVAL, "fd_adjoint_step: source outside the interior");
  }
  const float *ex, *ey, *ez;
  rc = check_sponge(sp, &ex, &ey, &ez);
  if (rc) return rc;
  const Geo geo = make_geo(g);
  const Coef c = make_coef(g);
  hipStream_t s = as_stream(stream);
  // the gradient reads a_n1 pointwise and must see it before a_out (which may
  // alias a_nn, not a_n1) is written; both kernels leave a_n1 untouched
  if (g_vdt2) {
    rc = check_hip(launch_grad(geo, c, u_n, a_n1, g_vdt2, ex, ey, ez, src, s), "gradient launch");
    if (rc) return rc;
  }
  return check_hip(launch_adjoint(geo, c, a_nn, a_n1, a_out, vdt2, ex, ey, ez, s),
                   "fd_adjoint_step launch");
}

int fd_scatter_add(const fd_grid* g, float* a, const int64_t* off, const float* vals, int32_t n,
                   void* stream) {
  int rc = check_grid(g);
  if (rc) return rc;
  if (n < 0) return fail(FD_EINVAL, "fd_scatter_add: n < 0");
  if (n == 0) return FD_OK;
  if (!a || !off || !vals) return fail(FD_EINVAL, "fd_scatter_add: NULL array");
  return check_hip(launch_scatter_add(a, off, vals, n, as_stream(stream)),
                   "fd_scatter_add launch");
}

int fd_grad_finalize(const fd_grid* g, const float* g_vdt2, const float* vdt2, double dt,
                     float* grad_m, void* stream) {
  int rc = check_grid(g);
  if (rc) return rc;
  if (!g_vdt2 || !vdt2 || !grad_m) return fail(FD_EINVAL, "fd_grad_finalize: NULL array");
  if (!finite_pos(dt)) return fail(FD_EINVAL, "fd_grad_finalize: dt must be > 0");
  if (overlaps(g, vdt2, grad_m)) return fail(FD_EINVAL, "fd_grad_finalize: grad_m overlaps vdt2");
  return check_hip(
      launch_grad_finalize(make_geo(g), g_vdt2, vdt2, dt, false, grad_m, as_stream(stream)),
      "fd_grad_finalize launch");
}

static int adjoint_scaled(const fd_grid* g, const float* b_nn, const float* b_n1, float* b_out,
                          const float* vdt2, const fd_sponge* sp, const float* u_n, float* g_b,
                          const fd_source* src, const RecPlane* inj, void* stream) {
  int rc = check_grid(g);
  if (rc) return rc;
  if (!b_nn || !b_n1 || !b_out || !vdt2)
    return fail(FD_EINVAL, "fd_adjoint_step_scaled: NULL array");
  if (overlaps(g, b_n1, b_out))
    return fail(FD_EINVAL, "fd_adjoint_step_scaled: b_out overlaps b_n1");
  if (overlaps(g, vdt2, b_out))
    return fail(FD_EINVAL, "fd_adjoint_step_scaled: b_out overlaps vdt2");
  if (b_out != b_nn && overlaps(g, b_nn, b_out))
    return fail(FD_EINVAL, "fd_adjoint_step_scaled: b_out partially overlaps b_nn");
  if (g_b) {
    if (!u_n) return fail(FD_EINVAL, "fd_adjoint_step_scaled: gradient needs u_n");
    if (overlaps(g, g_b, b_out) || overlaps(g, g_b, b_n1) || overlaps(g, g_b, u_n) ||
        overlaps(g, g_b, vdt2) || overlaps(g, g_b, b_nn))
      return fail(FD_EINVAL, "fd_adjoint_step_scaled: g_b overlaps another array");
    if (src && (src->i < 0 || src->i >= g->nx || src->j < 0 || src->j >= g->ny || src->k < 0 ||
                src->k >= g->nz))
      return fail(FD_EINVAL, "fd_adjoint_step_scaled: source outside the interior");
  }
  const float *ex, *ey, *ez;
  rc = check_sponge(sp, &ex, &ey, &ez);
  if (rc) return rc;
  const Geo geo = make_geo(g);
  const Coef c = make_coef(g);
  hipStream_t s = as_stream(stream);
  // gradient first: it reads b_n1, which neither kernel writes; no damping
  // factor (D is inside b)
  if (g_b) {
    rc = check_hip(launch_grad(geo, c, u_n, b_n1, g_b, nullptr, nullptr, nullptr, src, s),
                   "gradient launch");
    if (rc) return rc;
  }
  // the forward update run backward in time: b_out = D (2 b_n1 - E b_nn + Q L b_n1),
  // with inj the scaled residual row added at the receivers in the same launch
  return check_hip(forward_update(geo, c, b_nn, b_n1, b_out, vdt2, ex, ey, ez, nullptr, s, inj),
                   "fd_adjoint_step_scaled launch");
}

int fd_adjoint_step_scaled(const fd_grid* g, const float* b_nn, const float* b_n1, float* b_out,
                           const float* vdt2, const fd_sponge* sp, const float* u_n, float* g_b,
                           const fd_source* src, void* stream) {
  return adjoint_scaled(g, b_nn, b_n1, b_out, vdt2, sp, u_n, g_b, src, nullptr, stream);
}

int fd_adjoint_step_scaled_res(const fd_grid* g, const float* b_nn, const float* b_n1,
                               float* b_out, const float* vdt2, const fd_sponge* sp,
                               const float* u_n, float* g_b, const fd_source* src,
                               const int32_t* res_map, int32_t res_k, const float* res_row,
                               void* stream) {
  if (!g) return fail(FD_EINVAL, "grid is NULL");
  if (!res_map || !res_row)
    return fail(FD_EINVAL, "fd_adjoint_step_scaled_res: NULL receiver map or row");
  if (res_k < 0 || res_k >= g->nz)
    return fail(FD_EINVAL, "fd_adjoint_step_scaled_res: receiver plane %d outside the interior",
                res_k);
  RecPlane inj{res_map, res_k, const_cast<float*>(res_row)};
  inj.add = true;
  return adjoint_scaled(g, b_nn, b_n1, b_out, vdt2, sp, u_n, g_b, src, &inj, stream);
}

int fd_scatter_add_scaled(const fd_grid* g, float* b, const int64_t* off, const float* vals,
                          const float* vdt2, const fd_sponge* sp, int32_t n, void* stream) {
  int rc = check_grid(g);
  if (rc) return rc;
  if (n < 0) return fail(FD_EINVAL, "fd_scatter_add_scaled: n < 0");
  if (n == 0) return FD_OK;
  if (!b || !off || !vals || !vdt2) return fail(FD_EINVAL, "fd_scatter_add_scaled: NULL array");
  if (overlaps(g, vdt2, b)) return fail(FD_EINVAL, "fd_scatter_add_scaled: b overlaps vdt2");
  const float *ex, *ey, *ez;
  rc = check_sponge(sp, &ex, &ey, &ez);
  if (rc) return rc;
  return check_hip(launch_scatter_add_scaled(make_geo(g), b, off, vals, vdt2, ex, ey, ez, n,
                                             as_stream(stream)),
                   "fd_scatter_add_scaled launch");
}

int fd_grad_finalize_scaled(const fd_grid* g, const float* g_b, const float* vdt2, double dt,
                            float* grad_m, void* stream) {
  int rc = check_grid(g);
  if (rc) return rc;
  if (!g_b || !vdt2 || !grad_m) return fail(FD_EINVAL, "fd_grad_finalize_scaled: NULL array");
  if (!finite_pos(dt)) return fail(FD_EINVAL, "fd_grad_finalize_scaled: dt must be > 0");
  if (overlaps(g, vdt2, grad_m))
    return fail(FD_EINVAL, "fd_grad_finalize_scaled: grad_m overlaps vdt2");
  return check_hip(
      launch_grad_finalize(make_geo(g), g_b, vdt2, dt, true, grad_m, as_stream(stream)),
      "fd_grad_finalize_scaled launch");
}

}  // extern "C"
