/*
 * fd_oracle.c -- plain, slow, FP64 reference of the acoustic isotropic
 * finite-difference hot path (the Minimod acoustic-iso kernel of Sec. 4.5).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or helper with the HIP path and includes nothing from it.
 *
 * For the acoustic isotropic kernel the paper gives only that its stencil is of
 * high order (Sec. 4.5) and that halos are exchanged with neighbouring ranks
 * (Listing 1).  Every numerical choice below is therefore a reading: 8th-order
 * central second differences in each axis (a 25-point star), second-order
 * leapfrog in time, an optional damping sponge, a Ricker source added after
 * the update and receivers sampling the updated field.
 *
 * Layout of every volume here: FP64, halo H = 4 on each face, x fastest,
 * (nz+8) x (ny+8) x (nx+8) elements, interior point (i,j,k) at
 * ((k+4)*(ny+8) + (j+4))*(nx+8) + (i+4).  Interior-only arrays handed in or
 * out are C-ordered (nz, ny, nx).
 *
 * The library also holds the local block product of Cannon's matrix multiply
 * (Sec. 4.4), ora_block_gemm, the one dense contraction in the paper.
 *
 * Build: gcc -O2 -fopenmp -shared -fPIC fd_oracle.c -lm (no -ffast-math).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define OH 4

/* 8th-order central coefficients of d2/dx2 on unit spacing: the unique
 * symmetric 9-point weights exact for polynomials up to degree 9
 * (Fornberg 1988), c_0 = -205/72, c_1 = 8/5, c_2 = -1/5, c_3 = 8/315,
 * c_4 = -1/560. */
static const double CM[5] = {-205.0 / 72.0, 8.0 / 5.0, -1.0 / 5.0,
                             8.0 / 315.0, -1.0 / 560.0};

typedef struct {
  int nx, ny, nz;
  int64_t sy, sz; /* element strides of the padded FP64 box */
  double ix2, iy2, iz2; /* 1/d^2 per axis */
} box;

static box mkbox(int nx, int ny, int nz, double dx, double dy, double dz) {
  box b;
  b.nx = nx; b.ny = ny; b.nz = nz;
  b.sy = nx + 2 * OH;
  b.sz = b.sy * (int64_t)(ny + 2 * OH);
  b.ix2 = 1.0 / (dx * dx);
  b.iy2 = 1.0 / (dy * dy);
  b.iz2 = 1.0 / (dz * dz);
  return b;
}

static inline int64_t at(const box* b, int i, int j, int k) {
  return (int64_t)(k + OH) * b->sz + (int64_t)(j + OH) * b->sy + (i + OH);
}

int64_t ora_elems(int nx, int ny, int nz) {
  return (int64_t)(nx + 2 * OH) * (ny + 2 * OH) * (nz + 2 * OH);
}

/* The 25-point Laplacian at one padded index: per axis the centre weight times
 * u plus the symmetric pairs, scaled by 1/d^2, summed over x, y, z. */
static double lap_at(const box* b, const double* u, int64_t c) {
  const int64_t st[3] = {1, b->sy, b->sz};
  const double id2[3] = {b->ix2, b->iy2, b->iz2};
  double total = 0.0;
  for (int a = 0; a < 3; ++a) {
    double s = CM[0] * u[c];
    for (int m = 1; m <= 4; ++m) s += CM[m] * (u[c + m * st[a]] + u[c - m * st[a]]);
    total += s * id2[a];
  }
  return total;
}

static double eta_at(const double* ex, const double* ey, const double* ez,
                     int i, int j, int k) {
  if (!ex) return 0.0;
  return ex[i] + ey[j] + ez[k];
}

/* ---------------------------------------------------------------- setup */

/* Time step from the Courant number C = vmax*dt/min(d). */
double ora_cfl_dt(const float* v, int64_t n, double dmin, double courant) {
  double vmax = 0.0;
  for (int64_t p = 0; p < n; ++p)
    if ((double)v[p] > vmax) vmax = (double)v[p];
  return courant * dmin / vmax;
}

/* Ricker wavelet of peak frequency f0 delayed by t0, sampled at t = (n0+n)*dt:
 * w = (1 - 2 a) exp(-a), a = (pi f0 (t - t0))^2. */
void ora_ricker(double* w, int nt, int n0, double dt, double f0, double t0) {
  const double pi = 3.14159265358979323846;
  for (int n = 0; n < nt; ++n) {
    double t = (double)(n0 + n) * dt;
    double a = pi * f0 * (t - t0);
    a = a * a;
    w[n] = (1.0 - 2.0 * a) * exp(-a);
  }
}

/* Peak damping of a quadratic absorbing layer of W cells with target
 * reflection R (Collino and Tsogka 2001): 3 vmax ln(1/R) / (2 W d). */
double ora_sponge_sigma_max(double vmax, double d, int W, double R) {
  if (W <= 0) return 0.0;
  return 3.0 * vmax * log(1.0 / R) / (2.0 * (double)W * d);
}

/* eta(i) = (dt/2) sigma_max (delta(i)/W)^2, delta(i) = max(W-i, i-(n-1-W), 0):
 * the W outermost cells of each side are damped. */
void ora_sponge_eta(double* eta, int n, int W, double sigma_max, double dt) {
  for (int i = 0; i < n; ++i) {
    double e = 0.0;
    if (W > 0) {
      int d = W - i;
      int d2 = i - (n - 1 - W);
      if (d2 > d) d = d2;
      if (d < 0) d = 0;
      double r = (double)d / (double)W;
      e = 0.5 * dt * sigma_max * r * r;
    }
    eta[i] = e;
  }
}

/* ------------------------------------------------------------- halos */

static int wrap(int i, int n) {
  int r = i % n;
  return r < 0 ? r + n : r;
}

/* Periodic face halos (what a loopback exchange of the six faces yields).
 * Edges and corners are never read by a star stencil and stay as they are. */
void ora_fill_halo_periodic(int nx, int ny, int nz, double* u) {
  box b = mkbox(nx, ny, nz, 1, 1, 1);
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int h = 1; h <= OH; ++h) {
        u[at(&b, -h, j, k)] = u[at(&b, wrap(-h, nx), j, k)];
        u[at(&b, nx - 1 + h, j, k)] = u[at(&b, wrap(nx - 1 + h, nx), j, k)];
      }
  for (int k = 0; k < nz; ++k)
    for (int h = 1; h <= OH; ++h)
      for (int i = 0; i < nx; ++i) {
        u[at(&b, i, -h, k)] = u[at(&b, i, wrap(-h, ny), k)];
        u[at(&b, i, ny - 1 + h, k)] = u[at(&b, i, wrap(ny - 1 + h, ny), k)];
      }
  for (int h = 1; h <= OH; ++h)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        u[at(&b, i, j, -h)] = u[at(&b, i, j, wrap(-h, nz))];
        u[at(&b, i, j, nz - 1 + h)] = u[at(&b, i, j, wrap(nz - 1 + h, nz))];
      }
}

/* ------------------------------------------------------ spatial operator */

/* out = L u on the interior; the halo of u is used as given. */
void ora_laplacian(int nx, int ny, int nz, double dx, double dy, double dz,
                   const double* u, double* out) {
  box b = mkbox(nx, ny, nz, dx, dy, dz);
#pragma omp parallel for schedule(static)
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        int64_t c = at(&b, i, j, k);
        out[c] = lap_at(&b, u, c);
      }
}

/* One leapfrog update on the interior, the halo of u used as given:
 * (1+eta) u_next = 2 u - (1-eta) u_prev + vdt2 * L u. */
void ora_step(int nx, int ny, int nz, double dx, double dy, double dz,
              const double* up, const double* u, double* un, const double* vdt2,
              const double* ex, const double* ey, const double* ez) {
  box b = mkbox(nx, ny, nz, dx, dy, dz);
#pragma omp parallel for schedule(static)
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        int64_t c = at(&b, i, j, k);
        double eta = eta_at(ex, ey, ez, i, j, k);
        un[c] = (2.0 * u[c] - (1.0 - eta) * up[c] + vdt2[c] * lap_at(&b, u, c)) /
                (1.0 + eta);
      }
}

/* Source term added to the updated field: vdt2*w/(1+eta) at (si,sj,sk). */
static void add_source(const box* b, double* un, const double* vdt2,
                       const double* ex, const double* ey, const double* ez,
                       int si, int sj, int sk, double w) {
  int64_t c = at(b, si, sj, sk);
  un[c] += vdt2[c] * w / (1.0 + eta_at(ex, ey, ez, si, sj, sk));
}


static void load_interior(const box* b, const double* src, double* dst) {
  for (int k = 0; k < b->nz; ++k)
    for (int j = 0; j < b->ny; ++j)
      for (int i = 0; i < b->nx; ++i)
        dst[at(b, i, j, k)] = src[((int64_t)k * b->ny + j) * b->nx + i];
}

static void zero_box_load(const box* b, const double* src, double* dst) {
  memset(dst, 0, sizeof(double) * ora_elems(b->nx, b->ny, b->nz));
  load_interior(b, src, dst);
}

static void store_interior(const box* b, const double* src, double* dst) {
  for (int k = 0; k < b->nz; ++k)
    for (int j = 0; j < b->ny; ++j)
      for (int i = 0; i < b->nx; ++i)
        dst[((int64_t)k * b->ny + j) * b->nx + i] = src[at(b, i, j, k)];
}

/* vdt2 = (v dt)^2 on the interior, returned as an interior (nz,ny,nx) array. */
void ora_vdt2(int nx, int ny, int nz, const float* v, double dt, double* out) {
  int64_t n = (int64_t)nx * ny * nz;
  for (int64_t p = 0; p < n; ++p) {
    double vv = (double)v[p] * dt;
    out[p] = vv * vv;
  }
}

/* Forward model: nt leapfrog steps from (state_prev, state_cur) (NULL = zero)
 * with q = vdt2 = (v dt)^2 given as an FP64 interior array, source wavelet w[nt] at (si,sj,sk)
 * (w NULL = no source), sponge tables (all NULL = none), periodic (1) or zero
 * Dirichlet (0) halos.  Step n: fill halo of u^n, update, add w[n] at the
 * source, record traces[n][r] = u^{n+1}(rec r), rotate.  On return
 * state_prev/state_cur (if non-NULL) hold u^{nt-1}, u^{nt}. */
int ora_forward(int nx, int ny, int nz, double dx, double dy, double dz,
                const double* q, int nt, const double* w, int si,
                int sj, int sk, const double* ex, const double* ey,
                const double* ez, int periodic, int nrec, const int32_t* rec,
                double* traces, double* state_prev, double* state_cur) {
  box b = mkbox(nx, ny, nz, dx, dy, dz);
  int64_t ne = ora_elems(nx, ny, nz);
  double* vdt2 = (double*)malloc(sizeof(double) * ne);
  double* a0 = (double*)calloc(ne, sizeof(double));
  double* a1 = (double*)calloc(ne, sizeof(double));
  double* a2 = (double*)calloc(ne, sizeof(double));
  if (!vdt2 || !a0 || !a1 || !a2) {
    free(vdt2); free(a0); free(a1); free(a2);
    return -12;
  }
  zero_box_load(&b, q, vdt2);
  if (state_prev) load_interior(&b, state_prev, a0);
  if (state_cur) load_interior(&b, state_cur, a1);
  double *up = a0, *u = a1, *un = a2;
  for (int n = 0; n < nt; ++n) {
    if (periodic) ora_fill_halo_periodic(nx, ny, nz, u);
    ora_step(nx, ny, nz, dx, dy, dz, up, u, un, vdt2, ex, ey, ez);
    if (w) add_source(&b, un, vdt2, ex, ey, ez, si, sj, sk, w[n]);
    for (int r = 0; r < nrec; ++r)
      traces[(int64_t)n * nrec + r] = un[at(&b, rec[3 * r], rec[3 * r + 1], rec[3 * r + 2])];
    double* t = up; up = u; u = un; un = t;
  }
  if (state_prev) store_interior(&b, up, state_prev);
  if (state_cur) store_interior(&b, u, state_cur);
  free(vdt2); free(a0); free(a1); free(a2);
  return 0;
}

/* One step evaluated at selected interior points only, straight from
 * float32 interior arrays (nz,ny,nx) of u^{n-1} and u^n and an FP64 interior
 * array q = vdt2: neighbours outside
 * the interior are wrapped (periodic) or zero (Dirichlet).  The source term
 * w_src is added where the point is the source (si < 0: none). */
void ora_step_points(int nx, int ny, int nz, double dx, double dy, double dz,
                     const float* up, const float* u, const double* q,
                     const double* ex, const double* ey, const double* ez,
                     int periodic, double w_src, int si, int sj, int sk,
                     int npts, const int32_t* pts, double* out) {
  const double id2[3] = {1.0 / (dx * dx), 1.0 / (dy * dy), 1.0 / (dz * dz)};
  const int n3[3] = {nx, ny, nz};
#pragma omp parallel for schedule(static)
  for (int p = 0; p < npts; ++p) {
    int pt[3] = {pts[3 * p], pts[3 * p + 1], pts[3 * p + 2]};
    int64_t c = ((int64_t)pt[2] * ny + pt[1]) * nx + pt[0];
    double lap = 0.0;
    for (int a = 0; a < 3; ++a) {
      double s = CM[0] * (double)u[c];
      for (int m = 1; m <= 4; ++m) {
        double pair = 0.0;
        for (int sgn = -1; sgn <= 1; sgn += 2) {
          int r[3] = {pt[0], pt[1], pt[2]};
          r[a] += sgn * m;
          if (r[a] < 0 || r[a] >= n3[a]) {
            if (!periodic) continue;
            r[a] = wrap(r[a], n3[a]);
          }
          pair += (double)u[((int64_t)r[2] * ny + r[1]) * nx + r[0]];
        }
        s += CM[m] * pair;
      }
      lap += s * id2[a];
    }
    double eta = eta_at(ex, ey, ez, pt[0], pt[1], pt[2]);
    double vdt2 = q[c];
    double r = (2.0 * (double)u[c] - (1.0 - eta) * (double)up[c] + vdt2 * lap) / (1.0 + eta);
    if (pt[0] == si && pt[1] == sj && pt[2] == sk) r += vdt2 * w_src / (1.0 + eta);
    out[p] = r;
  }
}

/* ------------------------------------------------------------- adjoint */

/* Transpose of one forward step with respect to its two state inputs.
 * Writing D = 1/(1+eta), E = 1-eta, Q = vdt2, the forward step is
 * u^{n+1} = D (2 u^n - E u^{n-1} + Q (L u^n + f^n)).  Given the cotangents
 * c = lambda^{n+1} and c2 = lambda^{n+2} (interior, padded FP64 boxes),
 * a_out = 2 D c + L(Q D c) - E D c2.  The halo of Q D c is zero (Dirichlet) or
 * its periodic image.  If g is non-NULL, g += D c (L u^n + f^n) with f^n = w at
 * the source (si < 0: no source), the halo of u_n used as given. */
void ora_adjoint_step(int nx, int ny, int nz, double dx, double dy, double dz,
                      const double* c2, const double* c, double* a_out,
                      const double* vdt2, const double* ex, const double* ey,
                      const double* ez, int periodic, const double* u_n,
                      double* g, double w, int si, int sj, int sk) {
  box b = mkbox(nx, ny, nz, dx, dy, dz);
  int64_t ne = ora_elems(nx, ny, nz);
  double* p = (double*)calloc(ne, sizeof(double));
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        int64_t q = at(&b, i, j, k);
        p[q] = vdt2[q] * c[q] / (1.0 + eta_at(ex, ey, ez, i, j, k));
      }
  if (periodic) ora_fill_halo_periodic(nx, ny, nz, p);
#pragma omp parallel for schedule(static)
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        int64_t q = at(&b, i, j, k);
        double eta = eta_at(ex, ey, ez, i, j, k);
        double D = 1.0 / (1.0 + eta);
        double cc = c[q];
        if (g) {
          double lu = u_n ? lap_at(&b, u_n, q) : 0.0;
          if (i == si && j == sj && k == sk) lu += w;
          g[q] += D * cc * lu;
        }
        a_out[q] = 2.0 * D * cc + lap_at(&b, p, q) - (1.0 - eta) * D * (c2 ? c2[q] : 0.0);
      }
  free(p);
}

/* Full-waveform-inversion gradient by the adjoint-state method with every
 * forward state stored (small grids only).
 * J = 1/2 sum_n sum_r (traces[n][r] - obs[n][r])^2.
 * Reverse sweep n = nt-1 .. 0 with lambda^{n+1} = a^{n+1} + R^T res[n]:
 *   g_vdt2 += D lambda^{n+1} (L u^n + f^n)
 *   a^n    += 2 D lambda^{n+1} + L(Q D lambda^{n+1})
 *   a^{n-1} += -E D lambda^{n+1}
 * q = vdt2 is an FP64 interior array.
 * grad_m = -g_vdt2 vdt2^2 / dt^2 (vdt2 = dt^2/m with m = 1/v^2, dt frozen);
 * grad_w[n] = D Q lambda^{n+1} at the source.  Returns J (or -1 on OOM). */
double ora_fwi_gradient(int nx, int ny, int nz, double dx, double dy, double dz,
                        const double* q, double dt, int nt, const double* w,
                        int si, int sj, int sk, const double* ex,
                        const double* ey, const double* ez, int periodic,
                        int nrec, const int32_t* rec, const double* obs,
                        double* traces_out, double* g_vdt2_out,
                        double* grad_m_out, double* grad_w_out) {
  box b = mkbox(nx, ny, nz, dx, dy, dz);
  int64_t ne = ora_elems(nx, ny, nz);
  double* vdt2 = (double*)malloc(sizeof(double) * ne);
  double* states = (double*)calloc((size_t)ne * (nt + 1), sizeof(double));
  double* zero = (double*)calloc(ne, sizeof(double));
  double* res = (double*)malloc(sizeof(double) * ((size_t)nt * nrec + 1));
  double* A[3];
  for (int t = 0; t < 3; ++t) A[t] = (double*)calloc(ne, sizeof(double));
  double* g = (double*)calloc(ne, sizeof(double));
  if (!vdt2 || !states || !zero || !res || !A[0] || !A[1] || !A[2] || !g) {
    free(vdt2); free(states); free(zero); free(res); free(g);
    for (int t = 0; t < 3; ++t) free(A[t]);
    return -1.0;
  }
  zero_box_load(&b, q, vdt2);
  /* forward, keeping u^n (with the halo it had when stepped) for n = 0..nt */
  double J = 0.0;
  for (int n = 0; n < nt; ++n) {
    double* up = n > 0 ? states + (size_t)(n - 1) * ne : zero;
    double* u = states + (size_t)n * ne;
    double* un = states + (size_t)(n + 1) * ne;
    if (periodic) ora_fill_halo_periodic(nx, ny, nz, u);
    ora_step(nx, ny, nz, dx, dy, dz, up, u, un, vdt2, ex, ey, ez);
    if (w) add_source(&b, un, vdt2, ex, ey, ez, si, sj, sk, w[n]);
    for (int r = 0; r < nrec; ++r) {
      double d = un[at(&b, rec[3 * r], rec[3 * r + 1], rec[3 * r + 2])];
      if (traces_out) traces_out[(int64_t)n * nrec + r] = d;
      double e = d - obs[(int64_t)n * nrec + r];
      res[(int64_t)n * nrec + r] = e;
      J += 0.5 * e * e;
    }
  }
  /* reverse sweep; A[m % 3] accumulates a^m */
  for (int n = nt - 1; n >= 0; --n) {
    double* c = A[(n + 1) % 3];
    double* cur = A[n % 3];
    double* old = A[(n + 2) % 3]; /* held lambda^{n+2}, no longer needed */
    for (int r = 0; r < nrec; ++r)
      c[at(&b, rec[3 * r], rec[3 * r + 1], rec[3 * r + 2])] += res[(int64_t)n * nrec + r];
    /* a^n gets 2Dc + L(QDc) on top of what it already holds (-E D lambda^{n+2});
     * a^{n-1} starts fresh with -E D c. */
    double* tmp = (double*)calloc(ne, sizeof(double));
    ora_adjoint_step(nx, ny, nz, dx, dy, dz, NULL, c, tmp, vdt2, ex, ey, ez,
                     periodic, states + (size_t)n * ne, g, w ? w[n] : 0.0,
                     w ? si : -1, sj, sk);
    memset(old, 0, sizeof(double) * ne);
    for (int k = 0; k < nz; ++k)
      for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
          int64_t q = at(&b, i, j, k);
          double eta = eta_at(ex, ey, ez, i, j, k);
          cur[q] += tmp[q];
          old[q] = -(1.0 - eta) * c[q] / (1.0 + eta);
        }
    if (grad_w_out) {
      int64_t s = at(&b, si, sj, sk);
      grad_w_out[n] = vdt2[s] * c[s] / (1.0 + eta_at(ex, ey, ez, si, sj, sk));
    }
    free(tmp);
  }
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        int64_t q = at(&b, i, j, k);
        int64_t o = ((int64_t)k * ny + j) * nx + i;
        if (g_vdt2_out) g_vdt2_out[o] = g[q];
        if (grad_m_out) grad_m_out[o] = -g[q] * vdt2[q] * vdt2[q] / (dt * dt);
      }
  free(vdt2); free(states); free(zero); free(res); free(g);
  for (int t = 0; t < 3; ++t) free(A[t]);
  return J;
}

/* ---------------------------------------------------------------------------
 * Cannon's matrix multiply (Sec. 4.4): each of P ranks holds a stripe of Ns = N/P
 * rows and performs P products of N * Ns * Ns multiply-adds; the product of one
 * step is a plain block product.  Here, by its definition, in FP64:
 *     C[i][j] = (accumulate ? C[i][j] : 0) + sum over p = 0 .. k-1 of A[i][p] B[p][j]
 * for 0 <= i < m, 0 <= j < n; row-major operands with leading dimensions lda, ldb,
 * ldc (elements between consecutive rows).  The sum runs over p in increasing
 * order, starting from the old C[i][j] (or 0).  Rows of C are independent (one
 * thread per row block; the arithmetic of an element never depends on it). */
void ora_block_gemm(int64_t m, int64_t n, int64_t k, const double* a, int64_t lda,
                    const double* b, int64_t ldb, double* c, int64_t ldc, int accumulate) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < m; ++i)
    for (int64_t j = 0; j < n; ++j) {
      double s = accumulate ? c[i * ldc + j] : 0.0;
      for (int64_t p = 0; p < k; ++p) s += a[i * lda + p] * b[p * ldb + j];
      c[i * ldc + j] = s;
    }
}

/* Sets the OpenMP threads of later parallel regions (n >= 1). */
void ora_set_threads(int n) {
  if (n >= 1) omp_set_num_threads(n);
}

/* Threads an OpenMP region of this library uses (for reporting only). */
int ora_threads(void) {
  int n = 1;
#pragma omp parallel
  {
#pragma omp single
    n = omp_get_num_threads();
  }
  return n;
}
