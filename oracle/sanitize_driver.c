/* Test driver (test infrastructure): exercises every oracle entry point on small
 * grids so the test suite can run them under AddressSanitizer and
 * UndefinedBehaviorSanitizer on the host.  Exit status 0 when all calls ran. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int64_t ora_elems(int nx, int ny, int nz);
double ora_cfl_dt(const float* v, int64_t n, double dmin, double courant);
void ora_ricker(double* w, int nt, int n0, double dt, double f0, double t0);
double ora_sponge_sigma_max(double vmax, double d, int W, double R);
void ora_sponge_eta(double* eta, int n, int W, double sigma_max, double dt);
void ora_fill_halo_periodic(int nx, int ny, int nz, double* u);
void ora_laplacian(int nx, int ny, int nz, double dx, double dy, double dz, const double* u,
                   double* out);
void ora_vdt2(int nx, int ny, int nz, const float* v, double dt, double* out);
int ora_forward(int nx, int ny, int nz, double dx, double dy, double dz, const double* q,
                int nt, const double* w, int si, int sj, int sk, const double* ex,
                const double* ey, const double* ez, int periodic, int nrec,
                const int32_t* rec, double* traces, double* sp, double* sc);
void ora_step_points(int nx, int ny, int nz, double dx, double dy, double dz, const float* up,
                     const float* u, const double* q, const double* ex, const double* ey,
                     const double* ez, int periodic, double w_src, int si, int sj, int sk,
                     int npts, const int32_t* pts, double* out);
double ora_fwi_gradient(int nx, int ny, int nz, double dx, double dy, double dz,
                        const double* q, double dt, int nt, const double* w, int si, int sj,
                        int sk, const double* ex, const double* ey, const double* ez,
                        int periodic, int nrec, const int32_t* rec, const double* obs,
                        double* traces_out, double* g_out, double* gm_out, double* gw_out);

int main(void) {
  const int shapes[3][3] = {{5, 4, 6}, {9, 7, 8}, {1, 1, 1}};
  for (int s = 0; s < 3; ++s) {
    const int nx = shapes[s][0], ny = shapes[s][1], nz = shapes[s][2];
    const int n = nx * ny * nz, nt = 12, W = nx > 4 ? 2 : 0;
    float* v = malloc(sizeof(float) * n);
    float* uf = malloc(sizeof(float) * n);
    double* q = malloc(sizeof(double) * n);
    double *ex = malloc(sizeof(double) * nx), *ey = malloc(sizeof(double) * ny),
           *ez = malloc(sizeof(double) * nz);
    for (int i = 0; i < n; ++i) { v[i] = 1500.f + (float)(i % 7) * 100.f; uf[i] = (float)(i % 5); }
    const double dt = ora_cfl_dt(v, n, 10.0, 0.4);
    ora_vdt2(nx, ny, nz, v, dt, q);
    const double sm = ora_sponge_sigma_max(2100.0, 10.0, W, 1e-3);
    ora_sponge_eta(ex, nx, W, sm, dt);
    ora_sponge_eta(ey, ny, W, sm, dt);
    ora_sponge_eta(ez, nz, W, sm, dt);
    double* w = malloc(sizeof(double) * nt);
    ora_ricker(w, nt, 0, dt, 15.0, 1.0 / 15.0);
    const int32_t rec[6] = {0, 0, 0, nx - 1, ny - 1, nz - 1};
    double* tr = malloc(sizeof(double) * nt * 2);
    double* st0 = calloc(n, sizeof(double));
    double* st1 = calloc(n, sizeof(double));
    for (int periodic = 0; periodic < 2; ++periodic) {
      if (ora_forward(nx, ny, nz, 10, 10, 10, q, nt, w, nx / 2, ny / 2, nz / 2, ex, ey, ez,
                      periodic, 2, rec, tr, st0, st1) != 0)
        return 2;
      double* out = malloc(sizeof(double) * 2);
      ora_step_points(nx, ny, nz, 10, 10, 10, uf, uf, q, ex, ey, ez, periodic, 0.5, 0, 0, 0, 2,
                      rec, out);
      free(out);
      double* obs = calloc(nt * 2, sizeof(double));
      double *g = malloc(sizeof(double) * n), *gm = malloc(sizeof(double) * n),
             *gw = malloc(sizeof(double) * nt), *t2 = malloc(sizeof(double) * nt * 2);
      const double J = ora_fwi_gradient(nx, ny, nz, 10, 10, 10, q, dt, nt, w, nx / 2, ny / 2,
                                        nz / 2, ex, ey, ez, periodic, 2, rec, obs, t2, g, gm, gw);
      if (!(J >= 0)) return 3;
      free(obs); free(g); free(gm); free(gw); free(t2);
    }
    const int64_t ne = ora_elems(nx, ny, nz);
    double* box = calloc(ne, sizeof(double));
    double* lo = calloc(ne, sizeof(double));
    ora_fill_halo_periodic(nx, ny, nz, box);
    ora_laplacian(nx, ny, nz, 10, 10, 10, box, lo);
    free(box); free(lo); free(v); free(uf); free(q); free(ex); free(ey); free(ez); free(w);
    free(tr); free(st0); free(st1);
  }
  printf("sanitized oracle driver: ok\n");
  return 0;
}
