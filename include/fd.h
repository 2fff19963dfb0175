/*
 * fd.h -- C ABI of the MI355X acoustic isotropic finite-difference library
 * (libfd.so, HIP for gfx950).
 *
 * What it computes.  The acoustic isotropic wave-propagation kernel that the
 * paper evaluates as its real-world application (Sec. 4.5: the Minimod proxy
 * application, seismic wave propagation by finite differences with a wide
 * stencil, run on 1200^3 grids for 1000 steps), on ONE device's subdomain,
 * together with the pack and unpack of the subdomain's boundary planes that the paper's
 * halo exchange moves between neighbouring ranks with one-sided puts and a
 * fence (Listing 1).  The paper does not state the stencil; this library uses
 *   - 8th order in space: per axis the 9-point central second difference
 *     c0 = -205/72, c1 = 8/5, c2 = -1/5, c3 = 8/315, c4 = -1/560, divided by
 *     the squared spacing; the three axes summed (a 25-point star, radius 4);
 *   - 2nd order in time (leapfrog) with an optional damping sponge eta >= 0:
 *       u_next = (2 u - (1 - eta) u_prev + vdt2 * L u) / (1 + eta),
 *     where vdt2 = (v dt)^2 and eta = eta_x[i] + eta_y[j] + eta_z[k];
 *   - a point source added after the update: u_next[s] += vdt2[s] w / (1+eta[s]);
 *   - receivers sampling the updated field.
 * All arithmetic on the device is FP32.
 *
 * Memory layout.  Every volume array is FP32, x fastest, with a halo of
 * H = 4 points on each face.  Interior point (i, j, k), 0 <= i < nx etc., is
 * element  origin + k*zstride + j*ystride + i;  halo points use i, j or k in
 * [-4, 0) or [n, n+4).  fd_grid_init picks an origin and strides that put
 * every interior row start on a 128-byte boundary.
 *
 * Conventions.
 *   - Pointers named *_dev or documented as "device" are device pointers
 *     owned by the caller; the library never frees or retains them.  The
 *     stepping calls (fd_step through fd_grad_finalize_scaled below) never
 *     allocate.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Calls enqueue work on it and return without synchronising, except
 *     where a call says it synchronises.
 *   - Return value: FD_OK or a negative FD_E* code; nothing is enqueued when
 *     a call returns an error.  fd_strerror() names a code; fd_last_error()
 *     returns a thread-local detail string for the last failing call.
 *   - Device faults in enqueued kernels surface at the caller's next
 *     synchronisation, as for any HIP kernel.
 *   - No C++ exception crosses this boundary.
 */
#ifndef FD_H
#define FD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FD_HALO 4

enum {
  FD_OK = 0,
  FD_ENOTFOUND = -2,   /* unknown shot id                                  */
  FD_EDEVICE = -5,     /* a HIP runtime or launch error                    */
  FD_EAGAIN = -11,     /* shot not finished yet                            */
  FD_ENOMEM = -12,     /* cannot fit in the given memory                   */
  FD_EINVAL = -22,     /* invalid argument, geometry or aliasing           */
  FD_ECANCELED = -125  /* shot cancelled by server shutdown                */
};

/* Geometry shared by every volume array of one call. */
typedef struct fd_grid {
  int32_t nx, ny, nz;       /* interior extent, each >= 1                            */
  int32_t halo;             /* must be FD_HALO (the stencil radius)                  */
  int64_t origin;           /* element offset of interior (0,0,0); >= 4*zstride+4*ystride+4 */
  int64_t ystride, zstride; /* element strides; ystride >= nx+8,
                               zstride >= ystride*(ny+8), zstride <= 2^29            */
  double dx, dy, dz;        /* grid spacing (metres), finite and > 0                 */
} fd_grid;

/* Damping tables (device pointers, FP32, lengths nx, ny, nz).  All three NULL
 * (or a NULL fd_sponge*) means no sponge.  eta = (dt/2) * sigma, see
 * fd_sponge_eta_max / fd_sponge_profile. */
typedef struct fd_sponge {
  const float* eta_x;
  const float* eta_y;
  const float* eta_z;
} fd_sponge;

/* A point source term: w added at interior point (i, j, k). */
typedef struct fd_source {
  int32_t i, j, k;
  float w;
} fd_source;

/* ------------------------------------------------------------- errors */

/* Static description of a return code; never NULL. */
const char* fd_strerror(int code);
/* Detail of the last error raised on the calling thread ("" if none). */
const char* fd_last_error(void);
/* ABI version (major*10000 + minor*100 + patch). */
int fd_version(void);

/* ----------------------------------------------------------- geometry */

/* The subdomain of one rank with its boundary planes (Sec. 4.5 and Listing 1:
 * each rank owns a block of the grid and exchanges the planes next to its
 * faces); the paper gives no memory layout, the one below is this library's.
 *
 * Fill *g for an nx*ny*nz interior with spacing (dx,dy,dz): halo 4, the
 * interior row start 128-byte aligned (32 floats of left padding, of which
 * the last 4 are the x halo), ystride a multiple of 32 floats, zstride =
 * ystride*(ny+8).  FD_EINVAL on bad sizes or spacing, or if zstride would
 * exceed 2^29 elements. */
int fd_grid_init(fd_grid* g, int32_t nx, int32_t ny, int32_t nz, double dx,
                 double dy, double dz);
/* Floats the caller must allocate per volume array (origin + the furthest
 * halo element + 1); -1 for an invalid grid. */
int64_t fd_grid_elems(const fd_grid* g);
/* Floats of face buffer `face` (0..5 = -x,+x,-y,+y,-z,+z): 4*ny*nz for x
 * faces, 4*nx*nz for y faces, 4*nx*ny for z faces; -1 if invalid. */
int64_t fd_face_elems(const fd_grid* g, int32_t face);
/* Element offset of point (i,j,k) (halo indices allowed); -1 if outside
 * [-4, n+4) on an axis. */
int64_t fd_offset(const fd_grid* g, int32_t i, int32_t j, int32_t k);

/* Performance knobs (no passage of the paper defines them; they change launch
 * shapes, never results).
 *
 * Number of z planes each block of the stencil kernels
 * marches through (0 = automatic, the default).  Process-wide; results do not
 * depend on it. */
int fd_set_kchunk(int32_t kchunk);

/* Performance knob: tile shape of the forward stencil kernels (fd_step,
 * fd_step_fused, fd_step_exchange, fd_forward_run, fd_adjoint_step_scaled):
 * 0 = automatic: a forward update that takes no faces inside the kernel --
 * fd_step, fd_step_fused, fd_forward_run without a second face set,
 * fd_adjoint_step_scaled(_res) -- runs one thread per point on grids of at most
 * 2^22 points, which stay in cache and whose step is latency-bound, and so does
 * fd_step_exchange / fd_forward_run with all twelve face buffers on grids of at
 * most 2^21 points, the faces then read and written in that one launch; grids of
 * at least 7.5 million points take the kernel of 16-byte lanes (the exchange form
 * where nx is a multiple of 128, with 128 x 32 tiles; the update without faces and
 * the gradient pass with 128 x 32 tiles, or 64 x 64 where the launch model prefers
 * them by a tenth, i.e. where a 128-wide tile column would be mostly empty; arrays
 * and face buffers 16-byte aligned); the others the z-marching kernel of one float
 * per lane, 64 x 16 tiles for grids of at most 2^20 points, 64 x 32 above.  1 =
 * always 64 x 32, 2 = always 64 x 16 (both: never one thread per point nor 16-byte
 * lanes), 3 = one thread per point wherever it applies (64 x 16 elsewhere), 4 =
 * 16-byte lanes wherever they apply, 128 x 32 tiles (64 x 32 elsewhere), 5 = the
 * same with 64 x 64 tiles where the 16-byte-lane kernel takes no faces.
 * Process-wide; results do not depend on it (fd_step_kernel reports the choice).
 * FD_EINVAL for another mode. */
int fd_set_tiles(int32_t mode);

/* Launch shape of the z-marching forward stencil kernel of one float per lane
 * (where a step over g takes it, see fd_set_tiles and fd_step_kernel) as the next
 * such call would use it: out[0..3] = x tiles, y tiles, z planes per block, z
 * chunks (blocks = their product; a tile is 64 x 32 points, or 64 x 16, see
 * fd_set_tiles).  Host only, no device call; FD_EINVAL for a bad grid or NULL out. */
int fd_step_launch(const fd_grid* g, int32_t out[4]);

/* Which forward kernel a step over g takes, as the next call would choose it
 * (process-wide fd_set_tiles mode included; volume arrays and face buffers
 * assumed 16-byte aligned, as torch allocates them): with_faces != 0 for
 * fd_step_exchange / fd_forward_run with all twelve face buffers, 0 for fd_step /
 * fd_step_fused / fd_forward_run without faces (no receiver row in the kernel).
 * out[0] = FD_KERNEL_*, out[1], out[2] = tile width and height in points (1 x 1:
 * one thread per point), out[3] = z planes per block, out[4] = z chunks, out[5] =
 * blocks (-1 for the one-thread-per-point kernel).  Host only; FD_EINVAL for a bad
 * grid or NULL out. */
enum {
  FD_KERNEL_POINT = 0,        /* one thread per point (small grids, in cache)   */
  FD_KERNEL_MARCH_64x32 = 1,  /* z-marching, one float per lane, 64 x 32 tiles  */
  FD_KERNEL_MARCH_64x16 = 2,  /* the same with 64 x 16 tiles                    */
  FD_KERNEL_WIDE = 3,         /* z-marching, 16-byte lanes, 128 x 32 tiles      */
  FD_KERNEL_WIDE_64x64 = 4    /* the same with 64 x 64 tiles (ragged x extents) */
};
int fd_step_kernel(const fd_grid* g, int32_t with_faces, int32_t out[6]);

/* ----------------------------------------------------------- model prep
 * (set-up, step S0; not on the per-step path).  The paper names the acoustic
 * isotropic kernel (Sec. 4.5) but states no time step, velocity scaling,
 * boundary damping, source or receivers; each call below is one reading of
 * what such a kernel needs, stated with the call. */

/* Device reduction of max(v) over the interior of v; writes it to
 * *vmax_host and computes dt = courant * min(dx,dy,dz) / max(v) into *dt_out
 * (either pointer may be NULL).  SYNCHRONISES `stream`.  `scratch_dev` is a
 * caller-owned device buffer of at least 2 int32.  FD_EINVAL unless every
 * interior velocity is > 0 and the maximum is finite. */
int fd_cfl_dt(const fd_grid* g, const float* v, double courant, int32_t* scratch_dev,
              double* vmax_host, double* dt_out, void* stream);

/* fd_cfl_dt without the caller's workspace, for callers that cannot allocate
 * device memory (code under stream capture, tight serving loops, harnesses that
 * forbid allocation): the two result slots live in the library's own static
 * device array (256 bytes per device, 64 int32 of which this call uses 2; no grid
 * size needs more, so none is refused for lack of room), which each device that
 * runs the library holds until the process ends.  No device or host memory is
 * allocated: the array's device address is looked up once per device, on the
 * first call made with that device current.  The slots are reset by a kernel at
 * every call.  All calls on one device share them: calls that overlap in time on
 * one device (several host threads, several streams) race and must be
 * serialised by the caller.  Same results, synchronisation and errors as
 * fd_cfl_dt (FD_EDEVICE if the array cannot be looked up). */
int fd_cfl_dt_static(const fd_grid* g, const float* v, double courant, double* vmax_host,
                     double* dt_out, void* stream);

/* vdt2 = (v*dt)^2, evaluated in FP64 and rounded to FP32, on every point of
 * the padded box [-4,n+4)^3 of vdt2: the interior from v's interior, each
 * face halo from the periodic image of the interior (i mod n), edges and
 * corners 0.  Only v's interior is read.  v and vdt2 must not overlap. */
int fd_prepare_vdt2(const fd_grid* g, const float* v, float* vdt2, double dt,
                    void* stream);

/* As fd_prepare_vdt2 from squared slowness m = 1/v^2: vdt2 = dt^2 / m
 * (FP64, rounded to FP32), same halo treatment.  FD_EINVAL on bad input;
 * m must be > 0 on the interior (not checked on the device). */
int fd_prepare_vdt2_m(const fd_grid* g, const float* m, float* vdt2, double dt,
                      void* stream);

/* Host helper: peak eta = (dt/2) * sigma_max of a quadratic absorbing layer
 * of `width` cells with target normal-incidence reflection R, where
 * sigma_max = 3 vmax ln(1/R) / (2 width d) (Collino & Tsogka 2001).
 * Returns 0 for width <= 0, negative FD_EINVAL on bad input. */
double fd_sponge_eta_max(double vmax, double d, double dt, int32_t width, double R);

/* Host helper: eta(i) = eta_max * (delta(i)/width)^2 for i < n, where
 * delta(i) = max(width - i, i - (n-1-width), 0); all zeros for width <= 0.
 * host_out has n floats. */
int fd_sponge_profile(float* host_out, int32_t n, int32_t width, double eta_max);

/* Host helper: Ricker wavelet w[n] = (1 - 2a) exp(-a), a = (pi f0 (t-t0))^2,
 * t = (n0+n)*dt, evaluated in FP64 and stored as FP32; host_out has nt floats. */
int fd_ricker(float* host_out, int32_t nt, int32_t n0, double dt, double f0, double t0);

/* Host helper: element offsets of nrec receivers given as (i,j,k) triples
 * (3*nrec int32, host) into off_host (nrec int64, host).  FD_EINVAL if a
 * receiver lies outside the interior. */
int fd_receiver_offsets(const fd_grid* g, const int32_t* ijk_host, int32_t nrec,
                        int64_t* off_host);

/* ------------------------------------------------------- per-step path */

/* S4, the stencil update that the paper's Minimod runs as one device kernel
 * per time step over the rank's subdomain (Sec. 4.5); the stencil order and
 * the time scheme are this library's reading (file header).
 * One leapfrog update of every interior point,
 *   u_next = (2u - (1-eta) u_prev + vdt2 * L u) / (1+eta)
 * (eta = 0 without a sponge).  L reads u's face halos as they are (zeros for
 * a Dirichlet boundary, or what halo_unpack wrote).  Reads only interior
 * points of u_prev and vdt2; writes only interior points of u_next.
 * u_next may alias u_prev (in-place two-array stepping); it must not overlap
 * u.  sp may be NULL. */
int fd_step(const fd_grid* g, const float* u_prev, const float* u, float* u_next,
            const float* vdt2, const fd_sponge* sp, void* stream);

/* S4+S5+S1 in one call (Sec. 4.5 update, then the pack of the planes that
 * Listing 1 puts to the neighbours): fd_step with (src non-NULL) the source term src->w
 * added in the same kernel exactly as inject_source adds it, then
 * (face_out non-NULL) the six-face pack of the new u_next exactly as
 * halo_pack writes it (NULL entries skipped; faces need n >= 4 on their axis
 * and must not overlap a volume array).  Bitwise the same results as
 * fd_step + inject_source + halo_pack; one stencil launch plus the pack. */
int fd_step_fused(const fd_grid* g, const float* u_prev, const float* u, float* u_next,
                  const float* vdt2, const fd_sponge* sp, const fd_source* src,
                  float* const face_out[6], void* stream);

/* S3+S4+S5+S1, the whole per-step exchange path (the paper's subdomain step
 * between two halo exchanges, Sec. 4.5 and Listing 1): the face halos of u are
 * read from the receive buffers face_in (halo_unpack layouts; NULL array or
 * NULL entry: u's own halo on that face), u_next is updated as by fd_step with
 * the source term of src (may be NULL), and the faces of u_next are written to
 * face_out (halo_pack layouts; NULL array or entry: skipped).  Bitwise the same
 * u_next and faces as halo_unpack(u, face_in) + fd_step_fused.  When nx is a
 * multiple of 64 and all four x-face buffers are given, the x faces are
 * exchanged inside the stencil kernel (their 16-byte row pieces would otherwise
 * cost whole cache lines in a separate pack and unpack); the y and z faces,
 * whole rows and planes, go through the unpack and pack kernels.  On grids of at
 * most 2^21 points with all twelve face buffers given, the whole step is one
 * launch of the one-thread-per-point kernel (see fd_set_tiles).  On return u's
 * face halos are unspecified (they may hold the face_in values).  face_in
 * buffers must not overlap face_out buffers or any volume array (a real
 * exchange double-buffers them: the loopback passes the faces of the previous
 * call's face_out); FD_EINVAL otherwise. */
int fd_step_exchange(const fd_grid* g, const float* u_prev, float* u, float* u_next,
                     const float* vdt2, const fd_sponge* sp, const fd_source* src,
                     const float* const face_in[6], float* const face_out[6],
                     void* stream);

/* S1-S7 for nt steps (the time loop of Sec. 4.5, with the exchange of
 * Listing 1 each step), the host loop in native code: per step n,
 *   (send given) halo_unpack(u, receive = the opposite face of send),
 *   fd_step_fused(u_prev, u -> u_next, source w[n] at src if wavelet non-NULL),
 *   (send given) halo_pack(u_next -> send),
 *   (nrec > 0) record_receivers(u_next -> traces + n*nrec),
 *   rotate (u_prev, u, u_next) <- (u, u_next, u_prev).
 * With send set the exchange is the single-device loopback (periodic
 * subdomain); on entry send must hold the faces of u (zeros for a zero
 * start, or what the previous run left).  With send2 set as well (a second,
 * distinct set of six buffers) each step is one fd_step_exchange reading the
 * loopback of send and writing the faces of u_next to send2, and the two sets
 * swap roles; on return send holds the faces of u (the struct's send and send2
 * pointers are swapped after an odd number of steps).  Same bits either way.
 * On return the struct's three
 * pointers are rotated so u_prev, u hold the last two states.  wavelet is a
 * host array of nt floats, read before the call returns; traces is a device
 * array of nt*nrec floats (may be NULL when nt == 0); rec_off device int64
 * offsets (needed whenever nrec > 0).  With rec_map set, a step without faces
 * over a grid of at most 2^20 points, or one that runs the one-thread-per-point
 * kernel (see fd_set_tiles), takes its receiver row in the stencil launch; with
 * faces the row is taken in the pack launch, otherwise in a launch of its own.
 * Same bits either way. */
typedef struct fd_run {
  float* u_prev;
  float* u;
  float* u_next;
  const float* vdt2;
  fd_sponge sponge;              /* all NULL: no sponge */
  int32_t nt;
  int32_t src[3];
  const float* wavelet;          /* host, nt values; NULL: no source */
  int32_t nrec;
  const int64_t* rec_off;        /* device */
  float* traces;                 /* device, nt*nrec */
  float* send[6];                /* device face buffers, or all NULL (no exchange) */
  float* send2[6];               /* second face set (one-kernel steps), or all NULL */
  const int32_t* rec_map;        /* device, optional: receivers on plane rec_k, map from
                                    fd_receiver_plane_map (entries -1 or < nrec, not
                                    checked on the device); the forward kernel then
                                    writes the trace row itself where it takes no faces */
  int32_t rec_k;
} fd_run;
int fd_forward_run(const fd_grid* g, fd_run* run, void* stream);

/* No passage of the paper defines this call (a launch-cost optimisation of
 * fd_forward_run).  A recorded forward run (HIP graph), for small grids that are modelled again
 * and again (FWI iterations, model scans): one graph launch replaces the
 * per-step launches of fd_forward_run, whose host and dispatch cost is a share
 * of a small grid's step (64^3: 3.37 against 3.61 us per step).  fd_forward_graph checks *run exactly as fd_forward_run does and
 * records, without running anything: zeroing u_prev, u and u_next (whole padded arrays)
 * and, with faces, send[0..5]; then the run->nt steps of fd_forward_run.  The
 * wavelet values and every pointer are fixed at recording; array contents (vdt2,
 * sponge tables, receiver map) are read at each launch, so a new model written
 * into vdt2 is picked up.  On FD_OK, *out holds the graph and *run is rotated as
 * one fd_forward_run would rotate it: after each launch u_prev, u (and, with
 * faces, send) name the arrays that hold the final state.  Each fd_graph_launch
 * enqueues the whole run on `stream` (of the device current at recording) and
 * gives the bits of fd_forward_run from a zero state; launches must not overlap
 * in time with one another or with other work on the same arrays.  FD_EINVAL as
 * fd_forward_run, FD_EDEVICE if recording fails. */
typedef struct fd_graph fd_graph;
int fd_forward_graph(const fd_grid* g, fd_run* run, fd_graph** out);
int fd_graph_launch(fd_graph* graph, void* stream);
/* Frees the graph (NULL: no-op); the caller makes sure no launch is pending. */
int fd_graph_destroy(fd_graph* graph);

/* No passage of the paper defines receivers (see record_receivers).
 * Host helper for fd_run.rec_map: when all nrec >= 1 receivers (rec_ijk: 3*nrec
 * interior (i,j,k) triples) lie on one z plane at distinct (i,j), fills map
 * (host, nx*ny int32) with map[j*nx + i] = r for receiver r and -1 elsewhere,
 * sets *k_out to the plane and returns FD_OK; else FD_EINVAL (the receivers
 * are then sampled by a separate launch). */
int fd_receiver_plane_map(const fd_grid* g, const int32_t* rec_ijk, int32_t nrec,
                          int32_t* map, int32_t* k_out);

/* S5: the paper's application is seismic wave propagation (Sec. 4.5) but it
 * states no source term; this is the reading the library takes:
 * u_next[s] += vdt2[s] * w / (1+eta[s]) at interior point s = (i,j,k). */
int inject_source(const fd_grid* g, float* u_next, const float* vdt2,
                  const fd_sponge* sp, int32_t i, int32_t j, int32_t k, float w,
                  void* stream);

/* S6: no passage of the paper defines receivers (Sec. 4.5 names the
 * application only); the reading here samples the updated field:
 * trace_row[r] = u[rec_off[r]] for r < nrec (rec_off: device int64
 * element offsets, e.g. from fd_receiver_offsets; trace_row: device). */
int record_receivers(const fd_grid* g, const float* u, const int64_t* rec_off,
                     int32_t nrec, float* trace_row, void* stream);

/* S1, the send side of the halo exchange of Listing 1 (Sec. 4.5): the
 * boundary planes a rank puts to its neighbours, here packed into contiguous
 * buffers (the paper's 1-D decomposition puts them in place; six faces serve
 * any decomposition).  Copy the 4 outermost interior planes of u on each face into the six
 * contiguous device buffers face[0..5] = -x,+x,-y,+y,-z,+z (the data a halo
 * exchange sends to the neighbour on that side).  Layouts, x fastest, q = 0..3
 * counting from the lower index:
 *   -x, +x: [nz][ny][4], -x holds i = q, +x holds i = nx-4+q;
 *   -y, +y: [nz][4][nx], -y holds j = q, +y holds j = ny-4+q;
 *   -z, +z: [4][ny][nx], -z holds k = q, +z holds k = nz-4+q.
 * A NULL face is skipped.  Faces need n >= 4 on their axis (else FD_EINVAL). */
int halo_pack(const fd_grid* g, const float* u, float* const face[6], void* stream);

/* S1 + S6 in one launch (Listing 1's send side and the receiver reading of
 * record_receivers): halo_pack(g, u, face) and record_receivers(g, u,
 * rec_off, nrec, trace_row), the faces and the receiver row of the same u (the
 * end of a step: the data the next exchange sends and the trace row n).  Same
 * arguments, layouts and errors as the two calls; nrec == 0 packs only.  Two
 * launches instead of one where the faces cannot take 16-byte accesses. */
int fd_halo_pack_record(const fd_grid* g, const float* u, float* const face[6],
                        const int64_t* rec_off, int32_t nrec, float* trace_row,
                        void* stream);

/* S3, the receive side of Listing 1: after the fence, the planes the
 * neighbours put are in place; here they are copied from contiguous receive
 * buffers into the halo.  Write six receive buffers (same layouts as halo_pack) into the face
 * halos of u: face[0] (-x, from the -x neighbour's +x face) fills
 * i = -4+q, face[1] (+x) fills i = nx+q, and likewise for y and z.  Edges and
 * corners of the halo are never touched.  A NULL face leaves that halo as it
 * is.  Passing {send[1],send[0],send[3],send[2],send[5],send[4]} of a
 * halo_pack of the same u gives periodic boundaries (single-device loopback). */
int halo_unpack(const fd_grid* g, float* u, const float* const face[6], void* stream);

/* ----------------------------------------------------------- adjoint
 * No passage of the paper defines an adjoint or a gradient (it runs the
 * forward kernel only); these calls are the exact transpose of the forward
 * recurrence above, an addition of this library.
 * Transpose of the forward step, for the FWI gradient with respect to
 * squared slowness.  With D = 1/(1+eta), E = 1-eta, Q = vdt2, the forward
 * step is u^{n+1} = D (2u^n - E u^{n-1} + Q (L u^n + f^n)). */

/* S11: a_out = 2 D a_n1 + L(Q D a_n1) - E D a_nn on the interior, where the
 * halo of Q D a_n1 is taken from a_n1's halo (as given: zero for Dirichlet),
 * vdt2's halo (as fd_prepare_vdt2 writes it) and eta at the periodic image.
 * a_nn may be NULL (treated as zero).  a_out may alias a_nn, never a_n1.
 * If g_vdt2 is non-NULL, also g_vdt2 += D a_n1 (L u_n + f) with u_n's halo as
 * given and f = src->w at src (src may be NULL: no source term); u_n must
 * then be non-NULL. */
int fd_adjoint_step(const fd_grid* g, const float* a_nn, const float* a_n1,
                    float* a_out, const float* vdt2, const fd_sponge* sp,
                    const float* u_n, float* g_vdt2, const fd_source* src,
                    void* stream);

/* a[off[r]] += vals[r] for r < n (device arrays; duplicate offsets add). */
int fd_scatter_add(const fd_grid* g, float* a, const int64_t* off, const float* vals,
                   int32_t n, void* stream);

/* grad_m = -g_vdt2 * vdt2^2 / dt^2 on the interior (m = 1/v^2, dt fixed);
 * grad_m may alias g_vdt2 (in place), not vdt2. */
int fd_grad_finalize(const fd_grid* g, const float* g_vdt2, const float* vdt2,
                     double dt, float* grad_m, void* stream);

/* The same adjoint in the scaled variable b = Q D a.  Multiplying the
 * fd_adjoint_step recurrence by Q D gives
 *   b^n = D (2 b^{n+1} - E b^{n+2} + Q L b^{n+1}),
 * the forward update run backward in time (L is symmetric, Q, D, E are
 * diagonal), so the adjoint sweep runs the forward stencil kernel.  Since Q and
 * D do not depend on n, g_vdt2 = g_b / Q with g_b = sum_n b^{n+1} (L u^n + f^n),
 * and the derivative of the loss with respect to the source amplitude w[n] is
 * b^{n+1} at the source point.
 *
 * S11 (scaled): b_out = D (2 b_n1 - E b_nn + Q L b_n1) on the interior, with
 * b_n1's halo as given (zero for Dirichlet halos).  b_nn and b_n1 must be
 * non-NULL; b_out may alias b_nn, never b_n1.  If g_b is non-NULL, also
 * g_b += b_n1 (L u_n + f) with u_n's halo as given and f = src->w at src (src
 * may be NULL); u_n must then be non-NULL.  Same error behaviour as
 * fd_adjoint_step. */
int fd_adjoint_step_scaled(const fd_grid* g, const float* b_nn, const float* b_n1,
                           float* b_out, const float* vdt2, const fd_sponge* sp,
                           const float* u_n, float* g_b, const fd_source* src,
                           void* stream);

/* fd_adjoint_step_scaled followed by fd_scatter_add_scaled(b_out, res_row) of
 * receivers that all lie on plane res_k (res_map: device nx*ny map from
 * fd_receiver_plane_map, each entry -1 or an index into res_row), the residual added in the update's own launch; same
 * bits as the two calls.  FD_EINVAL for a NULL map or row or a plane outside
 * the interior, else as fd_adjoint_step_scaled. */
int fd_adjoint_step_scaled_res(const fd_grid* g, const float* b_nn, const float* b_n1,
                               float* b_out, const float* vdt2, const fd_sponge* sp,
                               const float* u_n, float* g_b, const fd_source* src,
                               const int32_t* res_map, int32_t res_k, const float* res_row,
                               void* stream);

/* The adjoint source in the scaled variable: b[off[r]] += vals[r] Q / (1+eta)
 * at each offset (device arrays; offsets must be interior points of g, an
 * offset outside the interior is taken with eta = 0; duplicates add). */
int fd_scatter_add_scaled(const fd_grid* g, float* b, const int64_t* off,
                          const float* vals, const float* vdt2, const fd_sponge* sp,
                          int32_t n, void* stream);

/* grad_m = -g_b * vdt2 / dt^2 on the interior, for the g_b accumulated by
 * fd_adjoint_step_scaled (grad_m may alias g_b, not vdt2). */
int fd_grad_finalize_scaled(const fd_grid* g, const float* g_b, const float* vdt2,
                            double dt, float* grad_m, void* stream);

/* ------------------------------------------------------- shot serving
 * No passage of the paper defines shot serving.  The server is this library's
 * one-device analogue of two runtime mechanisms of the paper: device memory
 * taken from one runtime-owned segment by a heap allocator (Sec. 3.1, the
 * global segment with a linear-heap or buddy allocator) and a bounded number
 * of concurrently active units of work (Sec. 3.2, MAX_ACTIVE_STREAMS).
 * S8/S9: a server that runs many independent forward-modelling shots of
 * different grid sizes at once.  In submission order (strict FIFO), a shot's
 * footprint is carved from the caller's device arena as soon as it fits (at most
 * four shots ahead of those running) and its admission work -- zeroing, the
 * max(v) reduction and stability check, vdt2, sponge and receiver tables -- runs
 * asynchronously on a stream of a bounded pool (at most four streams, created
 * when first needed, reused when idle, half of the finished ones synchronised and
 * released when the bound is reached), overlapping the steps of running shots.
 * A shot joins the batched step when a slot is free and the activation policy
 * lets it (fd_server_set_admission), as soon as its admission work is enqueued:
 * the compute stream waits for that work, not the host.  Where the sponge's design
 * velocity is known without max(v) (sponge_vmax given, or no sponge), all of it is
 * enqueued at once and the stability check follows when max(v) reaches the host:
 * a shot found unstable then leaves the step and ends with FD_EINVAL.  Every active shot
 * advances one time step per batched step (one launch per kernel family over the
 * tiles of its grids, each shot at its own step, then one batched receiver
 * launch), so shots that arrive while others run share the device.  Finished
 * shots' traces are copied to pinned host memory on a copy stream and their arena
 * block is freed.  Each shot is the forward model of fd_step_fused with Dirichlet
 * halos, a quadratic sponge of `sponge_width` cells (reflection 1e-3) and a
 * Ricker source; its traces are bitwise those of the same shot run alone
 * through fd_step_fused + record_receivers with the same dt and sponge. */

typedef struct fd_shot_desc {
  int32_t nx, ny, nz;        /* interior extent, each >= 1                       */
  int32_t nt;                /* time steps, >= 1                                  */
  double dx, dy, dz;         /* spacing, > 0                                       */
  double dt;                 /* time step; the shot ends with FD_EINVAL at admission
                                if max(v) dt sqrt(s_pi sum_a 1/d_a^2) > 2, the
                                leapfrog stability limit of this stencil (s_pi =
                                6.5016 is its 1-D symbol at the Nyquist wavenumber;
                                Courant 0.45286 on a cube)                     */
  double f0, t0;             /* Ricker peak frequency and delay                   */
  int32_t src[3];            /* source point, inside the interior                 */
  int32_t sponge_width;      /* damping cells per face (0: none)                  */
  double sponge_vmax;        /* velocity the sponge is designed for; <= 0: the
                                shot's own max(v)                                  */
  const float* v_dev;        /* caller-owned device velocity view: point (i,j,k)
                                at v_dev[k*v_zstride + j*v_ystride + i]; fully
                                written before shot_submit (the server reads it
                                on a stream of its own) and unchanged until the
                                shot is done                                       */
  int64_t v_ystride, v_zstride;
  int32_t nrec;              /* receivers, >= 0                                    */
  const int32_t* rec_ijk_host; /* 3*nrec (i,j,k) triples, copied at submit        */
} fd_shot_desc;

/* Arena bytes one shot occupies while active (4 padded volumes, sponge
 * tables, receiver offsets, traces, and with receivers an nx*ny receiver-plane
 * map, used when they share one z plane); -1 for an invalid descriptor. */
int64_t fd_shot_footprint(const fd_shot_desc* d);

/* Create a server over the caller-owned device arena [arena_dev,
 * arena_dev + arena_bytes) (256-byte aligned; about 1.1 MB of it holds the
 * server's tables), running at most max_slots (1..64) shots at once.
 * compute_stream / copy_stream are hipStream_t (NULL: the server creates
 * its own); the server also creates one stream of its own for admission work
 * (zeroing, model preparation, sponge and receiver uploads), so admitting a shot never waits
 * for the steps queued on the compute stream.  The arena must outlive the
 * server.  Starts the progress thread. */
int fd_server_create(void** srv, void* arena_dev, size_t arena_bytes, int32_t max_slots,
                     void* compute_stream, void* copy_stream);
/* Queue a shot.  FD_EINVAL for a bad descriptor (sizes, source or receiver
 * outside the interior, NULL velocity), FD_ENOMEM if its footprint can never
 * fit the arena, FD_ECANCELED after shutdown.  Thread-safe. */
int shot_submit(void* srv, const fd_shot_desc* d, int64_t* shot_id);
/* FD_EAGAIN while queued or running.  When finished: copies min(cap,
 * nt*nrec) floats of traces ([nt][nrec], u^{n+1} at receiver r after step n)
 * into traces_host (may be NULL), fills t_ns (may be NULL) with the
 * submit, admit and done times (steady clock, ns; done = when the server saw
 * the traces land in host memory), forgets the shot and returns its final
 * code: FD_OK, FD_EINVAL (rejected at admission, e.g. unstable dt),
 * FD_EDEVICE or FD_ECANCELED.  FD_ENOTFOUND for an unknown or already
 * collected id.  Thread-safe. */
int shot_poll(void* srv, int64_t shot_id, float* traces_host, size_t cap, int64_t t_ns[3]);
/* Activation policy: which prepared shot joins the batched step.  Shots join in
 * submission order (the next one waits for those before it), only with a free slot
 * and tile-table room.  Shots of one batched step advance in lockstep, so joining a
 * running shot trades its latency for throughput.  With max_active_points = 0 (the
 * default) a shot joins if the interior points of the running shots and its own stay
 * within the fill, 256 x 128 x 32 x 8 = 8,388,608 (each of the 256 CUs one 128 x 32
 * tile of 8 z planes: grids that together leave the device short of work), or, while
 * more shots wait behind it (a backlog), within twice that (one launch of two
 * mid-size grids beats two launches); with max_active_points > 0 if they
 * stay within that many.  A shot always joins when none runs.  FD_EINVAL for a NULL
 * server or a negative limit.  Thread-safe. */
int fd_server_set_admission(void* srv, int64_t max_active_points);
/* Allocator of the shots' blocks in the arena (the paper's global segment carved by
 * a linear-heap or a buddy allocator, Sec. 3.1): FD_ARENA_FIRST_FIT (the default:
 * lowest hole that fits, neighbours merged on release) or FD_ARENA_BUDDY (binary
 * buddy blocks of a power of two times 256 bytes; a shot then takes its footprint
 * rounded up to such a block).  Only before the first shot_submit (FD_EINVAL
 * after, or for another kind).  Thread-safe. */
enum { FD_ARENA_FIRST_FIT = 0, FD_ARENA_BUDDY = 1 };
int fd_server_set_allocator(void* srv, int32_t kind);
/* Counts of waiting (queued or being prepared), running (in the batched step or
 * copying out), finished-but-uncollected shots, and batched steps launched so far
 * (4 int64).  Thread-safe. */
int fd_server_stats(void* srv, int64_t out[4]);
/* Stop the progress thread: queued and running shots finish as
 * FD_ECANCELED; finished shots stay collectable by shot_poll; later submits
 * fail with FD_ECANCELED.  Idempotent. */
int fd_server_shutdown(void* srv);
/* Shut down (as above) and free the server; its shot ids become invalid. */
int fd_server_destroy(void* srv);

/* ------------------------------------------------------------------------
 * Cannon's matrix multiply: the local block product (Sec. 4.4).  Each of P ranks
 * holds row stripes of Ns = N/P rows and at each of its P steps adds the product
 * of an Ns x Ns block of its A stripe and the B stripe it holds (N * Ns * Ns
 * multiply-adds) to its C stripe.  This is that step on one device:
 *     C = (accumulate ? C : 0) + A B,
 * A m x k, B k x n, C m x n, FP64, row-major device arrays with leading dimensions
 * lda >= k, ldb >= n, ldc >= n (elements between consecutive rows), on the FP64
 * matrix cores.  The ring shift of the B stripes between ranks is not part of it.
 * Each element is a sum of the same products as the definition, in another order
 * (within the FP64 error bound of the definition; exact where every partial sum is
 * exactly representable, e.g. small integers).  m == 0 or n == 0: nothing happens;
 * k == 0: C becomes C (accumulate) or 0.  FD_EINVAL for a negative extent, a NULL
 * array that is needed, a leading dimension too small, or C overlapping A or B.
 * Asynchronous on `stream`; the arrays stay the caller's. */
int fd_block_gemm_f64(int64_t m, int64_t n, int64_t k, const double* a, int64_t lda,
                      const double* b, int64_t ldb, double* c, int64_t ldc, int32_t accumulate,
                      void* stream);

#ifdef __cplusplus
}
#endif

#endif /* FD_H */
