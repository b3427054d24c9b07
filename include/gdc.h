/*
 * gdc.h -- C ABI of the MI355X (gfx950) library for the generalised
 * drift-correcting (gDC) Brownian-dynamics step of rigid multiblob particles
 * with fluctuating force-coupling (FCM) hydrodynamics in a periodic box.
 *
 * Method: Westwood, Delmotte & Keaveny, "A generalised drift-correcting time
 * integration scheme for Brownian suspensions of rigid particles with
 * arbitrary shape", arXiv 2106.00449.  Paper sections are cited per entry.
 *
 * Conventions common to every entry point
 *   - Arrays are row-major FP64 at the boundary in both precision modes.
 *     Y: N x 3 body reference points (unwrapped, box coordinates);
 *     q: N x 4 unit quaternions, scalar first, Hamilton product (Appendix A);
 *     blob vectors (lambda, v): M x 3 with the blobs of body 0 first, then
 *     body 1, ..., each body's blobs in its shape's order;
 *     body vectors (F, V): N x 6 = (force or velocity, torque or angular
 *     velocity), lab frame.
 *     Grid fields: 3 x n0 x n1 x n2 (component, then axis 0, 1, 2 of the box;
 *     axis 2 fastest); grid point g sits at (g0 dx0, g1 dx1, g2 dx2).
 *   - memspace = GDC_HOST: the pointers are host memory, the library copies
 *     in and out and synchronises its stream before returning.
 *     memspace = GDC_DEVICE: the pointers are device memory on the handle's
 *     device, read and written in stream order on the handle's stream; the
 *     call still synchronises where it must read a scalar back (GMRES
 *     convergence) and before returning.
 *   - The caller owns every array passed in or out.  The library owns all
 *     state inside a handle until gdc_free.  A handle is used by one thread
 *     at a time; distinct handles are independent.
 *   - Return value: GDC_OK (0) or a negative error code; nothing aborts or
 *     throws across the ABI.  gdc_last_error() gives a message for the most
 *     recent failure on the calling thread.
 *   - Units are the caller's; with a = 1, eta = 1/(6 pi) and kT = 1 the
 *     one-blob mobility and the diffusive time a^2/D are 1 (Sec. 6.2).
 */
#ifndef GDC_H
#define GDC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  GDC_OK = 0,
  GDC_EINVAL = -1,    /* bad argument: sizes, non-unit quaternion, grid size */
  GDC_ENOMEM = -2,    /* device or host allocation failed */
  GDC_ENOTCONV = -3,  /* GMRES hit its iteration limit; outputs still written */
  GDC_ENUMERIC = -4,  /* NaN or Inf in a result */
  GDC_EDEVICE = -5    /* a HIP runtime error */
};

enum { GDC_FP32 = 0, GDC_FP64 = 1 };          /* grid precision */
enum { GDC_HOST = 0, GDC_DEVICE = 1 };        /* memspace */
enum { GDC_BLOB = 0, GDC_BODY = 1 };          /* gdc_mobility_apply mode */
enum { GDC_SCHEME_GDC = 0, GDC_SCHEME_EM = 1 };
enum { GDC_DIV_FD = 0, GDC_DIV_RFD = 1 };
enum { GDC_UNTIL_ALL = 0, GDC_UNTIL_ANY = 1 };  /* gdc_batch_step return condition */

/* A rigid body shape: n_blobs body-frame blob offsets b_i (n_blobs x 3);
 * a body with reference point Y and orientation q has blobs at
 * r_i = Y + R(q) b_i (Sec. 2, eq. quaternion_rotation_matrix). */
typedef struct {
  int n_blobs;
  const double* b;
} gdc_shape;

/* Forces applied at the midpoint of each step (Sec. 3, step 5).
 *   steric_k, steric_cutoff: harmonic repulsion V(r) = k/2 (r - cutoff)^2 for
 *     r < cutoff between blobs of different bodies (the harmonic potential of
 *     Sec. 6.3 applied to blob pairs); 0 disables it.
 *   const_force: force and torque added to every body.
 *   shear_rate: background flow u(r) = rate (y - L1/2) e_x at each blob, y
 *     measured from the body's wrapped reference point (not Lees-Edwards).
 *   sine_force: f0 of the periodic force density f0 sin(k y) e_x on the
 *     fluid, k = 2 pi / L1 (the rheology forcing of Sec. 6.4); its flow
 *     f0/(eta k^2) sin(k y) e_x, averaged at each blob, enters the step-5
 *     slip, and each step reports the sine amplitude v_x of the fluid's
 *     x-velocity (gdc_stats.sine_vx), so that eta_eff = f0 / (k^2 v_x).
 *   wall_k, wall_cutoff: in the slip channel (gdc_config.channel), the
 *     harmonic blob-wall repulsion V(h) = k/2 (h - cutoff)^2 for h < cutoff,
 *     h the blob's distance from the wall y = 0 or y = L1/2 (Sec. 6.3:
 *     cutoff 2.2a, k = 40 kT/(a cutoff)); 0 disables it. */
typedef struct {
  double steric_k;
  double steric_cutoff;
  double const_force[6];
  double shear_rate;
  double sine_force;
  double wall_k;
  double wall_cutoff;
} gdc_forces;

/* Suspension and solver parameters (Sec. 2-4, Sec. 6.1).
 *   L[3], n[3]: periodic box and grid; each n_d even, of the form 2^a 3^b,
 *     8 <= n_d <= 384 (8, 12, 16, 24, 32, 48, 64, 96,
 *     128, 192, 256, 384).
 *   a: blob radius; sigma: Gaussian envelope width (0 -> a/sqrt(pi), Sec. 4.2);
 *   trunc: envelope cutoff radius (0 -> 3a, Sec. 6.1), below min(L)/2.
 *   eta, kT, dt: viscosity, thermal energy, time step.
 *   fd_delta: finite-difference parameter of step 3 (0 -> 1e-6, Sec. 6.2).
 *   gmres_tol: relative residual of the step-5 saddle solve (0 -> 1e-6);
 *   gmres_maxit (0 -> 200), gmres_restart (0 -> 50).
 *   precision: GDC_FP32 (grid in FP32, bodies and Krylov in FP64) or GDC_FP64.
 *   scheme: GDC_SCHEME_GDC (Sec. 3) or GDC_SCHEME_EM (Appendix D).
 *   divergence: GDC_DIV_FD (eq. FD) or GDC_DIV_RFD (eq. rfd_div).
 *   channel: 0 for the periodic box; 1 for the slip channel of Sec. 6.3:
 *     free-slip walls at y = 0 and y = L1/2 (u_y = 0, no tangential stress),
 *     the box of height L1 being twice the channel, kept by an image system:
 *     every blob force has its mirror image R lambda at (x, L1 - y, z),
 *     R = diag(1, -1, 1), and the stress noise is mirrored the same way.
 *     Bodies belong in 0 < y < L1/2; no shear or sine forcing there.
 *   seed: Philox4x32-10 key of every random number of the run.
 *   shapes[n_shapes]; body_shape[n_bodies]: shape index of each body.
 *   device: HIP device ordinal; stream: a hipStream_t or NULL (the library
 *     then creates its own stream at default priority). */
typedef struct {
  double L[3];
  int n[3];
  double a, sigma, trunc, eta, kT, dt, fd_delta;
  double gmres_tol;
  int gmres_maxit, gmres_restart;
  int precision, scheme, divergence, channel;
  uint64_t seed;
  int n_shapes;
  const gdc_shape* shapes;
  int n_bodies;
  const int* body_shape;
  gdc_forces forces;
  int device;
  void* stream;
} gdc_config;

/* Per-call statistics of gdc_step and gdc_batch_step: values of the last
 * step completed in the call, and means over the steps completed in it. */
typedef struct {
  int steps_done;            /* steps completed in this call */
  int gmres_iterations;      /* preconditioned GMRES iterations, last step */
  double gmres_relres;       /* final relative residual, last step */
  double nu;                 /* drift factor nu of the last step (Sec. 3, step 3) */
  int nu_nonpositive;        /* steps of this call whose nu was <= 0 */
  double ms;                 /* gdc_step: wall time of the call; gdc_batch_step:
                                time from the call's start to this handle's
                                last completed step (0 if none) */
  double sine_vx;            /* with sine forcing: mean over the call's steps of
                                the sin(k y) amplitude of the fluid x-velocity,
                                (f0 + (2/V) sum_i lambda_ix J[sin(k y)](r_i)) /
                                (eta k^2) at the midpoint solve; else 0 */
  double gmres_iterations_mean; /* mean GMRES iterations over the call's steps */
  double nu_mean;            /* mean nu over the call's steps (1 for EM) */
  double nu_std;             /* standard deviation of nu over the call's steps */
  double nu_min, nu_max;     /* extremes of nu over the call's steps */
  int status;                /* this handle's own outcome of the steps completed
                                in the call: GDC_OK, GDC_ENOTCONV (a solve missed
                                the tolerance) or GDC_ENUMERIC (non-finite state,
                                pair-force cell overflow) */
  int fused_iterations;      /* GMRES iterations of this handle launched fused
                                with other suspensions' in the call
                                (gdc_batch_step, gdc_set_fusion) */
} gdc_stats;

typedef struct gdc_handle gdc_handle;

/* Validate cfg, copy what the library needs (shapes are copied), allocate
 * the device arena and build the per-shape tables (pseudo-inverse of K^T K,
 * null-space projector, preconditioner inverse).  *out receives the handle.
 * Errors: GDC_EINVAL (bad sizes or parameters), GDC_ENOMEM, GDC_EDEVICE. */
int gdc_init(const gdc_config* cfg, gdc_handle** out);

/* Release everything the handle owns.  NULL is accepted. */
void gdc_free(gdc_handle* h);

/* Message of the last failed call on this thread ("" if none). */
const char* gdc_last_error(void);

/* Apply the deterministic mobility at configuration (Y, q) (Sec. 2.2, 4.2).
 *   mode GDC_BLOB: in = lambda (M x 3) -> out = M_FCM lambda (M x 3),
 *     M_FCM = J L^-1 S: Gaussian spreading, spectral Stokes solve with the
 *     k = 0 and Nyquist modes removed, trapezoidal averaging.
 *   mode GDC_BODY: in = F (N x 6) -> out = V = N F (N x 6), the solution of
 *     the saddle problem [[M, -K], [-K^T, 0]] [lambda; V] = [0; -F] (eq.
 *     saddle_point_sys) by right-preconditioned GMRES to gmres_tol with the
 *     block-diagonal preconditioner of Sec. 2.2.  Degrees of freedom that move
 *     no blob (spin of a straight rod, rotation of a one-blob body) are held
 *     at zero and the matching torque component is ignored.
 * No noise.  Errors: GDC_EINVAL, GDC_ENOTCONV (out still written),
 * GDC_ENUMERIC, GDC_EDEVICE. */
int gdc_mobility_apply(gdc_handle* h, int mode, const double* Y, const double* q,
                       const double* in, double* out, int memspace);

/* Advance (Y, q) in place by n_steps steps of the configured scheme (Sec. 3:
 * noise, least-squares velocity, finite-difference or RFD divergence, midpoint,
 * full saddle solve with the same noise, update; or Appendix D).  The noise of
 * internal step s uses Philox counters keyed by (seed, s); the internal step
 * counter starts at 0 and advances by one per step.  st may be NULL.
 * Errors: GDC_EINVAL, GDC_ENOTCONV (the step is still taken), GDC_ENUMERIC,
 * GDC_EDEVICE. */
int gdc_step(gdc_handle* h, int n_steps, double* Y, double* q, int memspace, gdc_stats* st);

/* Resident state for gdc_batch_step (Sec. 3: the state of a suspension is
 * (Y, q)).  gdc_set_state copies Y (N x 3) and q (N x 4, unit norm within
 * 1e-6, host arrays checked) into the handle; gdc_get_state copies the
 * current state out.  gdc_step also leaves its result resident.  Both wait
 * for the handle's stream.  Errors: GDC_EINVAL (no state yet, a step in
 * flight, bad quaternion), GDC_EDEVICE. */
int gdc_set_state(gdc_handle* h, const double* Y, const double* q, int memspace);
int gdc_get_state(gdc_handle* h, double* Y, double* q, int memspace);

/* Advance several independent resident suspensions together (the steps of
 * Sec. 3 for each).  One host thread keeps every handle's step in flight:
 * each handle's kernels go to its own stream, so the work of different
 * suspensions overlaps on the device, and each handle's GMRES status is
 * polled without blocking the others.  The result of each handle is the
 * same as gdc_step on it alone (same kernels, same order, same noise).
 *   hs[nh]: distinct handles holding a state (gdc_set_state / gdc_step),
 *     each on its own stream (handles sharing a stream are serialised, still
 *     correct).
 *   steps[nh] (in/out): steps still to take per handle; each completed step
 *     decrements it.
 *   until: GDC_UNTIL_ALL returns when every entry of steps is 0;
 *     GDC_UNTIL_ANY as soon as one handle that had steps left at entry has
 *     none.  A handle whose state turns non-finite (or whose pair-force cell
 *     list overflows) is not advanced further in the call and counts as
 *     done for both conditions; its status is GDC_ENUMERIC.  max_ms > 0 also returns once that much wall time has passed
 *     (0: no limit).  A handle left in the middle of a step keeps its place:
 *     its queued kernels continue on the device, and the next
 *     gdc_batch_step call resumes it; every other call on that handle except
 *     gdc_free returns GDC_EINVAL until the step is finished.
 *   st[nh] (optional): per-handle statistics of this call; st[i].status is
 *     handle i's own outcome, so a failed solve is attributed to the
 *     suspension that produced it.  Each call counts only the steps it
 *     completes.
 * Errors: GDC_EINVAL; GDC_ENOTCONV / GDC_ENUMERIC (as gdc_step, for the
 * first handle that hit one; the steps are still taken; st[i].status names
 * every handle's); GDC_EDEVICE. */
int gdc_batch_step(gdc_handle* const* hs, int nh, int* steps, int until, double max_ms, gdc_stats* st);

/* Completion times of the handle's steps, in milliseconds of the host's
 * monotonic clock (CLOCK_MONOTONIC), oldest first: the time of the last
 * gdc_set_state, then one entry per completed step.  Copies up to cap
 * entries into t_ms, sets *count, and drops them from the handle's log
 * except the newest, from which the next step's latency is measured. */
int gdc_step_log(gdc_handle* h, double* t_ms, int cap, int* count);

/* Device memory a handle for cfg would hold, in bytes, without allocating
 * or touching a device (admission control by HBM footprint).  gdc_device_bytes
 * gives the same figure for an existing handle.  Errors: as gdc_init's
 * validation. */
int gdc_footprint(const gdc_config* cfg, size_t* bytes);
int gdc_device_bytes(const gdc_handle* h, size_t* bytes);

/* Workgroup sizes (threads) of the FFT passes of the handle's grid, in the
 * order: three-pass path (plane forward, projection, plane inverse), then
 * five-pass path (R2C, axis-1 forward, projection, axis-1 inverse, C2R):
 * GDC_FFT_PASSES values.  gdc_init times every size of every pass on the
 * handle's grid and keeps the fastest (cached per grid and precision for the
 * process); gdc_set_launch_config overrides them (plane passes: 256, 512 or
 * 1024; others: 256 or 512).  Every size gives the same results bit for bit.
 * Errors: GDC_EINVAL (NULL, n < GDC_FFT_PASSES, a size not allowed). */
enum { GDC_FFT_PASSES = 8 };
int gdc_get_launch_config(const gdc_handle* h, int* threads, int n);
int gdc_set_launch_config(gdc_handle* h, const int* threads, int n);

/* Launch mode of a step (Sec. 3): with graphs on (the default) the step's
 * set-up (steps 1-5 and the first GMRES cycle's start), each Krylov
 * column's iteration of the step-5 solve, and the step's end (update and
 * readback) are captured once into HIP graphs and replayed, a few launches
 * per step instead of about a hundred; the set-up graph reads the step
 * counter from device memory, which the library keeps equal to the
 * handle's.  Off, every kernel is launched on its own.  Results are the same
 * bit for bit.  While gdc_probe_kernel watches a family, kernels launch on
 * their own so the probe can stamp them; gdc_set_launch_config drops the
 * captured graphs.  Errors: GDC_EINVAL (NULL, step in flight). */
int gdc_set_graphs(gdc_handle* h, int on);
int gdc_get_graphs(const gdc_handle* h, int* on);

/* Fused batching (the GMRES iterations of Sec. 3 step 5 over several
 * suspensions): with fusion on, a handle stepped by gdc_batch_step does not
 * launch its GMRES iterations itself.  After each pass over its handles the
 * call launches every kernel of an iteration (preconditioner, spreading
 * once per table width, the three plane passes of the transform,
 * averaging, the three Arnoldi kernels) once for all the fused handles that
 * have an iteration ready, each at its own Krylov column, grouped by what
 * the kernels are instantiated for (grid size, transform workgroup sizes,
 * vector-length class); each group launches on a library stream of its own
 * (up to four per GPU), and waits while two of its fused iterations are
 * still in flight.  The handle's stream and the group's are joined only
 * where work crosses them, and the handle's stream follows all of its work
 * when the call returns.  Each suspension's arithmetic is unchanged:
 * results equal the unfused ones bit for bit.  Only handles on the FP32
 * plane-path transforms (grids up to 128^3) with the matrix-core
 * preconditioner, outside the slip channel, are fused; others run as
 * before, and so does gdc_step.  Off by default.  Errors: GDC_EINVAL (NULL,
 * step in flight). */
int gdc_set_fusion(gdc_handle* h, int on);
int gdc_get_fusion(const gdc_handle* h, int* on);

/* Internal step counter (checkpoint / resume: with the same state and
 * counter a resumed run repeats an uninterrupted one exactly). */
int gdc_get_step(const gdc_handle* h, uint64_t* step);
int gdc_set_step(gdc_handle* h, uint64_t step);

/* The random velocity field u_brev = L^-1 D W of step `step` (Sec. 4.2, 5):
 * 3 x n0 x n1 x n2, FP64 (rounded from FP32 in FP32 mode).  The stress
 * spectrum is drawn in Fourier space: per stored half-spectrum mode 12
 * normals (Re, Im of W_xx, W_yy, W_zz, W_xy, W_xz, W_yz), scaled to the law of
 * the real-space construction of Sec. 6.1. */
int gdc_fluct_velocity(gdc_handle* h, uint64_t step, double* u, int memspace);

/* Steps 1-3 of Sec. 3 at (Y, q) for step `step`: calV (N x 6), the
 * least-squares rigid velocity of the averaged random velocities (eq.
 * sol_unconst), and d (N), each body's term of the divergence, so that
 * nu = 1 + dt/2 sum_p d_p (eq. FD, or eq. rfd_div in RFD mode). */
int gdc_predictor(gdc_handle* h, const double* Y, const double* q, uint64_t step,
                  double* calV, double* d, int memspace);

/* The library's normal generator, for checking the noise contract: for
 * c0 in [c0_begin, c0_begin + count), Philox4x32-10 with key = seed and
 * counter (c0, c1, step lo, step hi), each word pair turned into two normals
 * by Box-Muller; out (host, count x 4). */
int gdc_philox_normals(gdc_handle* h, uint64_t seed, uint32_t c1, uint64_t step,
                       uint32_t c0_begin, int count, double* out);

/* gdc_philox_normals without any device allocation, for callers that
 * cannot allocate (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the same normals, bit for bit, staged
 * through a fixed device array that the library holds per GPU until the
 * process ends (2 MiB: count <= 65536 groups of four normals; larger
 * counts return GDC_EINVAL).  Every call on one GPU shares that array, so
 * calls that overlap on one GPU (from several threads or handles) race;
 * the call waits for its copy before returning.  out: host, count x 4. */
int gdc_philox_normals_noalloc(gdc_handle* h, uint64_t seed, uint32_t c1, uint64_t step, uint32_t c0_begin,
                               int count, double* out);

/* Measurement helpers (process-wide, not tied to a handle).
 * gdc_probe_kernel(family): from now on, every launch of the named kernel
 * family carries a start and a stop HIP event that the dispatch itself
 * stamps (hipExtLaunchKernel on the stream it is launched on), so the
 * elapsed time is the kernel's own duration ("spread", "interp", "fft_r2c",
 * "fft_fwd1", "fft_project", "fft_inv1", "fft_c2r", "fft_plane_fwd",
 * "fft_plane_inv", "fft_noise"; NULL or "" switches probing off; at most
 * 8192 launches are kept).  gdc_probe_read: total elapsed milliseconds and number
 * of probed launches since the last read (waits for the last stop event),
 * and, when each_ms is not NULL, the duration of each launch in launch
 * order (host array; the first `capacity` are written), then clears the
 * record.  Launches of a GMRES iteration queued ahead of the convergence
 * test return at the solver's done flag and take microseconds: the
 * per-launch durations let a caller tell them from launches that did the
 * work. */
int gdc_probe_kernel(const char* family);
int gdc_probe_read(double* total_ms, long long* launches, float* each_ms, long long capacity);

#ifdef __cplusplus
}
#endif

#endif /* GDC_H */
