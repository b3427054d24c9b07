// Internal declarations shared by the translation units of libgdc.
// Device helpers here are header-inline; each .hip file owns its kernels and
// exposes host launchers declared below.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/gdc.h"

namespace gdc {

// ------------------------------------------------------------ error plumbing

void set_error(const std::string& msg);

struct Status {
  int code = GDC_OK;
  explicit operator bool() const { return code == GDC_OK; }
};

#define GDC_HIP(call)                                                           \
  do {                                                                          \
    hipError_t e_ = (call);                                                     \
    if (e_ != hipSuccess) {                                                     \
      ::gdc::set_error(std::string(#call) + ": " + hipGetErrorString(e_));       \
      return GDC_EDEVICE;                                                       \
    }                                                                           \
  } while (0)

#define GDC_TRY(expr)          \
  do {                         \
    int rc_ = (expr);          \
    if (rc_ != GDC_OK) return rc_; \
  } while (0)

// Checks the launch of the kernel just issued.
int check_launch(const char* what);

// Optional timing of one kernel family with HIP events on the stream it is
// launched on (enabled by gdc_probe_kernel).  Start and stop events for the next launch of `family` when
// gdc_probe_kernel watches it, else nulls: the launch passes them to
// hipExtLaunchKernelGGL, which stamps them from the dispatch itself, so a
// probed launch runs exactly as an unprobed one.
struct ProbeEvents {
  hipEvent_t start = nullptr, stop = nullptr;
};
ProbeEvents probe_claim(const char* family);
// Whether a kernel family is being probed (launches then stay out of graphs).
bool probe_active();

// A launch that carries the probe's events when a probe claimed it (the
// dispatch stamps them: hipExtLaunchKernelGGL), a plain launch otherwise, so
// that unprobed launches can be captured into a HIP graph.
#define GDC_LAUNCH_PROBED(kernel, grid, block, shm, stream, pe, ...)                                 \
  do {                                                                                                \
    if ((pe).start)                                                                                   \
      hipExtLaunchKernelGGL(kernel, grid, block, shm, stream, (pe).start, (pe).stop, 0, __VA_ARGS__); \
    else                                                                                              \
      hipLaunchKernelGGL(kernel, grid, block, shm, stream, __VA_ARGS__);                              \
  } while (0)

// ------------------------------------------------------------ block coordinates
// A kernel body takes its block coordinates as a BlockIx: from the hardware
// in an ordinary launch, or, in a launch fused over several suspensions,
// from the flat block index through the table of each suspension's first
// block.  A block's arithmetic does not depend on which.
struct BlockIx {
  int x, y, z;
  int gx, gy, gz;
};
__device__ __forceinline__ BlockIx hw_block() {
  return BlockIx{(int)blockIdx.x, (int)blockIdx.y, (int)blockIdx.z,
                 (int)gridDim.x,  (int)gridDim.y,  (int)gridDim.z};
}

// One suspension's grid in a fused launch.
struct LocalGrid {
  int gx, gy, gz;
};

// Suspension of flat block b: first[s] is suspension s's first block (first
// is nondecreasing, first[0] = 0, ns entries).
__device__ __forceinline__ int fused_suspension(const int* __restrict__ first, int ns, int b) {
  int lo = 0, hi = ns - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (first[mid] <= b) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ BlockIx fused_block(const LocalGrid& g, int local) {
  const int x = local % g.gx, yz = local / g.gx;
  return BlockIx{x, yz % g.gy, yz / g.gy, g.gx, g.gy, g.gz};
}

// ------------------------------------------------------------ complex values

template <typename R>
struct alignas(2 * sizeof(R)) Cx {
  R x, y;
};

// Explicit fused multiply-adds, so that the product rounds the same way in
// every kernel instantiation (the transform file turns automatic contraction
// off).
__host__ __device__ inline float fused_ma(float a, float b, float c) { return fmaf(a, b, c); }
__host__ __device__ inline double fused_ma(double a, double b, double c) { return fma(a, b, c); }

template <typename R>
__host__ __device__ inline Cx<R> cmul(Cx<R> a, Cx<R> b) {
  return Cx<R>{fused_ma(a.x, b.x, -(a.y * b.y)), fused_ma(a.x, b.y, a.y * b.x)};
}

// ------------------------------------------------------------ rigid-body algebra
// Scalar-first unit quaternions and the Hamilton product (Appendix A).

// R(q), row-major, eq. (quaternion_rotation_matrix).
__host__ __device__ inline void rotmat(const double* q, double* R) {
  const double q0 = q[0], q1 = q[1], q2 = q[2], q3 = q[3];
  R[0] = 1.0 - 2.0 * q2 * q2 - 2.0 * q3 * q3;
  R[1] = 2.0 * (q1 * q2 - q3 * q0);
  R[2] = 2.0 * (q1 * q3 + q2 * q0);
  R[3] = 2.0 * (q1 * q2 + q3 * q0);
  R[4] = 1.0 - 2.0 * q1 * q1 - 2.0 * q3 * q3;
  R[5] = 2.0 * (q3 * q2 - q1 * q0);
  R[6] = 2.0 * (q1 * q3 - q2 * q0);
  R[7] = 2.0 * (q3 * q2 + q1 * q0);
  R[8] = 1.0 - 2.0 * q2 * q2 - 2.0 * q1 * q1;
}

// p . q
__host__ __device__ inline void qmul(const double* p, const double* q, double* out) {
  const double s = p[0] * q[0] - (p[1] * q[1] + p[2] * q[2] + p[3] * q[3]);
  const double x = p[0] * q[1] + q[0] * p[1] + (p[2] * q[3] - p[3] * q[2]);
  const double y = p[0] * q[2] + q[0] * p[2] + (p[3] * q[1] - p[1] * q[3]);
  const double z = p[0] * q[3] + q[0] * p[3] + (p[1] * q[2] - p[2] * q[1]);
  out[0] = s;
  out[1] = x;
  out[2] = y;
  out[3] = z;
}

// exp(u) = (cos(|u|/2), sin(|u|/2) u/|u|); below |u| = 1e-4 the factor
// sin(t/2)/t is its Taylor series 1/2 - t^2/48 + t^4/3840.
__host__ __device__ inline void qexp(const double* u, double* out) {
  const double t = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
  const double s = t < 1e-4 ? 0.5 - t * t / 48.0 + t * t * t * t / 3840.0 : sin(0.5 * t) / t;
  out[0] = cos(0.5 * t);
  out[1] = s * u[0];
  out[2] = s * u[1];
  out[3] = s * u[2];
}

// R x and R^T x for a row-major 3x3 R.
__host__ __device__ inline void matvec3(const double* R, const double* x, double* y) {
  y[0] = R[0] * x[0] + R[1] * x[1] + R[2] * x[2];
  y[1] = R[3] * x[0] + R[4] * x[1] + R[5] * x[2];
  y[2] = R[6] * x[0] + R[7] * x[1] + R[8] * x[2];
}
__host__ __device__ inline void matTvec3(const double* R, const double* x, double* y) {
  y[0] = R[0] * x[0] + R[3] * x[1] + R[6] * x[2];
  y[1] = R[1] * x[0] + R[4] * x[1] + R[7] * x[2];
  y[2] = R[2] * x[0] + R[5] * x[1] + R[8] * x[2];
}
__host__ __device__ inline void cross3(const double* a, const double* b, double* c) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}

// ------------------------------------------------------------ grid geometry

// Workgroup sizes (threads) of the FFT passes of a grid, chosen at set-up by
// fft_autotune; every choice gives the same results.
struct FftShape {
  int plane_fwd = 512, proj_plane = 512, plane_inv = 512;        // three-pass path
  int r2c = 256, fwd1 = 256, proj = 256, inv1 = 256, c2r = 256;   // five-pass path
};

// Everything a grid kernel needs about the periodic box and the envelope.
struct GridGeom {
  int n[3];
  int n2h;            // n[2] / 2: stored k2 modes (the Nyquist plane is dropped)
  long long G;        // n0 n1 n2
  double L[3], dx[3], inv_dx[3];
  double dV;
  double eta;
  double sigma, rc, rc2;
  double inv2s2;      // 1 / (2 sigma^2)
  double wnorm;       // (2 pi sigma^2)^(-3/2)
  int P[3];           // stencil points per axis: floor(2 rc / dx) + 1
  // Layout of each component of a real-space field: row-major [i0][i1][i2]
  // (tiled = 0) or tile-major (tiled = 1, when 8 | n0, 8 | n1, 32 | n2):
  // tiles of 8 x 8 x 32 points in row-major tile order, each tile stored
  // contiguously as [i0 % 8][i1 % 8][i2 % 32].  A spreading workgroup then
  // writes its tile as one contiguous block.
  int tiled;
  // Slip channel (Sec. 6.3): walls at y = 0 and y = L1/2, kept by images in
  // the upper half of the box; spreading then also carries the M image blobs
  // (numbered M .. 2M - 1), and the stress noise is mirrored.
  int channel;
  FftShape fft;       // host side: launch shapes of the transform passes
};

// Offset of grid point (i0, i1, i2) within one component of a real-space
// field: field_plane_off(i0) + field_col_off(i1, i2).
__host__ __device__ inline long long field_plane_off(int tiled, int n1, int n2, int i0) {
  return tiled ? (((long long)(i0 >> 3) * n1 * n2) << 3) + ((i0 & 7) << 8) : (long long)i0 * n1 * n2;
}
__host__ __device__ inline long long field_col_off(int tiled, int n2, int i1, int i2) {
  return tiled ? ((long long)((i1 >> 3) * (n2 >> 5) + (i2 >> 5)) << 11) + ((i1 & 7) << 5) + (i2 & 31)
               : (long long)i1 * n2 + i2;
}

// Tiling of the grid for the spreading kernel: tiles of T[0] x T[1] x T[2]
// points (the last tile along an axis may be partial), nt[d] tiles per axis,
// and H[d] neighbour tiles per side whose anchored blobs can reach a tile.
struct TileGeom {
  int T[3];
  int nt[3];
  int H[3];
  int ntiles;
  int S;       // work-item slots per blob: a power of two >= min(T1, P1) min(T2, P2)
  int wz8;         // spreading tables keep 8 axis-2 entries per hit (stencil <= 8 points, >= 2 tiles on axis 2)
};

// Device tables of a suspension's bodies (see BodyHost for the meaning).
struct BodyTables {
  int N, M, n_shapes;
  const int* body_shape;      // N
  const int* body_off;        // N + 1: first blob of each body
  const int* blob_body;       // M
  const int* blob_local;      // M: index of the blob within its shape
  const double* shape_b;      // sum_s n_b(s) x 3, body frame
  const int* shape_boff;      // n_shapes + 1
  const double* shape_pinv;   // n_shapes x 36: body-frame (K^T K)^+
  const double* shape_null;   // n_shapes x 36: body-frame projector onto null(K)
  const double* shape_Lp;     // n_shapes: max blob-blob distance (or a)
  const double* shape_precT;  // concatenated transposed preconditioner inverses
  const long long* shape_prec_off;  // n_shapes
  // Groups of up to PREC_GROUP_MAX bodies of one shape for the matrix-core
  // preconditioner: group g covers bodies group_body[group_first[g] ..
  // group_first[g] + group_count[g]) of shape group_shape[g].
  int n_groups;
  const int* group_body;
  const int* group_first;
  const int* group_count;
  const int* group_shape;
  int mfma;                   // every block fits the matrix-core kernel
};

// ------------------------------------------------------------ launchers

// Parameters of the projection pass: grid, wavenumber scales 2 pi / L_d,
// 1/eta and 1/G; for the noise pass also the Philox key and counter and the
// stress scales.
struct ProjParams {
  int n0, n1, n2h;
  double kf0, kf1, kf2;    // 2 pi / L_d
  double inv_eta;
  double invG;
  // noise
  uint64_t seed, step;
  const uint64_t* step_ptr;   // when set, the step is read from here (graph replays)
  double sdiag, soff;      // sqrt(G var / 2) of diagonal / off-diagonal components
  int channel;             // slip channel: the stress is given its mirror image in y
};

// Arguments and grids of the three plane passes of one stokes_solve (FP32,
// plane path), for launches fused over several suspensions of one grid
// size and one set of workgroup sizes.
struct PlaneArgs {
  const void* in;
  void* out;
  const void *tw1, *tw2;
  int n0, tiled;
  const int* skip;
  LocalGrid grid;
};
struct ProjPlaneArgs {
  void* Z;
  const void* tw;
  ProjParams P;
  const int* skip;
  LocalGrid grid;
};
struct StokesArgs {
  PlaneArgs fwd;
  ProjPlaneArgs proj;
  PlaneArgs inv;
};
// Whether stokes_solve of this geometry runs the FP32 plane path (the
// fusable one).
bool stokes_fusable(const GridGeom& g, int precision);
void stokes_describe(StokesArgs& a, const GridGeom& g, const void* const tw[3], void* real, void* X,
                     const int* skip);
// fwd / inv and proj: ns argument sets each on the device; first_plane
// (shared by the forward and inverse passes) and first_proj: the first
// block of every suspension.
int stokes_fused(const GridGeom& g, const PlaneArgs* fwd, const ProjPlaneArgs* proj, const PlaneArgs* inv, int ns,
                 const int* first_plane, int tot_plane, const int* first_proj, int tot_proj, hipStream_t s);

// FFT / projection / noise (fft.hip).  The three grid buffers hold 3 G values
// of R each; `real` is the real-space field (spread output in, velocity out),
// X and Y are the two transposed half-spectrum layouts.
// Kernels given `skip` (a device int) return at once when *skip != 0: the
// GMRES loop queues iterations ahead and stops them this way once converged.
template <typename R>
int stokes_solve(const GridGeom& g, const Cx<R>* const tw[3], R* real, Cx<R>* X, Cx<R>* Y,
                 hipStream_t s, const int* skip = nullptr);
template <typename R>
// step_ptr (optional): a device counter the kernels read the step from at
// run time instead of `step`, for launches replayed from a captured graph.
int fluct_field(const GridGeom& g, const Cx<R>* const tw[3], R* real, Cx<R>* X, Cx<R>* Y,
                uint64_t seed, uint64_t step, double kT, double dt, hipStream_t s,
                const uint64_t* step_ptr = nullptr);
bool fft_size_supported(int n);
// Times every workgroup size of each pass of g's transform on the given
// buffers (zeroed first) and stores the fastest in g.fft; cached per grid and
// precision for the process.
template <typename R>
int fft_autotune(GridGeom& g, const Cx<R>* const tw[3], R* real, Cx<R>* X, Cx<R>* Y, hipStream_t s);
int philox_normals_dev(uint64_t seed, uint32_t c1, uint64_t step, uint32_t c0_begin, int count,
                       double* out_dev, hipStream_t s);

// Grid <-> blob transfer (grid.hip).
// Counting sort of blobs by the tile of their anchor point; off has
// ntiles + 1 entries and rec (2 M records of tile_record_bytes(); the second
// half is scratch) holds in its first half each blob's stencil origin, tile
// by tile, in blob order within a tile.
size_t tile_record_bytes();
// spos[i] is blob i's position in the sorted order.
// zeroed: count (tile_count_bytes) was already cleared on the stream.
int tile_sort(const GridGeom& g, const TileGeom& t, const double* r, int M, int* tile, int* count, int* off,
              int* cursor, void* rec, int* spos, hipStream_t s, bool zeroed = false);
inline size_t tile_count_bytes(const TileGeom& t) { return ((size_t)t.ntiles * sizeof(int) + 15) / 16 * 16; }
// Spreading tables: per tile, the blobs whose stencil reaches it and their
// per-axis Gaussian factors at the tile's coordinates, built once per
// configuration (after tile_sort) into `tabs` (spread_table_bytes bytes);
// tab_start / tab_count (ntiles each) locate each tile's entries, `order`
// (4 ntiles ints) receives the launch order of the tiles for spread,
// `claimed` is spread_claim_bytes() of scratch (the room counter, then the
// hit-count histogram and its cursors).
constexpr int ORDER_BUCKETS = 256;
constexpr size_t spread_claim_bytes() { return 16 + 2 * ORDER_BUCKETS * sizeof(unsigned int); }
size_t spread_table_bytes(const GridGeom& g, const TileGeom& t, int M, int precision);
template <typename R>
int spread_prepare(const GridGeom& g, const TileGeom& t, const void* rec, const int* off, void* tabs,
                   int* tab_start, int* tab_count, int* order, unsigned int* claimed, hipStream_t s,
                   bool zeroed = false);
// f = S lam on every grid point (the whole field is written) from the
// tables and tile order of the last spread_prepare.  lam_sorted, when
// given, holds lam in the sorted order (3 x M) and is read instead.
template <typename R>
int spread(const GridGeom& g, const TileGeom& t, const void* tabs, const int* order, const double* lam,
           const double* lam_sorted, R* f, hipStream_t s, const int* skip = nullptr);
// v = scale J u, minus U_p + Omega_p x (r_i - Y_p) when V (N x 6) is given.
// sorted, when given, is the record array of tile_sort for the same
// positions r: blobs are then visited in the sorted order (same results).
template <typename R>
int interp(const GridGeom& g, const double* r, const R* u, double* v, int M, double scale,
           const int* blob_body, const double* Y, const double* V, hipStream_t s,
           const int* skip = nullptr, const void* sorted = nullptr);
// Arguments and grids of one spread / interp launch, for launches fused over
// several suspensions of one precision (and, for spreading, one table
// width wz8).  The fields follow spread's and interp's parameters.
struct SpreadArgs {
  GridGeom G;
  TileGeom T;
  const void* tabs;
  const int4* order;
  const double *lam, *lam_sorted;
  void* f;
  const int* skip;
  LocalGrid grid;
};
struct InterpArgs {
  GridGeom G;
  const double* r;
  const void* u;
  double* v;
  int M;
  double scale;
  const int* blob_body;
  const double *Y, *V;
  const int* skip;
  const void* rec;
  LocalGrid grid;
};
void spread_describe(SpreadArgs& a, const GridGeom& g, const TileGeom& t, const void* tabs, const int* order,
                     const double* lam, const double* lam_sorted, void* f, const int* skip);
template <typename R>
int spread_fused(const SpreadArgs* dev_args, int ns, int wz8, const int* first, int total, hipStream_t s);
void interp_describe(InterpArgs& a, const GridGeom& g, const double* r, const void* u, double* v, int M,
                     double scale, const int* blob_body, const double* Y, const double* V, const int* skip,
                     const void* sorted);
template <typename R>
int interp_fused(const InterpArgs* dev_args, int ns, const int* first, int total, hipStream_t s);
// v (M x 3) and the NP differences J(r + dr_k) u - J(r) u into vd (M x NP x 3),
// dr given per blob as M x NP x 3.
template <typename R>
int interp_fd(const GridGeom& g, const double* r, const double* dr, int NP, const R* u,
              double* v, double* vd, int M, hipStream_t s);
int fill_zero(void* p, size_t bytes, hipStream_t s);
// Clears n <= 4 buffers (16-byte aligned sizes and addresses) in one launch.
int fill_zero_many(void* const* ptrs, const size_t* bytes, int n, hipStream_t s);
// y (3 x n0 x n1 x n2, row-major, FP64) = the real-space field x in the layout of g.
template <typename R>
int field_to_rowmajor(const GridGeom& g, const R* x, double* y, hipStream_t s);
// f = (sin(k y_g), 0, 0) on the grid in its layout, k = 2 pi / L1.
template <typename R>
int fill_sine_field(const GridGeom& g, R* f, hipStream_t s);
// *out = sum_i a[3 i] b[3 i] over M blobs, in a fixed order (one workgroup).
int blob_dot_x(const double* a, const double* b, int M, double* out, hipStream_t s);

// Body kernels (body.hip).
int blob_positions(const BodyTables& b, const double* Y, const double* q, double* r,
                   hipStream_t s);
// Largest preconditioner block (3 n_b + 6) the matrix-core kernel takes.
constexpr int PREC_MFMA_MAXDIM = 64;
// Bodies per workgroup of the matrix-core preconditioner: between 4 and 16
// (the columns of one MFMA tile), the most that leave PREC_MIN_GROUPS
// workgroups (fewer bodies give more workgroups to hide the gather and
// scatter latency; more amortise staging the shape's block).
constexpr int PREC_GROUP_MIN = 4;
constexpr int PREC_GROUP_MAX = 16;
constexpr int PREC_MIN_GROUPS = 1024;
// z = P^-1 x (block-diagonal preconditioner, Sec. 2.2) and, when yV is
// given, the body rows of the saddle operator at z: yV = -K^T z_lam - Pi z_V.
// When zs is given, z_lam is also written in the spreading order:
// zs[3 spos[i] + c] = z_lam[3 i + c].
// With mirror = M (slip channel), blob i's image (spreading blob M + i) also
// gets its force R z_lam in the spreading order: zs[3 spos[M + i] + c].
int precond_apply(const BodyTables& b, const double* q, const double* x, double* z, double* yV,
                  const int* spos, double* zs, int maxdim, hipStream_t s, const int* skip = nullptr,
                  int mirror = 0);
// The arguments and grid of one matrix-core precond_apply, for launches fused
// over several suspensions.
struct PrecondArgs {
  BodyTables B;
  const double* q;
  const double* x;
  double *z, *yV;
  const int* spos;
  double* zs;
  const int* skip;
  int mirror;
  LocalGrid grid;
};
// Whether precond_apply runs on the matrix cores (the fusable kernel).
bool precond_fusable(const BodyTables& b, int maxdim);
void precond_describe(PrecondArgs& a, const BodyTables& b, const double* q, const double* x, double* z, double* yV,
                      const int* spos, double* zs, const int* skip, int mirror);
int precond_fused(const PrecondArgs* dev_args, int ns, const int* first, int total, hipStream_t s);
// Slip channel: rs = [r; sigma(r)] (2M x 3), sigma(x, y, z) = (x, L1 - y, z).
int mirror_positions(const double* r, int M, double L1, double* rs, hipStream_t s);
// Blob forces lam in the spreading order of the last tile sort: zs[3 spos[i] +
// c] = lam[3 i + c] and, with mirror = M, the images' R lam at spos[M + i].
int sort_forces(const double* lam, const int* spos, int M, int mirror, double* zs, hipStream_t s);
// Harmonic blob-wall repulsion of the slip channel (Sec. 6.3) on the y
// component of fblob (M x 3): k (b - y) for y < b, -k (b - (H - y)) for
// H - y < b; add: add to fblob (else fblob is overwritten).
int wall_forces(const double* r, int M, double H, double k, double b, double* fblob, bool add, hipStream_t s);
// FD / RFD perturbations: displacements of each blob (M x NP x 3) and, for
// RFD, the Philox normals of each body (N x 6); step_ptr as in fluct_field.
int fd_displacements(const BodyTables& b, const double* q, double delta, int mode,
                     uint64_t seed, uint64_t step, double* dr, double* wrfd, hipStream_t s,
                     const double* Y = nullptr, double* r = nullptr, const uint64_t* step_ptr = nullptr);
// The device step counter of a handle: set to v, or advanced by one.
int step_counter_set(uint64_t* c, uint64_t v, hipStream_t s);
int step_counter_bump(uint64_t* c, hipStream_t s);
// calV, d_p and (same launch) nu = 1 + half_dt sum_p d_p; counter: one
// zeroed unsigned int, left at zero.
int body_lsq_div(const BodyTables& b, const double* q, const double* v, const double* vd,
                 const double* wrfd, double delta, int mode, double* calV, double* d,
                 unsigned int* counter, double half_dt, double* nu, hipStream_t s);
// Step 4 with the midpoint blob positions rm in the same launch.
int midpoint_positions(const BodyTables& b, const double* Y, const double* q, const double* calV, double h,
                       double* Ym, double* qm, double* rm, hipStream_t s);
// Step 6; sets *nonfinite (when given) if a new position or quaternion is not finite.
int update(const BodyTables& b, double* Y, double* q, const double* V, const double* nu,
           double dt, int* nonfinite, hipStream_t s);
// rhs = [-(vslip + cbg vbg_x e_x + shear flow); -(I - Pi) F]; vslip, vbg
// (M x 3, only the x components of vbg are used) may be null.
int rhs_build(const BodyTables& b, const double* q, const double* Y, const double* r,
              const double* vslip, const double* vbg, double cbg, const double* F, double shear,
              double Ly, double* rhs, hipStream_t s);
// zeroed: cell_count (cell_count_bytes) was already cleared on the stream.
int steric_forces(const BodyTables& b, const GridGeom& g, const double* r, double k,
                  double cutoff, int* cell_count, int* cell_list, int cap, const int nc[3],
                  int* overflow, double* fblob, hipStream_t s, bool zeroed = false);
inline size_t cell_count_bytes(const int nc[3]) {
  return ((size_t)nc[0] * nc[1] * nc[2] * sizeof(int) + 15) / 16 * 16;
}
int body_forces(const BodyTables& b, const double* Y, const double* r, const double* fblob,
                const double* cforce, double* F, hipStream_t s);
int check_finite(const double* x, long long n, int* flag, hipStream_t s);
// Sets flag[0] if a position of Y (N x 3) is not finite and flag[1] if a
// quaternion of q (N x 4) is off unit norm by more than qtol (flags zeroed
// by the caller).
int check_state(const double* Y, const double* q, int N, double qtol, int* flag, hipStream_t s);

// Krylov vector kernels (solver.hip).
constexpr int DOT_MAX_BLOCKS = 512;
// h[j] = V_j . w (j < k), plus h[k] = w . w when with_self; partial holds
// (k + 1) x DOT_MAX_BLOCKS doubles, counter one zeroed unsigned int.  With
// init (k = 0, with_self: h[0] = |b|^2), the reduction's last block also sets
// up the GMRES state (tolerance, iteration limit, |b|).
struct GmresState;
int multi_dot(const double* V, long long ld, int k, const double* w, long long n, bool with_self,
              double* partial, unsigned int* counter, double* h, hipStream_t s, GmresState* init = nullptr,
              double tol = 0.0, int maxit = 0);
int multi_axpy(double* w, const double* V, long long ld, int k, const double* h, double sign,
               long long n, hipStream_t s);
// out = (w - V h2) / sqrt(h2[k] - |h2[0..k)|^2)
int ortho_finish(const double* w, const double* V, long long ld, int k, const double* h2, double* out,
                 long long n, hipStream_t s);
// Device-resident GMRES bookkeeping (restart length <= GM_MAXR).  The first
// GM_STATUS_BYTES hold what the host polls: est, its, kdone, done, converged.
constexpr int GM_MAXR = 64;
struct GmresState {
  double est;        // relative residual estimate
  int its;           // iterations so far (all cycles)
  int kdone;         // columns of the current cycle
  int done;          // the current cycle is over
  int converged;
  double nb;         // |b|
  double tol;
  int maxit, pad;
  double g[GM_MAXR + 1], cs[GM_MAXR], sn[GM_MAXR], y[GM_MAXR];
  double H[(GM_MAXR + 1) * GM_MAXR];   // H[j * GM_MAXR + k]
};
constexpr size_t GM_STATUS_BYTES = 24;
// One Arnoldi orthogonalisation (CGS with one re-orthogonalisation) of w
// against V_0..V_{k-1}: out = normalised remainder, h1 (k) and h2s (k + 1:
// h2 then w.w) stored for the Hessenberg column.  With st, the last kernel
// also updates Hessenberg column k - 1 of a restart of length m and writes
// the status to hstat (device-visible pinned host memory, or null).  partial1/2 hold
// (k + 1) x ceil(n / 1024) doubles each.
int arnoldi_orthogonalise(double* w, const double* V, long long ld, int k, long long n, double* partial1,
                          double* partial2, double* out, double* h1, double* h2s, hipStream_t s,
                          const int* skip, GmresState* st, int m, unsigned char* hstat);

// The arguments and grids of one arnoldi_orthogonalise, for launches fused
// over several suspensions (the fields follow arnoldi_orthogonalise's
// parameters; shortv selects the kernels' chunk length).
struct ArnoldiArgs {
  double* w;
  const double* V;
  long long ld, n;
  int k, m, nchunk, shortv;
  double *partial1, *partial2, *out, *h1, *h2s;
  const int* skip;
  GmresState* st;
  unsigned char* hstat;
  LocalGrid g_dot, g_axpy, g_fin;
};
int arnoldi_describe(ArnoldiArgs& a, double* w, const double* V, long long ld, int k, long long n,
                     double* partial1, double* partial2, double* out, double* h1, double* h2s, const int* skip,
                     GmresState* st, int m, unsigned char* hstat);
// One fused launch of each Arnoldi kernel over ns suspensions with the same
// shortv: dev_args (ns entries) and, for each kernel, the first block of
// every suspension (first_dot, first_axpy, first_fin: ns entries) on the
// device; tot_* the total block counts.
int arnoldi_fused(const ArnoldiArgs* dev_args, int ns, int shortv, const int* first_dot, int tot_dot,
                  const int* first_axpy, int tot_axpy, const int* first_fin, int tot_fin, hipStream_t s);

// y = H^-1 g over the cycle, then x += V y.
int gm_finish_cycle(GmresState* st, double* x, const double* V, long long ld, long long n, hipStream_t s);
// out = w / sqrt(nrm2[0]); with cycle, also starts a GMRES restart cycle
// from beta^2 = nrm2[0]; with zero, also clears zero[0, nzero).
int scale_by_inv_sqrt(const double* w, const double* nrm2, double* out, long long n,
                      hipStream_t s, GmresState* cycle = nullptr, double* zero = nullptr,
                      long long nzero = 0);
int copy_scaled(const double* x, double a, double* y, long long n, hipStream_t s);
int sub_from(const double* b, double* w, long long n, hipStream_t s);   // w = b - w

}  // namespace gdc
