// Krylov vector kernels for the device-resident GMRES of the saddle problem
// (Sec. 2.2).  Vectors are FP64 and live in one basis array V[(m+1) x ld].
//
// Each Arnoldi step orthogonalises by classical Gram-Schmidt with one
// re-orthogonalisation in three launches over fixed chunks of the vectors
// (k_dot2d, k_axpy_dot, k_ortho_finish2):
//   (1) partial sums of h1 = V^T w per chunk;
//   (2) every block reduces those partials (fixed order), w -= V h1 on its
//       chunk, and writes the chunk's partial sums of h2 = V^T w and w^T w;
//   (3) every block reduces them, V_{k+1} = (w - V h2) / sqrt(w^T w - |h2|^2)
// (|w - V h2|^2 = w^T w - |h2|^2 for orthonormal V, and h2 is a small
// correction, so there is no cancellation).  No atomics: a solve is
// reproducible run to run.  Block 0 also stores h1, h2 and w^T w for the
// host's Hessenberg column.

#include "gdc_internal.h"

namespace gdc {
namespace {

constexpr int NT = 256;
constexpr int MAXK = 64;   // vectors per launch

__device__ __forceinline__ double block_sum(double v, double* sh) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < NT / 64; ++w) t += sh[w];
  return t;
}

// h[j] = V_j . w for j < k, and h[k] = w . w when with_self.  Grid
// (nchunk, kk): block (c, j) sums vector j over chunk c into
// partial[j * nchunk + c]; the last block to finish (counter, zero on entry
// and left at zero) reduces each row with one wavefront per row.
__device__ void gm_init_dev(GmresState* st, double nb2, double tol, int maxit);
__device__ void gm_cycle_dev(GmresState* st, const double* __restrict__ beta2);

__global__ __launch_bounds__(NT) void k_multi_dot(const double* __restrict__ V, long long ld, int k,
                                                  const double* __restrict__ w, long long n,
                                                  double* __restrict__ partial, unsigned int* __restrict__ counter,
                                                  double* __restrict__ h, GmresState* ist, double tol, int maxit) {
  __shared__ double sh[NT / 64];
  __shared__ bool last;
  const int j = blockIdx.y, nchunk = gridDim.x, kk = gridDim.y;
  const long long chunk = (n + nchunk - 1) / nchunk;
  const long long lo = chunk * blockIdx.x;
  const long long hi = min(n, lo + chunk);
  const double* v = j < k ? V + ld * j : w;
  double s = 0.0;
  for (long long e = lo + threadIdx.x; e < hi; e += NT) s += v[e] * w[e];
  const double t = block_sum(s, sh);
  if (threadIdx.x == 0) partial[(long long)j * nchunk + blockIdx.x] = t;
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) last = atomicAdd(counter, 1u) == (unsigned)(nchunk * kk - 1);
  __syncthreads();
  if (!last) return;
  __threadfence();
  const volatile double* pv = partial;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int jj = wave; jj < kk; jj += NT / 64) {
    double a = 0.0;
    for (int c = lane; c < nchunk; c += 64) a += pv[(long long)jj * nchunk + c];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o, 64);
    if (lane == 0) h[jj] = a;
    // a solve's set-up: the GMRES state from |b|^2 (row 0, this thread's own sum)
    if (ist && jj == 0 && lane == 0) gm_init_dev(ist, a, tol, maxit);
  }
  if (threadIdx.x == 0) *counter = 0u;
}

// Vector elements per block in the Arnoldi kernels: EPT elements per thread,
// 1 for vectors of up to DOT_MAX_BLOCKS * NT elements (more blocks, shorter
// dependency chains), else 4.
constexpr int EPT_LONG = 4;

// Sum over waves of a per-wave value, one barrier; valid in thread 0.
__device__ __forceinline__ void wave_reduce_to(double v, double* slot) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  if ((threadIdx.x & 63) == 0) slot[threadIdx.x >> 6] = v;
}

// partial[j * gridDim.x + c] = sum over chunk c of V_j . w, grid (nchunk, kk);
// row j = k (when kk = k + 1) is w . w.  One vector per block keeps every
// load of a block independent.
template <int EPT>
__device__ __forceinline__ void dot2d_body(const double* __restrict__ V, long long ld, int k,
                                           const double* __restrict__ w, long long n,
                                           double* __restrict__ partial, const int* __restrict__ skip,
                                           const BlockIx& bi) {
  if (skip && *skip) return;
  __shared__ double sh[NT / 64];
  const int j = bi.y;
  const double* v = j < k ? V + ld * j : w;
  const long long lo = (long long)bi.x * (EPT * NT);
  double a = 0.0;
#pragma unroll
  for (int m = 0; m < EPT; ++m) {
    const long long e = lo + threadIdx.x + m * NT;
    if (e < n) a += v[e] * w[e];
  }
  wave_reduce_to(a, sh);
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int q = 0; q < NT / 64; ++q) t += sh[q];
    partial[(long long)j * bi.gx + bi.x] = t;
  }
}

template <int EPT>
__global__ __launch_bounds__(NT) void k_dot2d(const double* __restrict__ V, long long ld, int k,
                                              const double* __restrict__ w, long long n,
                                              double* __restrict__ partial, const int* __restrict__ skip) {
  dot2d_body<EPT>(V, ld, k, w, n, partial, skip, hw_block());
}

// Reduces rows j < k of partial (ncol columns) into hs[j]: wave w takes
// rows w, w + 4, ..., lane l columns l, l + 64, ... summed in that order,
// then across the wave by shuffles.  Four rows' loads per wave, up to 512
// columns each, are in flight together.
__device__ __forceinline__ void reduce_rows(const double* __restrict__ partial, int k, int ncol, double* hs) {
  constexpr int QMAX = 8, RB = 4;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int j0 = wave; j0 < k; j0 += RB * (NT / 64)) {
    double a[RB];
#pragma unroll
    for (int r = 0; r < RB; ++r) a[r] = 0.0;
    for (int c0 = 0; c0 < ncol; c0 += 64 * QMAX) {
#pragma unroll
      for (int r = 0; r < RB; ++r) {
        const int j = j0 + r * (NT / 64);
        double x[QMAX];
#pragma unroll
        for (int q = 0; q < QMAX; ++q) {
          const int c = c0 + lane + 64 * q;
          x[q] = (j < k && c < ncol) ? partial[(long long)j * ncol + c] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < QMAX; ++q) a[r] += x[q];
      }
    }
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      double v = a[r];
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
      const int j = j0 + r * (NT / 64);
      if (lane == 0 && j < k) hs[j] = v;
    }
  }
}

// w -= V h1 with h1 reduced from partial1 (k rows); block 0 stores h1.
// Then, from the updated chunk, partial2[j * gridDim.x + c] = chunk sums of
// V_j . w (j < k) and w . w (row k), each reduced within waves by shuffles
// and across the block's waves in a fixed order.  The dot rows go eight at a
// time so that their loads are in flight together.
template <int EPT>
__device__ __forceinline__ void axpy_dot_body(double* __restrict__ w, const double* __restrict__ V,
                                              long long ld, int k, const double* __restrict__ partial1,
                                              long long n, double* __restrict__ hout,
                                              double* __restrict__ partial2, const int* __restrict__ skip,
                                              const BlockIx& bi) {
  if (skip && *skip) return;
  constexpr int JB = 8;
  __shared__ double hs[MAXK];
  __shared__ double wp[MAXK][NT / 64];
  reduce_rows(partial1, k, bi.gx, hs);
  __syncthreads();
  if (bi.x == 0)
    for (int j = threadIdx.x; j < k; j += NT) hout[j] = hs[j];
  const long long lo = (long long)bi.x * (EPT * NT);
  double xw[EPT];
#pragma unroll
  for (int m = 0; m < EPT; ++m) {
    const long long e = lo + threadIdx.x + m * NT;
    double x = 0.0;
    if (e < n) {
      x = w[e];
#pragma unroll 8
      for (int j = 0; j < k; ++j) x -= hs[j] * V[ld * j + e];
      w[e] = x;
    }
    xw[m] = x;
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int j0 = 0; j0 <= k; j0 += JB) {
    double a[JB];
#pragma unroll
    for (int u = 0; u < JB; ++u) {
      const int j = j0 + u;
      a[u] = 0.0;
#pragma unroll
      for (int m = 0; m < EPT; ++m) {
        const long long e = lo + threadIdx.x + m * NT;
        const double vj = j < k ? (e < n ? V[ld * j + e] : 0.0) : (j == k ? xw[m] : 0.0);
        a[u] += vj * xw[m];
      }
    }
#pragma unroll
    for (int u = 0; u < JB; ++u) {
      double v = a[u];
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
      if (lane == 0 && j0 + u <= k) wp[j0 + u][wave] = v;
    }
  }
  __syncthreads();
  for (int j = threadIdx.x; j <= k; j += NT) {
    double t = 0.0;
    for (int q = 0; q < NT / 64; ++q) t += wp[j][q];
    partial2[(long long)j * bi.gx + bi.x] = t;
  }
}

template <int EPT>
__global__ __launch_bounds__(NT) void k_axpy_dot(double* __restrict__ w, const double* __restrict__ V,
                                                 long long ld, int k, const double* __restrict__ partial1,
                                                 long long n, double* __restrict__ hout,
                                                 double* __restrict__ partial2, const int* __restrict__ skip) {
  axpy_dot_body<EPT>(w, V, ld, k, partial1, n, hout, partial2, skip, hw_block());
}

// Column k of the Hessenberg matrix from the Gram-Schmidt coefficients, by
// one workgroup: H[j][k] = h1[j] + h2[j] (j <= k), H[k+1][k] =
// sqrt(w.w - |h2|^2) with w.w = h2[k+1]; then the previous rotations, a new
// one, and the residual estimate |g[k+1]| / |b|; done (and converged) are set
// when the cycle ends.  The rotations are staged in LDS first so that thread
// 0 works without global-memory round trips; the status fields (est, its,
// kdone, done, converged) then go to `out` (pinned host memory) when given.
// Must be called by every thread of the block.
__device__ void gm_column_block(GmresState* st, int k, int m, const double* __restrict__ h1,
                                const double* h2, unsigned char* out) {
  __shared__ double cs[GM_MAXR], sn[GM_MAXR], col[GM_MAXR + 1], h1s[GM_MAXR];
  __shared__ double g_k, nb, tol, est;
  __shared__ int done, its, maxit, conv;
  const int tid = threadIdx.x;
  for (int j = tid; j < k; j += NT) {
    cs[j] = st->cs[j];
    sn[j] = st->sn[j];
  }
  for (int j = tid; j <= k; j += NT) h1s[j] = h1[j];
  if (tid == 0) {
    done = st->done;
    its = st->its;
    maxit = st->maxit;
    g_k = st->g[k];
    nb = st->nb;
    tol = st->tol;
    est = st->est;
    conv = st->converged;
  }
  __syncthreads();
  const bool update = !done;
  if (update && tid == 0) {
    double h2sq = 0.0;
    for (int j = 0; j <= k; ++j) {
      col[j] = h1s[j] + h2[j];
      h2sq += h2[j] * h2[j];
    }
    col[k + 1] = sqrt(fmax(0.0, h2[k + 1] - h2sq));
    for (int j = 0; j < k; ++j) {
      const double a = col[j], b = col[j + 1];
      col[j] = cs[j] * a + sn[j] * b;
      col[j + 1] = -sn[j] * a + cs[j] * b;
    }
    const double a = col[k], b = col[k + 1];
    const double den = hypot(a, b);
    const double c = den > 0.0 ? a / den : 1.0, sv = den > 0.0 ? b / den : 0.0;
    col[k] = den;
    col[k + 1] = 0.0;
    st->cs[k] = c;
    st->sn[k] = sv;
    st->g[k + 1] = -sv * g_k;
    st->g[k] = c * g_k;
    its += 1;
    est = fabs(sv * g_k) / nb;
    if (est <= tol) {
      conv = 1;
      done = 1;
    } else if (its >= maxit || den == 0.0 || k + 1 >= m) {
      done = 1;
    }
    st->its = its;
    st->kdone = k + 1;
    st->est = est;
    st->done = done;
    st->converged = conv;
  }
  __syncthreads();
  if (update)
    for (int j = tid; j <= k + 1; j += NT) st->H[j * GM_MAXR + k] = col[j];
  if (out && tid == 0) {
    volatile double* d = reinterpret_cast<volatile double*>(out);
    volatile int* i = reinterpret_cast<volatile int*>(out + 8);
    d[0] = est;
    i[0] = its;
    i[1] = update ? k + 1 : st->kdone;
    i[2] = done;
    i[3] = conv;
  }
}

// out = (w - V h2) / sqrt(s - |h2|^2) with (h2, s) reduced from partial2
// (ncol columns), by blocks 0 .. nchunk - 1 of EPT * NT elements.  The extra last block (nchunk) stores h2 and s
// in hout and, when st is given and its cycle is not over, updates
// Hessenberg column k - 1 from h1 and h2 and writes the status to hstat
// (pinned host memory; visible to the host once the kernel has completed),
// in parallel with the chunk work.  No skip flag: the last block reads
// `done` before it may set it, and an iteration past the end of a cycle only
// writes a basis vector that is never used.
template <int EPT>
__device__ __forceinline__ void ortho_finish2_body(const double* __restrict__ w, const double* __restrict__ V,
                                                   long long ld, int k, const double* __restrict__ partial2,
                                                   int ncol, long long n, double* __restrict__ out,
                                                   double* __restrict__ hout, GmresState* st, int m,
                                                   const double* __restrict__ h1, unsigned char* hstat,
                                                   const BlockIx& bi) {
  __shared__ double hs[MAXK];
  __shared__ double scale;
  reduce_rows(partial2, k + 1, ncol, hs);
  __syncthreads();
  if (threadIdx.x == 0) {
    double hh = 0.0;
    for (int j = 0; j < k; ++j) hh += hs[j] * hs[j];
    const double nrm2 = hs[k] - hh;
    scale = nrm2 > 0.0 ? 1.0 / sqrt(nrm2) : 0.0;
  }
  const int nchunk = bi.gx - 1;
  if (bi.x == nchunk) {
    for (int j = threadIdx.x; j <= k; j += NT) hout[j] = hs[j];
    if (st) gm_column_block(st, k - 1, m, h1, hs, hstat);
    return;
  }
  __syncthreads();
  const double a = scale;
  const long long lo = (long long)bi.x * (EPT * NT);
#pragma unroll
  for (int m = 0; m < EPT; ++m) {
    const long long e = lo + threadIdx.x + m * NT;
    if (e < n) {
      double x = w[e];
#pragma unroll 8
      for (int j = 0; j < k; ++j) x -= hs[j] * V[ld * j + e];
      out[e] = a * x;
    }
  }
}

template <int EPT>
__global__ __launch_bounds__(NT) void k_ortho_finish2(const double* __restrict__ w, const double* __restrict__ V,
                                                      long long ld, int k, const double* __restrict__ partial2,
                                                      int ncol, long long n, double* __restrict__ out,
                                                      double* __restrict__ hout, GmresState* st, int m,
                                                      const double* __restrict__ h1, unsigned char* hstat) {
  ortho_finish2_body<EPT>(w, V, ld, k, partial2, ncol, n, out, hout, st, m, h1, hstat, hw_block());
}

// The three Arnoldi launches fused over several suspensions (one ArnoldiArgs
// each): block b belongs to the suspension s with first[s] <= b <
// first[s + 1], and runs that suspension's block b - first[s].
template <int EPT>
__global__ __launch_bounds__(NT) void k_dot2d_fused(const ArnoldiArgs* __restrict__ a,
                                                    const int* __restrict__ first, int ns) {
  const int sidx = fused_suspension(first, ns, blockIdx.x);
  const ArnoldiArgs& A = a[sidx];
  dot2d_body<EPT>(A.V, A.ld, A.k, A.w, A.n, A.partial1, A.skip,
                  fused_block(A.g_dot, (int)blockIdx.x - first[sidx]));
}

template <int EPT>
__global__ __launch_bounds__(NT) void k_axpy_dot_fused(const ArnoldiArgs* __restrict__ a,
                                                       const int* __restrict__ first, int ns) {
  const int sidx = fused_suspension(first, ns, blockIdx.x);
  const ArnoldiArgs& A = a[sidx];
  axpy_dot_body<EPT>(A.w, A.V, A.ld, A.k, A.partial1, A.n, A.h1, A.partial2, A.skip,
                     fused_block(A.g_axpy, (int)blockIdx.x - first[sidx]));
}

template <int EPT>
__global__ __launch_bounds__(NT) void k_ortho_finish2_fused(const ArnoldiArgs* __restrict__ a,
                                                            const int* __restrict__ first, int ns) {
  const int sidx = fused_suspension(first, ns, blockIdx.x);
  const ArnoldiArgs& A = a[sidx];
  ortho_finish2_body<EPT>(A.w, A.V, A.ld, A.k, A.partial2, A.nchunk, A.n, A.out, A.h2s, A.st, A.m, A.h1,
                          A.hstat, fused_block(A.g_fin, (int)blockIdx.x - first[sidx]));
}

// w += sign * sum_j h_j V_j
__global__ __launch_bounds__(NT) void k_multi_axpy(double* __restrict__ w, const double* __restrict__ V,
                                                   long long ld, int k, const double* __restrict__ h,
                                                   double sign, long long n) {
  __shared__ double hs[MAXK];
  for (int j = threadIdx.x; j < k; j += NT) hs[j] = h[j];
  __syncthreads();
  const long long stride = (long long)gridDim.x * NT;
  for (long long e = (long long)blockIdx.x * NT + threadIdx.x; e < n; e += stride) {
    double acc = 0.0;
    for (int j = 0; j < k; ++j) acc += hs[j] * V[ld * j + e];
    w[e] += sign * acc;
  }
}

// out = (w - V h) / sqrt(s - |h|^2), h = h2[0..k), s = h2[k]
__global__ __launch_bounds__(NT) void k_ortho_finish(const double* __restrict__ w, const double* __restrict__ V,
                                                     long long ld, int k, const double* __restrict__ h2,
                                                     double* __restrict__ out, long long n) {
  __shared__ double hs[MAXK];
  __shared__ double scale;
  for (int j = threadIdx.x; j < k; j += NT) hs[j] = h2[j];
  __syncthreads();
  if (threadIdx.x == 0) {
    double hh = 0.0;
    for (int j = 0; j < k; ++j) hh += hs[j] * hs[j];
    const double nrm2 = h2[k] - hh;
    scale = nrm2 > 0.0 ? 1.0 / sqrt(nrm2) : 0.0;
  }
  __syncthreads();
  const double a = scale;
  const long long stride = (long long)gridDim.x * NT;
  for (long long e = (long long)blockIdx.x * NT + threadIdx.x; e < n; e += stride) {
    double acc = 0.0;
    for (int j = 0; j < k; ++j) acc += hs[j] * V[ld * j + e];
    out[e] = a * (w[e] - acc);
  }
}

// out = w / sqrt(nrm2); with cst, block 0 also starts the GMRES cycle from
// nrm2 = beta^2; with zero, the kernel also clears zero[0, nzero).
__global__ void k_scale_inv_sqrt(const double* __restrict__ w, const double* __restrict__ nrm2,
                                 double* __restrict__ out, long long n, GmresState* cst,
                                 double* __restrict__ zero, long long nzero) {
  if (cst && blockIdx.x == 0 && threadIdx.x == 0) gm_cycle_dev(cst, nrm2);
  const double a = nrm2[0] > 0.0 ? 1.0 / sqrt(nrm2[0]) : 0.0;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) out[e] = a * w[e];
  if (zero)
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < nzero; e += stride) zero[e] = 0.0;
}

__global__ void k_copy_scaled(const double* __restrict__ x, double a, double* __restrict__ y, long long n) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) y[e] = a * x[e];
}

__global__ void k_sub_from(const double* __restrict__ b, double* __restrict__ w, long long n) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) w[e] = b[e] - w[e];
}

// ------------------------------------------------------------ GMRES bookkeeping
// The Hessenberg matrix, its Givens rotations and the residual estimate live
// on the device (GmresState), updated by the extra block of each iteration's
// last Arnoldi kernel, so the host can queue iterations ahead of the GPU;
// `done` ends a restart cycle and makes the queued kernels of later
// iterations return.  The set-up runs in the last block of the |b|^2
// reduction, a cycle's start in the kernel that scales V_0.

__device__ void gm_init_dev(GmresState* st, double nb2, double tol, int maxit) {
  const double nb = sqrt(fmax(nb2, 0.0));
  st->nb = nb;
  st->tol = tol;
  st->maxit = maxit;
  st->its = 0;
  st->kdone = 0;
  st->converged = nb == 0.0 ? 1 : 0;
  st->done = st->converged;
  st->est = nb == 0.0 ? 0.0 : 1.0;
}

// Start of a restart cycle with residual norm^2 beta2: g = (beta, 0, ...).
__device__ void gm_cycle_dev(GmresState* st, const double* __restrict__ beta2) {
  st->kdone = 0;
  if (st->converged) {
    st->done = 1;
    return;
  }
  const double beta = sqrt(fmax(beta2[0], 0.0));
  st->est = beta / st->nb;
  st->g[0] = beta;
  if (st->est <= st->tol) {
    st->converged = 1;
    st->done = 1;
  } else {
    st->done = st->its >= st->maxit ? 1 : 0;
  }
}

// y = H^-1 g over the cycle's kdone columns (back substitution).
// End of a restart cycle: y = H^-1 g by back-substitution over the cycle's
// kdone columns, then x += sum_j y_j V_j.  Every block stages H's upper
// triangle and g in LDS and solves the small system itself (thread 0, the
// same arithmetic in every block, so all blocks hold the same y); block 0
// also stores y in the state.
__global__ __launch_bounds__(NT) void k_gm_update(double* __restrict__ x, const double* __restrict__ V,
                                                  long long ld, GmresState* __restrict__ st, long long n) {
  __shared__ double Hs[GM_MAXR * GM_MAXR];
  __shared__ double gs[GM_MAXR], ys[GM_MAXR];
  const int k = st->kdone;
  for (int e = threadIdx.x; e < k * k; e += NT) {
    const int i = e / k, j = e - i * k;
    Hs[i * GM_MAXR + j] = j >= i ? st->H[i * GM_MAXR + j] : 0.0;
  }
  for (int j = threadIdx.x; j < k; j += NT) gs[j] = st->g[j];
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = k - 1; i >= 0; --i) {
      double t = gs[i];
      for (int j = i + 1; j < k; ++j) t -= Hs[i * GM_MAXR + j] * ys[j];
      const double d = Hs[i * GM_MAXR + i];
      ys[i] = d != 0.0 ? t / d : 0.0;
    }
  }
  __syncthreads();
  if (blockIdx.x == 0)
    for (int j = threadIdx.x; j < k; j += NT) st->y[j] = ys[j];
  const long long stride = (long long)gridDim.x * NT;
  for (long long e = (long long)blockIdx.x * NT + threadIdx.x; e < n; e += stride) {
    double acc = 0.0;
    for (int j = 0; j < k; ++j) acc += ys[j] * V[ld * j + e];
    x[e] += acc;
  }
}

inline unsigned grid_for(long long n) {
  const long long b = (n + NT - 1) / NT;
  return (unsigned)(b < 1024 ? (b > 0 ? b : 1) : 1024);
}

}  // namespace

int multi_dot(const double* V, long long ld, int k, const double* w, long long n, bool with_self,
              double* partial, unsigned int* counter, double* h, hipStream_t s, GmresState* init, double tol,
              int maxit) {
  if (k + (with_self ? 1 : 0) <= 0) return GDC_OK;
  if (k + 1 > MAXK) {
    set_error("multi_dot: too many vectors");
    return GDC_EINVAL;
  }
  const long long want = (n + 16 * NT - 1) / (16 * NT);
  const unsigned nchunk = (unsigned)(want < DOT_MAX_BLOCKS ? (want > 0 ? want : 1) : DOT_MAX_BLOCKS);
  const unsigned kk = (unsigned)(k + (with_self ? 1 : 0));
  if (init && !(k == 0 && with_self)) {
    set_error("multi_dot: the GMRES set-up needs exactly |w|^2");
    return GDC_EINVAL;
  }
  hipLaunchKernelGGL(k_multi_dot, dim3(nchunk, kk), dim3(NT), 0, s, V, ld, k, w, n, partial, counter, h, init, tol,
                     maxit);
  return check_launch("k_multi_dot");
}

int multi_axpy(double* w, const double* V, long long ld, int k, const double* h, double sign, long long n,
               hipStream_t s) {
  if (k <= 0) return GDC_OK;
  if (k > MAXK) {
    set_error("multi_axpy: too many vectors");
    return GDC_EINVAL;
  }
  hipLaunchKernelGGL(k_multi_axpy, dim3(grid_for(n)), dim3(NT), 0, s, w, V, ld, k, h, sign, n);
  return check_launch("k_multi_axpy");
}

int ortho_finish(const double* w, const double* V, long long ld, int k, const double* h2, double* out, long long n,
                 hipStream_t s) {
  if (k >= MAXK) {
    set_error("ortho_finish: too many vectors");
    return GDC_EINVAL;
  }
  hipLaunchKernelGGL(k_ortho_finish, dim3(grid_for(n)), dim3(NT), 0, s, w, V, ld, k, h2, out, n);
  return check_launch("k_ortho_finish");
}

int arnoldi_describe(ArnoldiArgs& a, double* w, const double* V, long long ld, int k, long long n,
                     double* partial1, double* partial2, double* out, double* h1, double* h2s, const int* skip,
                     GmresState* st, int m, unsigned char* hstat) {
  if (k < 1 || k + 1 >= MAXK) {
    set_error("arnoldi_orthogonalise: basis size out of range");
    return GDC_EINVAL;
  }
  const bool shortv = n <= (long long)DOT_MAX_BLOCKS * NT;
  const long long per = shortv ? NT : (long long)EPT_LONG * NT;
  const unsigned nchunk = (unsigned)((n + per - 1) / per);
  if (nchunk > (unsigned)DOT_MAX_BLOCKS * 4) {
    set_error("arnoldi_orthogonalise: vector too long");
    return GDC_EINVAL;
  }
  if (st && (k > m || m > GM_MAXR)) {
    set_error("arnoldi_orthogonalise: column out of range");
    return GDC_EINVAL;
  }
  a.w = w;
  a.V = V;
  a.ld = ld;
  a.n = n;
  a.k = k;
  a.m = m;
  a.nchunk = (int)nchunk;
  a.shortv = shortv ? 1 : 0;
  a.partial1 = partial1;
  a.partial2 = partial2;
  a.out = out;
  a.h1 = h1;
  a.h2s = h2s;
  a.skip = skip;
  a.st = st;
  a.hstat = hstat;
  a.g_dot = LocalGrid{(int)nchunk, k, 1};
  a.g_axpy = LocalGrid{(int)nchunk, 1, 1};
  // the finishing pass is a plain scaled update: with short vectors, longer
  // chunks and fewer blocks reducing the partial sums
  const unsigned nfin = shortv ? (unsigned)((n + EPT_LONG * NT - 1) / (EPT_LONG * NT)) : nchunk;
  a.g_fin = LocalGrid{(int)nfin + 1, 1, 1};
  return GDC_OK;
}

int arnoldi_orthogonalise(double* w, const double* V, long long ld, int k, long long n, double* partial1,
                          double* partial2, double* out, double* h1, double* h2s, hipStream_t s,
                          const int* skip, GmresState* st, int m, unsigned char* hstat) {
  ArnoldiArgs a;
  GDC_TRY(arnoldi_describe(a, w, V, ld, k, n, partial1, partial2, out, h1, h2s, skip, st, m, hstat));
  const dim3 gd(a.g_dot.gx, a.g_dot.gy), ga(a.g_axpy.gx), gf(a.g_fin.gx);
  if (a.shortv) {
    hipLaunchKernelGGL(k_dot2d<1>, gd, dim3(NT), 0, s, V, ld, k, (const double*)w, n, partial1, skip);
    GDC_TRY(check_launch("k_dot2d"));
    hipLaunchKernelGGL(k_axpy_dot<1>, ga, dim3(NT), 0, s, w, V, ld, k, partial1, n, h1, partial2, skip);
  } else {
    hipLaunchKernelGGL(k_dot2d<EPT_LONG>, gd, dim3(NT), 0, s, V, ld, k, (const double*)w, n, partial1, skip);
    GDC_TRY(check_launch("k_dot2d"));
    hipLaunchKernelGGL(k_axpy_dot<EPT_LONG>, ga, dim3(NT), 0, s, w, V, ld, k, partial1, n, h1, partial2, skip);
  }
  GDC_TRY(check_launch("k_axpy_dot"));
  hipLaunchKernelGGL(k_ortho_finish2<EPT_LONG>, gf, dim3(NT), 0, s, w, V, ld, k, partial2, a.nchunk, n, out, h2s,
                     st, m, (const double*)h1, hstat);
  return check_launch("k_ortho_finish2");
}

int arnoldi_fused(const ArnoldiArgs* dev_args, int ns, int shortv, const int* first_dot, int tot_dot,
                  const int* first_axpy, int tot_axpy, const int* first_fin, int tot_fin, hipStream_t s) {
  if (ns <= 0) return GDC_OK;
  if (shortv) {
    hipLaunchKernelGGL(k_dot2d_fused<1>, dim3(tot_dot), dim3(NT), 0, s, dev_args, first_dot, ns);
    GDC_TRY(check_launch("k_dot2d_fused"));
    hipLaunchKernelGGL(k_axpy_dot_fused<1>, dim3(tot_axpy), dim3(NT), 0, s, dev_args, first_axpy, ns);
  } else {
    hipLaunchKernelGGL(k_dot2d_fused<EPT_LONG>, dim3(tot_dot), dim3(NT), 0, s, dev_args, first_dot, ns);
    GDC_TRY(check_launch("k_dot2d_fused"));
    hipLaunchKernelGGL(k_axpy_dot_fused<EPT_LONG>, dim3(tot_axpy), dim3(NT), 0, s, dev_args, first_axpy, ns);
  }
  GDC_TRY(check_launch("k_axpy_dot_fused"));
  hipLaunchKernelGGL(k_ortho_finish2_fused<EPT_LONG>, dim3(tot_fin), dim3(NT), 0, s, dev_args, first_fin, ns);
  return check_launch("k_ortho_finish2_fused");
}


int gm_finish_cycle(GmresState* st, double* x, const double* V, long long ld, long long n, hipStream_t s) {
  hipLaunchKernelGGL(k_gm_update, dim3(grid_for(n)), dim3(NT), 0, s, x, V, ld, st, n);
  return check_launch("k_gm_update");
}

int scale_by_inv_sqrt(const double* w, const double* nrm2, double* out, long long n, hipStream_t s,
                      GmresState* cycle, double* zero, long long nzero) {
  hipLaunchKernelGGL(k_scale_inv_sqrt, dim3(grid_for(n > nzero ? n : nzero)), dim3(NT), 0, s, w, nrm2, out, n, cycle,
                     zero, nzero);
  return check_launch("k_scale_inv_sqrt");
}

int copy_scaled(const double* x, double a, double* y, long long n, hipStream_t s) {
  hipLaunchKernelGGL(k_copy_scaled, dim3(grid_for(n)), dim3(NT), 0, s, x, a, y, n);
  return check_launch("k_copy_scaled");
}

int sub_from(const double* b, double* w, long long n, hipStream_t s) {
  hipLaunchKernelGGL(k_sub_from, dim3(grid_for(n)), dim3(NT), 0, s, b, w, n);
  return check_launch("k_sub_from");
}

}  // namespace gdc
