// Krylov vector kernels for the device-resident GMRES of the saddle problem
// (Sec. 2.2).  Vectors are FP64 and live in one basis array V[(m+1) x ld].
// Dot products are two-stage (fixed-order partial sums per block, then one
// block per result), so a solve is reproducible run to run.

#include "gdc_internal.h"

namespace gdc {
namespace {

constexpr int NT = 256;
constexpr int MAXK = 64;   // vectors per multi-dot launch

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

// partial[j * nblk + block] = sum over the block's slice of V_j . w, j < k.
__global__ __launch_bounds__(NT) void k_multi_dot_partial(const double* __restrict__ V, long long ld, int k,
                                                          const double* __restrict__ w, long long n,
                                                          double* __restrict__ partial) {
  __shared__ double sh[NT / 64];
  const long long chunk = (n + gridDim.x - 1) / gridDim.x;
  const long long lo = chunk * blockIdx.x;
  const long long hi = min(n, lo + chunk);
  for (int j = 0; j < k; ++j) {
    const double* v = V + ld * j;
    double s = 0.0;
    for (long long e = lo + threadIdx.x; e < hi; e += NT) s += v[e] * w[e];
    const double t = block_sum(s, sh);
    if (threadIdx.x == 0) partial[(long long)j * gridDim.x + blockIdx.x] = t;
  }
}

__global__ __launch_bounds__(NT) void k_multi_dot_final(const double* __restrict__ partial, int nblk,
                                                        double* __restrict__ h) {
  __shared__ double sh[NT / 64];
  const int j = blockIdx.x;
  double s = 0.0;
  for (int b = threadIdx.x; b < nblk; b += NT) s += partial[(long long)j * nblk + b];
  const double t = block_sum(s, sh);
  if (threadIdx.x == 0) h[j] = t;
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

__global__ void k_scale_inv_sqrt(const double* __restrict__ w, const double* __restrict__ nrm2,
                                 double* __restrict__ out, long long n) {
  const double a = nrm2[0] > 0.0 ? 1.0 / sqrt(nrm2[0]) : 0.0;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) out[e] = a * w[e];
}

__global__ void k_copy_scaled(const double* __restrict__ x, double a, double* __restrict__ y, long long n) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) y[e] = a * x[e];
}

__global__ void k_sub_from(const double* __restrict__ b, double* __restrict__ w, long long n) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) w[e] = b[e] - w[e];
}

inline unsigned grid_for(long long n) {
  const long long b = (n + NT - 1) / NT;
  return (unsigned)(b < 2048 ? (b > 0 ? b : 1) : 2048);
}

}  // namespace

int multi_dot(const double* V, long long ld, int k, const double* w, long long n, double* partial, int nblk,
              double* h, hipStream_t s) {
  if (k <= 0) return GDC_OK;
  hipLaunchKernelGGL(k_multi_dot_partial, dim3(nblk), dim3(NT), 0, s, V, ld, k, w, n, partial);
  GDC_TRY(check_launch("k_multi_dot_partial"));
  hipLaunchKernelGGL(k_multi_dot_final, dim3(k), dim3(NT), 0, s, partial, nblk, h);
  return check_launch("k_multi_dot_final");
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

int scale_by_inv_sqrt(const double* w, const double* nrm2, double* out, long long n, hipStream_t s) {
  hipLaunchKernelGGL(k_scale_inv_sqrt, dim3(grid_for(n)), dim3(NT), 0, s, w, nrm2, out, n);
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
