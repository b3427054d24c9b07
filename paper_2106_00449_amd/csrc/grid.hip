// Gaussian spreading S and averaging J = S* between blobs and the grid
// (Sec. 4.2, eq. spreading and eq. averaging).
//
// Delta_i(x) = (2 pi sigma^2)^{-3/2} exp(-|x - r_i|^2 / 2 sigma^2), set to zero
// beyond the cutoff radius rc (minimum-image distance, no renormalisation), so
// J = dV S^T exactly.  One 64-wide wavefront handles one blob; its lanes walk
// the blob's stencil cube.  Positions arrive in FP64; each blob's offset to
// the first stencil point is formed in FP64 before any rounding to the grid
// precision, so an FP32 grid does not lose the position to the box size.
//
// interp_fd also returns, for NP small displacements dr of each blob, the
// differences J(r + dr) u - J(r) u needed by the finite-difference (or random
// finite-difference) divergence of step 3 of the gDC.  With dr ~ 1e-6 the
// difference would vanish in FP32 if formed from two averages, so it is summed
// directly from weight differences w' - w = w expm1((2 dr.d - |dr|^2)/2 sigma^2)
// (d = x_g - r), with the cutoff applied to both positions.

#include "gdc_internal.h"

namespace gdc {
namespace {

constexpr int NT = 256;
constexpr int WAVES = NT / 64;

template <typename R>
__device__ __forceinline__ R gexp(R x);
template <>
__device__ __forceinline__ float gexp<float>(float x) { return expf(x); }
template <>
__device__ __forceinline__ double gexp<double>(double x) { return exp(x); }

template <typename R>
__device__ __forceinline__ R gexpm1(R x);
template <>
__device__ __forceinline__ float gexpm1<float>(float x) { return expm1f(x); }
template <>
__device__ __forceinline__ double gexpm1<double>(double x) { return expm1(x); }

template <typename R>
__device__ __forceinline__ R wave_sum(R v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// First stencil index along each axis and the FP64 offset of that point
// from the wrapped blob position.  lo_shift = 0: ceil((r - rc)/dx), the first
// point that can be within rc, followed by P = floor(2 rc/dx) + 1 points;
// lo_shift = 1: one point further down and P + 2 points, so that positions
// displaced by |dr| < dx are covered too.
struct BlobBase {
  int g[3];      // first stencil index, wrapped into [0, n)
  double e[3];   // x_g - r of that point (FP64)
};

// A non-finite or absurdly large coordinate gets an offset that puts every
// stencil point outside the cutoff (the blob then touches no grid point); the
// wrapped base index keeps every access inside the grid whatever r is.
__device__ __forceinline__ BlobBase blob_base(const GridGeom& G, const double* r, int lo_shift) {
  BlobBase b;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const double rw = r[d] - G.L[d] * floor(r[d] / G.L[d]);
    if (!(rw > -G.L[d] && rw < 2.0 * G.L[d])) {
      b.g[d] = 0;
      b.e[d] = 1e300;
      continue;
    }
    const double gf = ceil((rw - G.rc) / G.dx[d]) - lo_shift;
    b.e[d] = gf * G.dx[d] - rw;
    int g = (int)gf % G.n[d];
    b.g[d] = g < 0 ? g + G.n[d] : g;
  }
  return b;
}

// Index of stencil point g + a (g in [0, n), 0 <= a <= n + 1).
__device__ __forceinline__ int wrap(int g, int n) {
  g -= (g >= n) ? n : 0;
  g -= (g >= n) ? n : 0;
  return g;
}

template <typename R>
__global__ __launch_bounds__(NT) void k_spread(GridGeom G, const double* __restrict__ r,
                                               const double* __restrict__ lam, R* __restrict__ f, int M) {
  const int blob = blockIdx.x * WAVES + threadIdx.x / 64;
  const int lane = threadIdx.x & 63;
  if (blob >= M) return;
  const BlobBase B = blob_base(G, r + 3LL * blob, 0);
  const R l0 = R(lam[3LL * blob]), l1 = R(lam[3LL * blob + 1]), l2 = R(lam[3LL * blob + 2]);
  const int P0 = G.P[0], P1 = G.P[1], P2 = G.P[2];
  const int PC = P0 * P1 * P2;
  const long long Gs = G.G;
  for (int l = lane; l < PC; l += 64) {
    const int a0 = l / (P1 * P2), rem = l - a0 * (P1 * P2);
    const int a1 = rem / P2, a2 = rem - a1 * P2;
    const double d0 = B.e[0] + a0 * G.dx[0], d1 = B.e[1] + a1 * G.dx[1], d2 = B.e[2] + a2 * G.dx[2];
    const double dd = d0 * d0 + d1 * d1 + d2 * d2;
    if (dd <= G.rc2) {
      const R w = R(G.wnorm) * gexp<R>(-R(dd) * R(G.inv2s2));
      const long long idx = ((long long)wrap(B.g[0] + a0, G.n[0]) * G.n[1] + wrap(B.g[1] + a1, G.n[1])) * G.n[2] +
                            wrap(B.g[2] + a2, G.n[2]);
      atomicAdd(f + idx, w * l0);
      atomicAdd(f + Gs + idx, w * l1);
      atomicAdd(f + 2 * Gs + idx, w * l2);
    }
  }
}

template <typename R>
__global__ __launch_bounds__(NT) void k_interp(GridGeom G, const double* __restrict__ r,
                                               const R* __restrict__ u, double* __restrict__ v, int M,
                                               double scale) {
  const int blob = blockIdx.x * WAVES + threadIdx.x / 64;
  const int lane = threadIdx.x & 63;
  if (blob >= M) return;
  const BlobBase B = blob_base(G, r + 3LL * blob, 0);
  const int P0 = G.P[0], P1 = G.P[1], P2 = G.P[2];
  const int PC = P0 * P1 * P2;
  const long long Gs = G.G;
  R s0 = 0, s1 = 0, s2 = 0;
  for (int l = lane; l < PC; l += 64) {
    const int a0 = l / (P1 * P2), rem = l - a0 * (P1 * P2);
    const int a1 = rem / P2, a2 = rem - a1 * P2;
    const double d0 = B.e[0] + a0 * G.dx[0], d1 = B.e[1] + a1 * G.dx[1], d2 = B.e[2] + a2 * G.dx[2];
    const double dd = d0 * d0 + d1 * d1 + d2 * d2;
    if (dd <= G.rc2) {
      const R w = R(G.wnorm) * gexp<R>(-R(dd) * R(G.inv2s2));
      const long long idx = ((long long)wrap(B.g[0] + a0, G.n[0]) * G.n[1] + wrap(B.g[1] + a1, G.n[1])) * G.n[2] +
                            wrap(B.g[2] + a2, G.n[2]);
      s0 += w * u[idx];
      s1 += w * u[Gs + idx];
      s2 += w * u[2 * Gs + idx];
    }
  }
  s0 = wave_sum(s0);
  s1 = wave_sum(s1);
  s2 = wave_sum(s2);
  if (lane == 0) {
    v[3LL * blob] = scale * (double)s0;
    v[3LL * blob + 1] = scale * (double)s1;
    v[3LL * blob + 2] = scale * (double)s2;
  }
}

template <typename R, int NP>
__global__ __launch_bounds__(NT) void k_interp_fd(GridGeom G, const double* __restrict__ r,
                                                  const double* __restrict__ dr, const R* __restrict__ u,
                                                  double* __restrict__ v, double* __restrict__ vd, int M) {
  const int blob = blockIdx.x * WAVES + threadIdx.x / 64;
  const int lane = threadIdx.x & 63;
  if (blob >= M) return;
  const BlobBase B = blob_base(G, r + 3LL * blob, 1);
  const int P0 = G.P[0] + 2, P1 = G.P[1] + 2, P2 = G.P[2] + 2;
  const int PC = P0 * P1 * P2;
  const long long Gs = G.G;
  double Dr[NP][3];
  double Dr2[NP];
#pragma unroll
  for (int k = 0; k < NP; ++k) {
#pragma unroll
    for (int d = 0; d < 3; ++d) Dr[k][d] = dr[(3LL * NP) * blob + 3 * k + d];
    Dr2[k] = Dr[k][0] * Dr[k][0] + Dr[k][1] * Dr[k][1] + Dr[k][2] * Dr[k][2];
  }
  const R wn = R(G.wnorm), i2 = R(G.inv2s2);
  R s[3] = {0, 0, 0};
  R sd[NP][3];
#pragma unroll
  for (int k = 0; k < NP; ++k) sd[k][0] = sd[k][1] = sd[k][2] = R(0);
  for (int l = lane; l < PC; l += 64) {
    const int a0 = l / (P1 * P2), rem = l - a0 * (P1 * P2);
    const int a1 = rem / P2, a2 = rem - a1 * P2;
    const double d0 = B.e[0] + a0 * G.dx[0], d1 = B.e[1] + a1 * G.dx[1], d2 = B.e[2] + a2 * G.dx[2];
    const double dd = d0 * d0 + d1 * d1 + d2 * d2;
    const bool in0 = dd <= G.rc2;
    bool any = in0;
    double ddp[NP];
#pragma unroll
    for (int k = 0; k < NP; ++k) {
      const double dot = Dr[k][0] * d0 + Dr[k][1] * d1 + Dr[k][2] * d2;
      ddp[k] = dd - 2.0 * dot + Dr2[k];
      any = any || (ddp[k] <= G.rc2);
    }
    if (!any) continue;
    const long long idx = ((long long)wrap(B.g[0] + a0, G.n[0]) * G.n[1] + wrap(B.g[1] + a1, G.n[1])) * G.n[2] +
                          wrap(B.g[2] + a2, G.n[2]);
    const R u0 = u[idx], u1 = u[Gs + idx], u2 = u[2 * Gs + idx];
    const R w = in0 ? wn * gexp<R>(-R(dd) * i2) : R(0);
    s[0] += w * u0;
    s[1] += w * u1;
    s[2] += w * u2;
#pragma unroll
    for (int k = 0; k < NP; ++k) {
      const bool in1 = ddp[k] <= G.rc2;
      R dw;
      if (in0 && in1) {
        const double dot = Dr[k][0] * d0 + Dr[k][1] * d1 + Dr[k][2] * d2;
        dw = w * gexpm1<R>(R(2.0 * dot - Dr2[k]) * i2);
      } else if (in0) {
        dw = -w;
      } else if (in1) {
        dw = wn * gexp<R>(-R(ddp[k]) * i2);
      } else {
        dw = R(0);
      }
      sd[k][0] += dw * u0;
      sd[k][1] += dw * u1;
      sd[k][2] += dw * u2;
    }
  }
  const double sc = G.dV;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const R t = wave_sum(s[c]);
    if (lane == 0) v[3LL * blob + c] = sc * (double)t;
  }
#pragma unroll
  for (int k = 0; k < NP; ++k) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const R t = wave_sum(sd[k][c]);
      if (lane == 0) vd[(3LL * NP) * blob + 3 * k + c] = sc * (double)t;
    }
  }
}

__global__ void k_fill_zero(uint4* __restrict__ p, long long n16) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long k = i; k < n16; k += stride) p[k] = make_uint4(0u, 0u, 0u, 0u);
}

__global__ void k_widen(const float* __restrict__ x, double* __restrict__ y, long long n) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) y[e] = (double)x[e];
}

inline unsigned blocks_for(int M) { return (unsigned)((M + WAVES - 1) / WAVES); }

}  // namespace

int fill_zero(void* p, size_t bytes, hipStream_t s) {
  if (bytes == 0) return GDC_OK;
  if (bytes % 16 != 0 || (reinterpret_cast<uintptr_t>(p) & 15) != 0) {
    set_error("fill_zero: size and address must be 16-byte aligned");
    return GDC_EINVAL;
  }
  const long long n16 = (long long)(bytes / 16);
  const long long want = (n16 + 255) / 256;
  const unsigned blocks = (unsigned)(want < 8192 ? want : 8192);
  hipLaunchKernelGGL(k_fill_zero, dim3(blocks), dim3(256), 0, s, (uint4*)p, n16);
  return check_launch("k_fill_zero");
}

int widen(const float* x, double* y, long long n, hipStream_t s) {
  const long long want = (n + 255) / 256;
  hipLaunchKernelGGL(k_widen, dim3((unsigned)(want < 8192 ? (want > 0 ? want : 1) : 8192)), dim3(256), 0, s, x, y, n);
  return check_launch("k_widen");
}

template <typename R>
int spread(const GridGeom& g, const double* r, const double* lam, R* f, int M, hipStream_t s) {
  if (M <= 0) return GDC_OK;
  hipLaunchKernelGGL((k_spread<R>), dim3(blocks_for(M)), dim3(NT), 0, s, g, r, lam, f, M);
  return check_launch("k_spread");
}

template <typename R>
int interp(const GridGeom& g, const double* r, const R* u, double* v, int M, double scale,
           hipStream_t s) {
  if (M <= 0) return GDC_OK;
  hipLaunchKernelGGL((k_interp<R>), dim3(blocks_for(M)), dim3(NT), 0, s, g, r, u, v, M, scale);
  return check_launch("k_interp");
}

template <typename R>
int interp_fd(const GridGeom& g, const double* r, const double* dr, int NP, const R* u,
              double* v, double* vd, int M, hipStream_t s) {
  if (M <= 0) return GDC_OK;
  switch (NP) {
    case 1:
      hipLaunchKernelGGL((k_interp_fd<R, 1>), dim3(blocks_for(M)), dim3(NT), 0, s, g, r, dr, u, v, vd, M);
      break;
    case 6:
      hipLaunchKernelGGL((k_interp_fd<R, 6>), dim3(blocks_for(M)), dim3(NT), 0, s, g, r, dr, u, v, vd, M);
      break;
    default:
      set_error("interp_fd: NP must be 1 or 6");
      return GDC_EINVAL;
  }
  return check_launch("k_interp_fd");
}

template int spread<float>(const GridGeom&, const double*, const double*, float*, int, hipStream_t);
template int spread<double>(const GridGeom&, const double*, const double*, double*, int, hipStream_t);
template int interp<float>(const GridGeom&, const double*, const float*, double*, int, double, hipStream_t);
template int interp<double>(const GridGeom&, const double*, const double*, double*, int, double, hipStream_t);
template int interp_fd<float>(const GridGeom&, const double*, const double*, int, const float*, double*,
                              double*, int, hipStream_t);
template int interp_fd<double>(const GridGeom&, const double*, const double*, int, const double*, double*,
                               double*, int, hipStream_t);

}  // namespace gdc
