// Gaussian spreading S and averaging J = S* between blobs and the grid
// (Sec. 4.2, eq. spreading and eq. averaging).
//
// Delta_i(x) = (2 pi sigma^2)^{-3/2} exp(-|x - r_i|^2 / 2 sigma^2), set to zero
// beyond the cutoff radius rc (minimum-image distance, no renormalisation), so
// J = dV S^T exactly.  Averaging: one 64-wide wavefront per blob walks the
// blob's stencil.  Spreading: one workgroup per grid tile gathers the blobs
// that reach it (k_spread_tab).  Positions arrive in FP64; each blob's offset to
// the first stencil point is formed in FP64 before any rounding to the grid
// precision, so an FP32 grid does not lose the position to the box size.
//
// interp_fd also returns, for NP small displacements dr of each blob, the
// differences J(r + dr) u - J(r) u needed by the finite-difference (or random
// finite-difference) divergence of step 3 of the gDC.  With dr ~ 1e-6 the
// difference would vanish in FP32 if formed from two averages, so it is summed
// directly from weight differences w' - w = w expm1((2 dr.d - |dr|^2)/2 sigma^2)
// (d = x_g - r), with the cutoff applied to both positions.

#include <hip/hip_ext.h>

#include "gdc_internal.h"

#include <algorithm>

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

// e^x - 1 for the small arguments of the finite-difference weights
// (|x| ~ 1e-4 at the default displacement): the Taylor series
// x + x^2/2 + x^3/6 + x^4/24 (Horner), whose truncation error x^5/120 is
// below FP32 rounding for |x| < 2^-7 and below FP64 rounding for
// |x| < 2^-12; larger arguments take the library function.
template <typename R>
__device__ __forceinline__ R small_expm1(R x) {
  constexpr R lim = sizeof(R) == 4 ? R(0.0078125) : R(0.000244140625);
  if (fabs(x) >= lim) return gexpm1<R>(x);
  return x * (R(1) + x * (R(0.5) + x * (R(1) / R(6) + x * (R(1) / R(24)))));
}

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

// Workgroups are handed to the 8 XCDs (each with its own L2) round-robin by
// block index.  The averaging kernels remap the block index so that XCD x
// takes a contiguous run of blobs (whole bodies: blobs are numbered body by
// body), which keeps the overlapping stencils of a body's blobs in one L2.
// The grid is padded to a multiple of 8 blocks; blocks past the end return.
constexpr int NXCD = 8;
__device__ __forceinline__ int xcd_block(int nb_padded) {
  const int per = nb_padded / NXCD;
  return (int)(blockIdx.x % NXCD) * per + (int)(blockIdx.x / NXCD);
}
__device__ __forceinline__ int xcd_block(const BlockIx& bi) {
  const int per = bi.gx / NXCD;
  return (bi.x % NXCD) * per + bi.x / NXCD;
}

// Index of stencil point g + a (g in [0, n), 0 <= a <= n + 1).
__device__ __forceinline__ int wrap(int g, int n) {
  g -= (g >= n) ? n : 0;
  g -= (g >= n) ? n : 0;
  return g;
}

// Loads of one field component through a buffer resource: the component's
// base and size sit in scalar registers and each load takes a 32-bit byte
// offset.  chunk(i) returns the 16 bytes at grid index i (CW consecutive
// points along axis 2; i a multiple of CW), one load instruction for four
// FP32 or two FP64 values.
constexpr int BUF_DWORD3 = 0x00020000;   // raw loads on gfx9-family parts

template <typename R>
struct Component;
template <>
struct Component<float> {
  static constexpr int CW = 4;
  __amdgpu_buffer_rsrc_t rs;
  __device__ Component(const float* p, long long n)
      : rs(__builtin_amdgcn_make_buffer_rsrc((void*)p, (short)0, (int)(n * 4), BUF_DWORD3)) {}
  __device__ void chunk(unsigned i, float* x) const {
    const float4 v = __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(rs, (int)(i * 4u), 0, 0));
    x[0] = v.x;
    x[1] = v.y;
    x[2] = v.z;
    x[3] = v.w;
  }
};
template <>
struct Component<double> {
  static constexpr int CW = 2;
  __amdgpu_buffer_rsrc_t rs;
  __device__ Component(const double* p, long long n)
      : rs(__builtin_amdgcn_make_buffer_rsrc((void*)p, (short)0, (int)(n * 8), BUF_DWORD3)) {}
  __device__ void chunk(unsigned i, double* x) const {
    const double2 v = __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(rs, (int)(i * 8u), 0, 0));
    x[0] = v.x;
    x[1] = v.y;
  }
};

// Stencil walk in chunks: the P2 points of each (a0, a1) row of the stencil
// lie in nck aligned chunks of CW points along axis 2 (the field is
// contiguous along axis 2 in runs of 32 points, and every grid size is a
// multiple of 4), and lane tasks are (a0, a1, chunk): one 16-byte load per
// component and task.  Rows outside the cutoff sphere are skipped.  Loads,
// not bytes, bound a gather of scattered short runs, so fewer and wider
// loads are what shortens it.

// A blob's record in the tile-sorted order: the FP64 offsets and grid index
// (10 bits per axis) of its first stencil point, as blob_base gives them, and
// the blob index.
struct SRec {
  double e[3];
  int g;
  int blob;
};

// Rigid-body term subtracted by the averaging epilogue of the saddle operator:
// U_p + Omega_p x (r_i - Y_p) for blob i of body p.
struct RigidTerm {
  const int* blob_body;   // M
  const double* Y;        // N x 3
  const double* V;        // N x 6 (U, Omega); null: no rigid term
};

// With rec (the tile-sorted records of the same positions), wave p takes the
// blob at sorted place p, so that each XCD's run of blobs is a compact region
// of the box and the stencils it reads stay in that XCD's L2; the arithmetic
// of each blob is unchanged.
template <typename R>
__device__ __forceinline__ void interp_body(const GridGeom& G, const double* __restrict__ r,
                                            const R* __restrict__ u, double* __restrict__ v, int M, double scale,
                                            const RigidTerm& K, const int* __restrict__ skip,
                                            const SRec* __restrict__ rec, const BlockIx& bi) {
  if (skip && *skip) return;
  // wave-uniform by construction; readfirstlane tells the compiler, so the
  // blob's record and body data come through scalar loads
  const int place = xcd_block(bi) * WAVES + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (place >= M) return;
  int blob;
  BlobBase B;
  if (rec) {
    const SRec x = rec[place];
    blob = x.blob;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      B.e[d] = x.e[d];
      B.g[d] = (x.g >> (10 * d)) & 1023;
    }
  } else {
    blob = place;
    B = blob_base(G, r + 3LL * blob, 0);
  }
  // the rigid velocity of the blob's body at the blob (K V), loaded here,
  // uniform per wave, so the loads overlap the gather instead of following it
  double kvel[3] = {0.0, 0.0, 0.0};
  if (K.V) {
    const int p = K.blob_body[blob];
    const double* Vp = K.V + 6LL * p;
    const double rel[3] = {r[3LL * blob] - K.Y[3LL * p], r[3LL * blob + 1] - K.Y[3LL * p + 1],
                           r[3LL * blob + 2] - K.Y[3LL * p + 2]};
    kvel[0] = Vp[0] + (Vp[4] * rel[2] - Vp[5] * rel[1]);
    kvel[1] = Vp[1] + (Vp[5] * rel[0] - Vp[3] * rel[2]);
    kvel[2] = Vp[2] + (Vp[3] * rel[1] - Vp[4] * rel[0]);
  }
  const int P0 = G.P[0], P1 = G.P[1], P2 = G.P[2];
  const Component<R> u0(u, G.G), u1(u + G.G, G.G), u2(u + 2 * G.G, G.G);
  const int n0 = G.n[0], n1 = G.n[1], n2 = G.n[2];
  const R wn = R(G.wnorm), i2 = R(G.inv2s2);
  constexpr int CW = Component<R>::CW;
  const int first2 = B.g[2] & ~(CW - 1);   // aligned chunk holding the first point
  const int skew = B.g[2] - first2;
  const int nck = (skew + P2 - 1) / CW + 1;
  const int per0 = P1 * nck;
  // The axis-2 factors of the blob, one per entry i = a2 + skew of its
  // nck CW points along axis 2 (lane i computes entry i): the squared
  // distance d2^2 (FP64; +inf outside the stencil) and exp(-d2^2 / 2 sigma^2).
  // The weight of a point is then wn exp(-(d0^2 + d1^2) / 2 sigma^2) times
  // its entry's factor, one exponential per task instead of one per point.
  __shared__ __align__(16) double q2s[WAVES][64];
  __shared__ __align__(16) R e2s[WAVES][64];
  const int wv_ix = threadIdx.x >> 6;
  {
    const int a2 = lane - skew;
    double q = __builtin_huge_val();
    R f = R(0);
    if (a2 >= 0 && a2 < P2) {
      const double d2 = B.e[2] + a2 * G.dx[2];
      q = d2 * d2;
      f = gexp<R>(-R(q) * i2);
    }
    q2s[wv_ix][lane] = q;
    e2s[wv_ix][lane] = f;
  }
  __builtin_amdgcn_wave_barrier();
  // tasks (a0, a1, c) by the reciprocals of per0 and nck: the exact quotient
  // of task + 1/2 lies at least 1/(2 per0) from an integer, far beyond FP32
  // rounding at these sizes
  const float rp0 = 1.0f / (float)per0, rnck = 1.0f / (float)nck;
  R s0 = 0, s1 = 0, s2 = 0;
  for (int task = lane; task < P0 * per0; task += 64) {
    const int a0 = (int)(((float)task + 0.5f) * rp0), rem = task - a0 * per0;
    const int a1 = (int)(((float)rem + 0.5f) * rnck), c = rem - a1 * nck;
    const double d0 = B.e[0] + a0 * G.dx[0], d1 = B.e[1] + a1 * G.dx[1];
    const double d01 = d0 * d0 + d1 * d1;
    if (d01 > G.rc2) continue;         // the row misses the cutoff sphere
    int c2 = first2 + c * CW;          // below 2 n2: first2 < n2, c CW < CW + P2 - 1
    c2 -= (c2 >= n2) ? n2 : 0;
    const unsigned ix = (unsigned)(field_plane_off(G.tiled, n1, n2, wrap(B.g[0] + a0, n0)) +
                                   field_col_off(G.tiled, n2, wrap(B.g[1] + a1, n1), c2));
    R x0[CW], x1[CW], x2[CW];
    u0.chunk(ix, x0);
    u1.chunk(ix, x1);
    u2.chunk(ix, x2);
    const R e01 = wn * gexp<R>(-R(d01) * i2);
#pragma unroll
    for (int j = 0; j < CW; ++j) {
      const int i = c * CW + j;
      const bool ok = d01 + q2s[wv_ix][i] <= G.rc2;
      const R wv = ok ? e01 * e2s[wv_ix][i] : R(0);
      s0 += wv * x0[j];
      s1 += wv * x1[j];
      s2 += wv * x2[j];
    }
  }
  s0 = wave_sum(s0);
  s1 = wave_sum(s1);
  s2 = wave_sum(s2);
  if (lane == 0) {
    double o[3] = {scale * (double)s0, scale * (double)s1, scale * (double)s2};
    if (K.V) {
      o[0] -= kvel[0];
      o[1] -= kvel[1];
      o[2] -= kvel[2];
    }
    v[3LL * blob] = o[0];
    v[3LL * blob + 1] = o[1];
    v[3LL * blob + 2] = o[2];
  }
}

template <typename R>
__global__ __launch_bounds__(NT) void k_interp(GridGeom G, const double* __restrict__ r,
                                               const R* __restrict__ u, double* __restrict__ v, int M,
                                               double scale, RigidTerm K, const int* __restrict__ skip,
                                               const SRec* __restrict__ rec) {
  interp_body<R>(G, r, u, v, M, scale, K, skip, rec, hw_block());
}

// Averaging fused over several suspensions (one InterpArgs each).
template <typename R>
__global__ __launch_bounds__(NT) void k_interp_fused(const InterpArgs* __restrict__ a,
                                                     const int* __restrict__ first, int ns) {
  const int sidx = fused_suspension(first, ns, blockIdx.x);
  const InterpArgs& A = a[sidx];
  const RigidTerm K{A.blob_body, A.Y, A.V};
  interp_body<R>(A.G, A.r, (const R*)A.u, A.v, A.M, A.scale, K, A.skip, (const SRec*)A.rec,
                 fused_block(A.grid, (int)blockIdx.x - first[sidx]));
}

template <typename R, int NP>
__global__ __launch_bounds__(NT) void k_interp_fd(GridGeom G, const double* __restrict__ r,
                                                  const double* __restrict__ dr, const R* __restrict__ u,
                                                  double* __restrict__ v, double* __restrict__ vd, int M) {
  const int blob = xcd_block(gridDim.x) * WAVES + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (blob >= M) return;
  const BlobBase B = blob_base(G, r + 3LL * blob, 1);
  const int P0 = G.P[0] + 2, P1 = G.P[1] + 2, P2 = G.P[2] + 2;
  const long long Gs = G.G;
  const int n0 = G.n[0], n1 = G.n[1], n2 = G.n[2];
  double Dr[NP][3];
  double Dr2[NP];
#pragma unroll
  for (int k = 0; k < NP; ++k) {
#pragma unroll
    for (int d = 0; d < 3; ++d) Dr[k][d] = dr[(3LL * NP) * blob + 3 * k + d];
    Dr2[k] = Dr[k][0] * Dr[k][0] + Dr[k][1] * Dr[k][1] + Dr[k][2] * Dr[k][2];
  }
  // a point can matter only within rc + max |dr| of the blob
  double drmax2 = 0.0;
#pragma unroll
  for (int k = 0; k < NP; ++k) drmax2 = fmax(drmax2, Dr2[k]);
  const double reach = G.rc + sqrt(drmax2);
  const double reach2 = reach * reach;
  const R wn = R(G.wnorm), i2 = R(G.inv2s2);
  R s[3] = {0, 0, 0};
  R sd[NP][3];
#pragma unroll
  for (int k = 0; k < NP; ++k) sd[k][0] = sd[k][1] = sd[k][2] = R(0);
  for (int pr = lane; pr < P1 * P2; pr += 64) {
    const int a1 = pr / P2, a2 = pr - a1 * P2;
    const double d1 = B.e[1] + a1 * G.dx[1], d2 = B.e[2] + a2 * G.dx[2];
    const double d12 = d1 * d1 + d2 * d2;
    if (d12 > reach2) continue;
    const long long col = field_col_off(G.tiled, n2, wrap(B.g[1] + a1, n1), wrap(B.g[2] + a2, n2));
    int g0 = B.g[0];
    for (int a0 = 0; a0 < P0; ++a0, g0 = (g0 + 1 == n0) ? 0 : g0 + 1) {
      const double d0 = B.e[0] + a0 * G.dx[0];
      const double dd = d0 * d0 + d12;
      if (dd > reach2) continue;
      const bool in0 = dd <= G.rc2;
      const long long idx = field_plane_off(G.tiled, n1, n2, g0) + col;
      const R u0 = u[idx], u1 = u[Gs + idx], u2 = u[2 * Gs + idx];
      const R w = in0 ? wn * gexp<R>(-R(dd) * i2) : R(0);
      s[0] += w * u0;
      s[1] += w * u1;
      s[2] += w * u2;
#pragma unroll
      for (int k = 0; k < NP; ++k) {
        const double dot = Dr[k][0] * d0 + Dr[k][1] * d1 + Dr[k][2] * d2;
        const double ddp = dd - 2.0 * dot + Dr2[k];
        const bool in1 = ddp <= G.rc2;
        R dw;
        if (in0 && in1)
          dw = w * small_expm1<R>(R(2.0 * dot - Dr2[k]) * i2);
        else if (in0)
          dw = -w;
        else if (in1)
          dw = wn * gexp<R>(-R(ddp) * i2);
        else
          dw = R(0);
        sd[k][0] += dw * u0;
        sd[k][1] += dw * u1;
        sd[k][2] += dw * u2;
      }
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

// ------------------------------------------------------------ tiled spreading
// The grid is cut into tiles of T0 x T1 x T2 points.  Blobs are counting-sorted
// by the tile of their anchor point floor(r/dx); a workgroup owns one tile,
// collects the blobs of the neighbouring tiles whose stencils reach it,
// accumulates their Gaussians in LDS (LDS atomics only) and writes the tile
// once: no global atomics and no zero fill of the field.

__device__ __forceinline__ int tile_of_blob(const GridGeom& G, const TileGeom& T, const double* r) {
  int t[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const double rw = r[d] - G.L[d] * floor(r[d] / G.L[d]);
    const double c = floor(rw / G.dx[d]);
    int ci = (c >= 0.0 && c < (double)G.n[d]) ? (int)c : 0;
    t[d] = ci / T.T[d];
  }
  return (t[0] * T.nt[1] + t[1]) * T.nt[2] + t[2];
}

__global__ void k_tile_count(GridGeom G, TileGeom T, const double* __restrict__ r, int M, int* __restrict__ tile,
                             int* __restrict__ count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= M) return;
  const int t = tile_of_blob(G, T, r + 3LL * i);
  tile[i] = t;
  atomicAdd(count + t, 1);
}

// Exclusive scan of count[0..n) into off[0..n], one block.
__global__ __launch_bounds__(1024) void k_tile_scan(const int* __restrict__ count, int n, int* __restrict__ off,
                                                    int* __restrict__ cursor) {
  __shared__ int sh[1024];
  __shared__ int carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int base = 0; base < n; base += 1024) {
    const int i = base + threadIdx.x;
    const int x = i < n ? count[i] : 0;
    sh[threadIdx.x] = x;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
      const int y = threadIdx.x >= (unsigned)o ? sh[threadIdx.x - o] : 0;
      __syncthreads();
      sh[threadIdx.x] += y;
      __syncthreads();
    }
    if (i < n) {
      off[i] = carry + sh[threadIdx.x] - x;
      cursor[i] = carry + sh[threadIdx.x] - x;
    }
    __syncthreads();
    if (threadIdx.x == 1023) carry += sh[1023];
    __syncthreads();
  }
  if (threadIdx.x == 0) off[n] = carry;
}

// Sorted blob record: offset of the first stencil point (FP64), its wrapped
// grid index packed 10 bits per axis, and the blob's index.
__global__ void k_tile_scatter(GridGeom G, const double* __restrict__ r, const int* __restrict__ tile, int M,
                               int* __restrict__ cursor, SRec* __restrict__ rec) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= M) return;
  const BlobBase B = blob_base(G, r + 3LL * i, 0);
  SRec x;
  x.e[0] = B.e[0];
  x.e[1] = B.e[1];
  x.e[2] = B.e[2];
  x.g = B.g[0] | (B.g[1] << 10) | (B.g[2] << 20);
  x.blob = i;
  rec[atomicAdd(cursor + tile[i], 1)] = x;
}

// Within each tile, records ordered by blob index, so that every sum over a
// tile's blobs has a fixed order: one wave per tile; a record's place is the
// number of records of its tile with a smaller blob index (indices are
// distinct), counted against the tile's indices staged 64 at a time in LDS.
__global__ __launch_bounds__(256) void k_tile_rank(const int* __restrict__ off, int ntiles,
                                                   const SRec* __restrict__ in, SRec* __restrict__ out,
                                                   int* __restrict__ spos) {
  __shared__ int idx[4][64];
  const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int t = blockIdx.x * 4 + w;
  if (t >= ntiles) return;   // whole wave leaves together; no block barrier below
  const int lo = off[t], hi = off[t + 1];
  if (hi - lo <= 64) {
    // the usual case: the tile's records fit one wave, ranked from the
    // blob indices the lanes already hold
    const int i = lo + lane;
    SRec x;
    int b = 0x7fffffff;
    if (i < hi) {
      x = in[i];
      b = x.blob;
    }
    idx[w][lane] = b;
    __builtin_amdgcn_wave_barrier();
    int rank = 0;
    const int cnt = hi - lo;
    for (int k = 0; k < cnt; ++k) rank += idx[w][k] < b;
    if (i < hi) {
      out[lo + rank] = x;
      spos[b] = lo + rank;
    }
    return;
  }
  for (int i0 = lo; i0 < hi; i0 += 64) {
    const int i = i0 + lane;
    SRec x;
    int b = 0x7fffffff;
    if (i < hi) {
      x = in[i];
      b = x.blob;
    }
    int rank = 0;
    for (int j0 = lo; j0 < hi; j0 += 64) {
      const int j = j0 + lane;
      idx[w][lane] = j < hi ? in[j].blob : 0x7fffffff;
      __builtin_amdgcn_wave_barrier();
      const int cnt = min(64, hi - j0);
      for (int k = 0; k < cnt; ++k) rank += idx[w][k] < b;
      __builtin_amdgcn_wave_barrier();
    }
    if (i < hi) {
      out[lo + rank] = x;
      spos[b] = lo + rank;
    }
  }
}

// Offsets j in [0, Teff) of a tile that a blob's stencil reaches along one
// axis, as up to two ranges: stencil offset a = u + j (first range) or
// u + j - n (second), u = (tile start - first stencil index) mod n.
struct Ranges {
  int s1, l1, s2, l2;
};

__device__ __forceinline__ Ranges axis_ranges(int g, int tstart, int Teff, int n, int P) {
  int u = tstart - g;
  u += (u < 0) ? n : 0;
  Ranges R;
  R.s1 = 0;
  R.l1 = (u < P) ? min(Teff, P - u) : 0;
  R.s2 = n - u;
  R.l2 = (n - u < Teff) ? min(Teff, n - u + P) - (n - u) : 0;
  if (R.l2 < 0) R.l2 = 0;
  return R;
}

// ------------------------------------------------------------ spreading
// The blobs whose stencil box meets a grid tile (8 x 8 x 32 points) are its
// "hits".  The truncated Gaussian is separable, w = wnorm e0(d0) e1(d1)
// e2(d2) with the cut d0^2 + d1^2 + d2^2 <= rc^2, so each hit carries
// per-axis tables over the tile's coordinates: factor and squared distance,
// zero and a large value off the stencil.  The tables depend on positions
// only, so k_spread_prep builds them once per configuration and every
// spread S lambda at that configuration (one per GMRES iteration) reads
// them back: gather the forces, accumulate, write the tile.

// Axis 2 keeps a window of WZ entries from tile offset zlo: WZ = 8 when a
// stencil spans at most 8 points and a tile never holds both ends of the
// axis (then the hit's points along axis 2 are one run of at most 8), else
// the whole 32-point tile (zlo = 0).
template <typename R, int WZ>
struct HitTab {
  R f0[8], s0[8];      // axis 0 (f0 carries wnorm)
  R f1[8], s1[8];      // axis 1
  R fz[WZ], sz[WZ];    // axis 2, tile offsets zlo .. zlo + WZ - 1
  int mask;            // bits 0-3: z-chunks the hit reaches; bits 8-15: axis-0 planes
  int pos;             // record position (index into the sorted order)
  int blob;
  int zlo;
};
static_assert(sizeof(HitTab<float, 8>) % 16 == 0 && sizeof(HitTab<double, 8>) % 16 == 0 &&
              sizeof(HitTab<float, 32>) % 16 == 0 && sizeof(HitTab<double, 32>) % 16 == 0, "16-byte rows");

// First tile offset along axis 2 of a hit's stencil run (origin g2 of an
// n2-point axis, tile start ts2, stencil of P2 points).
__device__ __forceinline__ int hit_zlo(int g2, int ts2, int n2, int P2) {
  int u = ts2 - g2;
  u += (u < 0) ? n2 : 0;
  return u < P2 ? 0 : n2 - u;
}

// Candidates of a tile: the records of the (up to 5 x 5 x 5) neighbour tiles
// whose anchored blobs can reach it, in neighbour order.
struct TileFrame {
  int ts[3], te[3];
  int nnb;
};

__device__ __forceinline__ TileFrame tile_frame(const GridGeom& G, const TileGeom& T, int tl, const int* off,
                                                int* nb_base, int* nb_pref) {
  TileFrame F;
  const int t2 = tl % T.nt[2], t1 = (tl / T.nt[2]) % T.nt[1], t0 = tl / (T.nt[1] * T.nt[2]);
  const int tt[3] = {t0, t1, t2};
  int c[3], st[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    F.ts[d] = tt[d] * T.T[d];
    F.te[d] = min(T.T[d], G.n[d] - F.ts[d]);
    c[d] = min(2 * T.H[d] + 1, T.nt[d]);
    st[d] = (c[d] == T.nt[d]) ? 0 : tt[d] - T.H[d];
  }
  F.nnb = c[0] * c[1] * c[2];
  const int tid = threadIdx.x;
  if (tid < F.nnb) {
    const int i2 = tid % c[2], i1 = (tid / c[2]) % c[1], i0 = tid / (c[1] * c[2]);
    const int a0 = ((st[0] + i0) % T.nt[0] + T.nt[0]) % T.nt[0];
    const int a1 = ((st[1] + i1) % T.nt[1] + T.nt[1]) % T.nt[1];
    const int a2 = ((st[2] + i2) % T.nt[2] + T.nt[2]) % T.nt[2];
    const int nt = (a0 * T.nt[1] + a1) * T.nt[2] + a2;
    nb_base[tid] = off[nt];
    nb_pref[tid + 1] = off[nt + 1] - off[nt];
  }
  __syncthreads();
  if (tid == 0) {
    nb_pref[0] = 0;
    for (int k = 1; k <= F.nnb; ++k) nb_pref[k] += nb_pref[k - 1];
  }
  __syncthreads();
  return F;
}

// Candidate ci: its record position, and whether its stencil box meets the
// tile (with the z-chunk / axis-0-plane mask).
__device__ __forceinline__ bool tile_candidate(const GridGeom& G, const TileFrame& F, const SRec* __restrict__ rec,
                                               const int* nb_base, const int* nb_pref, int ci, int& pos, int& mask,
                                               SRec& x) {
  int lo = 0, hi = F.nnb;   // neighbour tile with nb_pref[lo] <= ci < nb_pref[lo + 1]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (nb_pref[mid] <= ci) lo = mid; else hi = mid;
  }
  pos = nb_base[lo] + (ci - nb_pref[lo]);
  x = rec[pos];
  const int gb[3] = {x.g & 1023, (x.g >> 10) & 1023, (x.g >> 20) & 1023};
  bool hit = true;
  mask = 0;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const Ranges Rg = axis_ranges(gb[d], F.ts[d], F.te[d], G.n[d], G.P[d]);
    hit = hit && (Rg.l1 + Rg.l2 > 0);
    if (d == 0) {
      // axis-0 planes [s1, s1 + l1) and [s2, s2 + l2) of the tile
      const int m1 = Rg.l1 > 0 ? ((1 << Rg.l1) - 1) << Rg.s1 : 0;
      const int m2 = Rg.l2 > 0 ? ((1 << Rg.l2) - 1) << Rg.s2 : 0;
      mask |= (m1 | m2) << 8;
    } else if (d == 2) {
      // z-chunks covered by [s1, s1 + l1) and [s2, s2 + l2)
      if (Rg.l1 > 0)
        for (int q = Rg.s1 >> 3; q <= (Rg.s1 + Rg.l1 - 1) >> 3; ++q) mask |= 1 << q;
      if (Rg.l2 > 0)
        for (int q = Rg.s2 >> 3; q <= (Rg.s2 + Rg.l2 - 1) >> 3; ++q) mask |= 1 << q;
    }
  }
  return hit;
}

// One axis of the tables of hits [0, nr) (origin offsets he, packed origins
// hg) into out[h]: for tile offset j < W along axis D, the stencil offset
// a = (ts + j - g) mod n; inside the stencil (a < P, j < te) the factor
// exp(-d^2 / 2 sigma^2) (axis 0 also carries wnorm) and d^2, else 0 and
// `big`.  The axis is a compile-time constant (a runtime index into the
// kernel-argument struct would be a memory load per entry).
template <typename R, int D, int WZ>
__device__ __forceinline__ void table_axis(const GridGeom& G, const TileFrame& F, int nr, const double (*he)[3],
                                           const int* hg, HitTab<R, WZ>* out, R big) {
  constexpr int W = D == 2 ? WZ : 8, LW = D == 2 ? (WZ == 32 ? 5 : 3) : 3;
  const int n = G.n[D], P = G.P[D];
  const double dx = G.dx[D], i2 = G.inv2s2, wn = G.wnorm;
  for (int e = threadIdx.x; e < nr * W; e += NT) {
    const int h = e >> LW, jw = e & (W - 1);
    const int gb = (hg[h] >> (10 * D)) & 1023;
    const int j = (D == 2 && WZ != 32) ? hit_zlo(gb, F.ts[2], n, P) + jw : jw;   // tile offset
    int a = F.ts[D] + j - gb;
    a += (a < 0) ? n : 0;
    a -= (a >= n) ? n : 0;
    R fv = R(0), sv = big;
    if (j < F.te[D] && a < P) {
      const double dd = he[h][D] + a * dx;
      const double s2 = dd * dd;
      sv = R(s2);
      fv = gexp<R>(R(-s2 * i2));
      if (D == 0) fv *= R(wn);
    }
    if (D == 0) {
      out[h].f0[jw] = fv;
      out[h].s0[jw] = sv;
    } else if (D == 1) {
      out[h].f1[jw] = fv;
      out[h].s1[jw] = sv;
    } else {
      out[h].fz[jw] = fv;
      out[h].sz[jw] = sv;
    }
  }
}

// Per tile: count its hits, claim room for them in `tabs` (tab_start,
// tab_count), and write their tables in candidate order.  The order fixes
// every later summation; the room's place does not matter.  Each tile also
// adds one to bucket min(hits, 255) of the histogram at claimed + 4, from
// which k_tile_order sets the launch order.
template <typename R, int WZ>
__global__ __launch_bounds__(NT) void k_spread_prep(GridGeom G, TileGeom T, const SRec* __restrict__ rec,
                                                    const int* __restrict__ off, HitTab<R, WZ>* __restrict__ tabs,
                                                    int* __restrict__ tab_start, int* __restrict__ tab_count,
                                                    unsigned int* __restrict__ claimed) {
  constexpr int HMAX = NT;
  __shared__ int nb_base[125], nb_pref[126];
  __shared__ double h_e[HMAX][3];
  __shared__ int h_g[HMAX];
  __shared__ int wave_cnt[WAVES];
  __shared__ int base_s;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const TileFrame F = tile_frame(G, T, blockIdx.x, off, nb_base, nb_pref);
  const int total = nb_pref[F.nnb];
  // 1. count the hits
  int mine = 0;
  for (int ci = tid; ci < total; ci += NT) {
    int pos, mask;
    SRec x;
    mine += tile_candidate(G, F, rec, nb_base, nb_pref, ci, pos, mask, x) ? 1 : 0;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) mine += __shfl_xor(mine, o, 64);
  if (lane == 0) wave_cnt[wave] = mine;
  __syncthreads();
  if (tid == 0) {
    int nh = 0;
    for (int w = 0; w < WAVES; ++w) nh += wave_cnt[w];
    base_s = (int)atomicAdd(claimed, (unsigned)nh);
    tab_start[blockIdx.x] = base_s;
    tab_count[blockIdx.x] = nh;
    atomicAdd(claimed + 4 + min(nh, ORDER_BUCKETS - 1), 1u);
  }
  __syncthreads();
  const R big = R(1e30);
  int running = base_s;
  // 2. candidates again, NT at a time: compact the hits, then their tables
  for (int cbase = 0; cbase < total; cbase += NT) {
    int pos = 0, mask = 0;
    SRec x;
    const bool hit = (cbase + tid < total) && tile_candidate(G, F, rec, nb_base, nb_pref, cbase + tid, pos, mask, x);
    const unsigned long long m = __ballot(hit);
    if (lane == 0) wave_cnt[wave] = __popcll(m);
    __syncthreads();
    int before = 0, nh = 0;
    for (int w = 0; w < WAVES; ++w) {
      if (w < wave) before += wave_cnt[w];
      nh += wave_cnt[w];
    }
    if (hit) {
      const int slot = before + __popcll(m & ((1ull << lane) - 1ull));
      h_e[slot][0] = x.e[0];
      h_e[slot][1] = x.e[1];
      h_e[slot][2] = x.e[2];
      h_g[slot] = x.g;
      HitTab<R, WZ>& t = tabs[running + slot];
      t.mask = mask;
      t.pos = pos;
      t.blob = x.blob;
      t.zlo = WZ == 32 ? 0 : hit_zlo((x.g >> 20) & 1023, F.ts[2], G.n[2], G.P[2]);
    }
    __syncthreads();
    table_axis<R, 0, WZ>(G, F, nh, h_e, h_g, tabs + running, big);
    table_axis<R, 1, WZ>(G, F, nh, h_e, h_g, tabs + running, big);
    table_axis<R, 2, WZ>(G, F, nh, h_e, h_g, tabs + running, big);
    running += nh;
    __syncthreads();
  }
}

// Launch order of the spreading workgroups: tiles by hit count, largest
// first, as {tile, start, count, 0}, so that the longest tiles start with
// the first workgroups instead of ending the launch.  One thread per tile:
// every workgroup scans the hit-count histogram of k_spread_prep (claimed +
// 4, descending), and a tile takes the next place of its bucket from the
// cursors at claimed + 4 + ORDER_BUCKETS.  Ties land in any order; a tile's
// result does not depend on where it is launched.
__global__ __launch_bounds__(NT) void k_tile_order(const int* __restrict__ tab_start,
                                                   const int* __restrict__ tab_count, int ntiles,
                                                   unsigned int* __restrict__ claimed, int4* __restrict__ order) {
  static_assert(ORDER_BUCKETS == NT, "one bucket per thread");
  __shared__ int base[ORDER_BUCKETS], wsum[WAVES];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int t = blockIdx.x * NT + tid;
  const int c = t < ntiles ? tab_count[t] : 0;
  const int st = t < ntiles ? tab_start[t] : 0;
  // thread i takes bucket ORDER_BUCKETS - 1 - i: an exclusive scan in descending count
  const int v = (int)claimed[4 + ORDER_BUCKETS - 1 - tid];
  int inc = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int u = __shfl_up(inc, o, 64);
    if (lane >= o) inc += u;
  }
  if (lane == 63) wsum[wave] = inc;
  __syncthreads();
  int before = 0;
  for (int w = 0; w < wave; ++w) before += wsum[w];
  base[ORDER_BUCKETS - 1 - tid] = before + inc - v;
  __syncthreads();
  if (t >= ntiles) return;
  const int b = min(c, ORDER_BUCKETS - 1);
  const int slot = base[b] + (int)atomicAdd(claimed + 4 + ORDER_BUCKETS + b, 1u);
  if (slot < ntiles) order[slot] = make_int4(t, st, c, 0);
}

// Spreading f = S lambda, one workgroup of 512 threads per tile, from the
// tables of k_spread_prep.  Wave w owns z-chunk w % 4 (8 consecutive axis-2
// points) and the hits of parity w / 4; lane = (axis-1 offset, point of the
// chunk), with the 8 axis-0 planes of its point in registers.  Per hit it
// skips, wave-uniformly, a chunk the hit misses and the axis-0 planes outside
// the hit's stencil; a point costs a product, a compare and three
// multiply-adds.  Splitting the hits between two waves per chunk halves the
// longest workgroup (the kernel lasts as long as its busiest tile); the odd
// half is added to the even one through LDS in a fixed order.  The tile then
// goes out with 16-byte stores, whole 128-byte rows at a time.  No atomics and
// a fixed summation order: results repeat bit for bit.
// Each round of up to 64 hits is staged in LDS; every wave keeps the round's
// hit masks and forces in its lanes and takes them with readlane.  A hit's
// axis-0 factors (f0, s0: the same for every lane) come from the table in
// global memory through scalar loads into scalar registers, one load per hit;
// each lane reads its four axis-1 and axis-2 factors from LDS together,
// before any test, so a hit costs one LDS round trip.
constexpr int NTS = 512;   // threads of a spreading workgroup

// Value of v in lane l (l wave-uniform), without LDS.
__device__ __forceinline__ float read_lane(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ __forceinline__ double read_lane(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

template <typename R, int WZ>
__device__ __forceinline__ void spread_tab_body(const GridGeom& G, const TileGeom& T,
                                                const HitTab<R, WZ>* __restrict__ tabs,
                                                const int4* __restrict__ order, const double* __restrict__ lam,
                                                const double* __restrict__ lam_sorted, R* __restrict__ f,
                                                const int* __restrict__ skip, const BlockIx& bi) {
  if (skip && *skip) return;
  constexpr int HR = 64;                // hits per round
  constexpr int TX = 8, TZ = 32;
  // staged row stride: the 8 rows (axis 1) a wave writes for one plane start
  // 40 words apart, 8 distinct bank groups (FP32); FP64 rows are 2 words per value
  constexpr int TZP = sizeof(R) == 4 ? TZ + 8 : TZ;
  constexpr int STAGE = 3 * TX * TX * TZP;
  constexpr int TABR = HR * (int)(sizeof(HitTab<R, WZ>) / sizeof(R));
  constexpr int SH = TABR > STAGE ? TABR : STAGE;
  __shared__ __align__(16) R sh[SH];    // a round of tables, then the staged tile
  __shared__ R h_l[HR][3];
  HitTab<R, WZ>* tab = reinterpret_cast<HitTab<R, WZ>*>(sh);
  // wave and half are wave-uniform; readfirstlane makes the per-hit tests scalar branches
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane((tid >> 6) & 3), half = __builtin_amdgcn_readfirstlane(tid >> 8);
  // workgroups take the tiles in the order of k_spread_prep, largest first
  const int4 ord = order[bi.x];
  const int tl = ord.x, start = ord.y, cnt = ord.z;
  const int t2 = tl % T.nt[2], t1 = (tl / T.nt[2]) % T.nt[1], t0 = tl / (T.nt[1] * T.nt[2]);
  const int ts[3] = {t0 * T.T[0], t1 * T.T[1], t2 * T.T[2]};
  const int te[3] = {min(T.T[0], G.n[0] - ts[0]), min(T.T[1], G.n[1] - ts[1]), min(T.T[2], G.n[2] - ts[2])};
  const R rc2 = R(G.rc2);
  const int j1 = lane >> 3, zl = lane & 7, z = wave * 8 + zl;
  const bool live = j1 < te[1] && z < te[2];
  R acc[TX][3];
#pragma unroll
  for (int k = 0; k < TX; ++k) acc[k][0] = acc[k][1] = acc[k][2] = R(0);
  constexpr int V16 = (int)(sizeof(HitTab<R, WZ>) / 16);
  for (int hb = 0; hb < cnt; hb += HR) {
    const int nr = min(HR, cnt - hb);
    // the round's table loads and the forces of its hits (record position,
    // then force) are all in flight before the first LDS store
    // native 4-word vectors: an array of them stays in registers
    typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
    const u32x4* src = reinterpret_cast<const u32x4*>(tabs + start + hb);
    u32x4* dstv = reinterpret_cast<u32x4*>(sh);
    // (one vector at a time: staged vectors would be live beside the
    // accumulators and cost a workgroup per CU)
    for (int v = tid; v < nr * V16; v += NTS) dstv[v] = src[v];
    double lv[3] = {0.0, 0.0, 0.0};
    if (tid < nr) {
      const HitTab<R, WZ>& g = tabs[start + hb + tid];
      const long long base = lam_sorted ? 3LL * g.pos : 3LL * g.blob;
      const double* ls = lam_sorted ? lam_sorted : lam;
#pragma unroll
      for (int q = 0; q < 3; ++q) lv[q] = ls[base + q];
    }
    if (tid < nr) {
#pragma unroll
      for (int q = 0; q < 3; ++q) h_l[tid][q] = R(lv[q]);
    }
    __syncthreads();
    // lane h of every wave holds hit h's mask and force for the round; the
    // hit loop takes them with readlane (no LDS round trip per hit)
    const int hr = lane < nr ? lane : 0;
    const int hmask = lane < nr ? tab[hr].mask : 0;
    const int hzlo = lane < nr ? tab[hr].zlo : 0;
    const R hl0 = h_l[hr][0], hl1 = h_l[hr][1], hl2 = h_l[hr][2];
    // the loop runs with every lane of the wave active up to the per-lane
    // test below, so each readlane sees values all lanes hold
    for (int h = half; h < nr; h += 2) {
      const int hm = __builtin_amdgcn_readlane(hmask, h);
      if (!((hm >> wave) & 1)) continue;
      const R l0 = read_lane(hl0, h), l1 = read_lane(hl1, h), l2 = read_lane(hl2, h);
      const HitTab<R, WZ>& t = tab[h];
      // the hit's axis-0 factors, the same for every lane: read from the
      // round's table in LDS at one address for the whole wave (h is
      // wave-uniform)
      R f0s[TX], s0s[TX];
#pragma unroll
      for (int k = 0; k < TX; ++k) {
        f0s[k] = t.f0[k];
        s0s[k] = t.s0[k];
      }
      // this lane's entry of the hit's axis-2 window (outside it: no weight)
      const int zz = z - (WZ == 32 ? 0 : __builtin_amdgcn_readlane(hzlo, h));
      const bool zin = (unsigned)zz < (unsigned)WZ;
      const int zi = zin ? zz : 0;
      // the lane's axis-1 and axis-2 factors, all four read before any test
      // (the empty asm marks them as needed here, so the compiler does not
      // move the second pair into the branch: one LDS round trip per hit)
      const R s1v = t.s1[j1], szv = t.sz[zi], f1v = t.f1[j1], fzv = t.fz[zi];
      asm volatile("" ::"v"(s1v), "v"(szv), "v"(f1v), "v"(fzv));
      if (!live || !zin) continue;
      const R s12 = s1v + szv;
      if (s12 > rc2) continue;
      const R f12 = f1v * fzv;
#pragma unroll
      for (int k = 0; k < TX; ++k) {
        if (!((hm >> (8 + k)) & 1)) continue;
        // a hit touches only some of the tile's 8 planes: the empty asm keeps
        // this a scalar branch (the compiler would otherwise evaluate all
        // eight planes and select, about 20% slower per launch)
        asm volatile("");
        const R w = (s0s[k] + s12 <= rc2) ? f12 * f0s[k] : R(0);
        acc[k][0] += w * l0;
        acc[k][1] += w * l1;
        acc[k][2] += w * l2;
      }
    }
    __syncthreads();
  }
  // stage [c][axis-0][axis-1][z]: the odd-hit half first, then the even
  // half adds its sums, and write rows with 16-byte stores
  if (half == 1) {
#pragma unroll
    for (int k = 0; k < TX; ++k) {
#pragma unroll
      for (int cc = 0; cc < 3; ++cc) sh[(cc * TX * TX + k * TX + j1) * TZP + z] = acc[k][cc];
    }
  }
  __syncthreads();
  if (half == 0) {
#pragma unroll
    for (int k = 0; k < TX; ++k) {
#pragma unroll
      for (int cc = 0; cc < 3; ++cc) {
        const int a = (cc * TX * TX + k * TX + j1) * TZP + z;
        sh[a] = acc[k][cc] + sh[a];
      }
    }
  }
  __syncthreads();
  constexpr int VW = 16 / sizeof(R);   // values per 16-byte store
  constexpr int NV = TZ / VW;          // stores per row
  const long long Gs = G.G;
  if (G.tiled) {
    // tile-major field: the tile (all tiles full) is one contiguous block per component
    for (int p = tid; p < 3 * TX * TX * NV; p += NTS) {
      const int cc = p / (TX * TX * NV), rem = p - cc * (TX * TX * NV);
      const int col = rem / NV, zv = (rem - col * NV) * VW;
      const R* srcv = sh + (cc * TX * TX + col) * TZP + zv;
      R* dst = f + cc * Gs + (long long)tl * (TX * TX * TZ) + col * TZ + zv;
      if constexpr (sizeof(R) == 4) {
        *reinterpret_cast<float4*>(dst) = make_float4(srcv[0], srcv[1], srcv[2], srcv[3]);
      } else {
        *reinterpret_cast<double2*>(dst) = make_double2(srcv[0], srcv[1]);
      }
    }
    return;
  }
  for (int p = tid; p < 3 * TX * TX * NV; p += NTS) {
    const int cc = p / (TX * TX * NV), rem = p - cc * (TX * TX * NV);
    const int col = rem / NV, zv = (rem - col * NV) * VW;
    const int c0 = col >> 3, c1 = col & 7;
    if (c0 >= te[0] || c1 >= te[1] || zv >= te[2]) continue;
    const long long idx = cc * Gs + ((long long)(ts[0] + c0) * G.n[1] + (ts[1] + c1)) * G.n[2] + ts[2] + zv;
    const R* srcv = sh + (cc * TX * TX + col) * TZP + zv;
    if (zv + VW <= te[2]) {
      if constexpr (sizeof(R) == 4) {
        *reinterpret_cast<float4*>(f + idx) = make_float4(srcv[0], srcv[1], srcv[2], srcv[3]);
      } else {
        *reinterpret_cast<double2*>(f + idx) = make_double2(srcv[0], srcv[1]);
      }
    } else {
      for (int v = 0; zv + v < te[2]; ++v) f[idx + v] = srcv[v];
    }
  }
}

// The ordinary FP32 launch is held to 8 waves per SIMD (four workgroups per
// CU; it needs 48 VGPRs and 76 SGPRs).  The fused launch, with its
// per-suspension arguments in registers, is left to the compiler: held to
// the same target it would spill.
#define GDC_SPREAD_OCCUPANCY __attribute__((amdgpu_waves_per_eu(sizeof(R) == 4 ? 8 : 1)))

template <typename R, int WZ>
__global__ __launch_bounds__(NTS) GDC_SPREAD_OCCUPANCY void k_spread_tab(
    GridGeom G, TileGeom T, const HitTab<R, WZ>* __restrict__ tabs, const int4* __restrict__ order,
    const double* __restrict__ lam, const double* __restrict__ lam_sorted, R* __restrict__ f,
    const int* __restrict__ skip) {
  spread_tab_body<R, WZ>(G, T, tabs, order, lam, lam_sorted, f, skip, hw_block());
}

// Spreading fused over several suspensions (one SpreadArgs each).
template <typename R, int WZ>
__global__ __launch_bounds__(NTS) void k_spread_tab_fused(
    const SpreadArgs* __restrict__ a, const int* __restrict__ first, int ns) {
  const int sidx = fused_suspension(first, ns, blockIdx.x);
  const SpreadArgs& A = a[sidx];
  spread_tab_body<R, WZ>(A.G, A.T, (const HitTab<R, WZ>*)A.tabs, A.order, A.lam, A.lam_sorted, (R*)A.f, A.skip,
                         fused_block(A.grid, (int)blockIdx.x - first[sidx]));
}

__global__ void k_fill_zero(uint4* __restrict__ p, long long n16) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long k = i; k < n16; k += stride) p[k] = make_uint4(0u, 0u, 0u, 0u);
}

template <typename R>
__global__ void k_to_rowmajor(GridGeom G, const R* __restrict__ x, double* __restrict__ y) {
  const long long n = 3 * G.G;
  const long long stride = (long long)gridDim.x * blockDim.x;
  const int n1 = G.n[1], n2 = G.n[2];
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) {
    const long long c = e / G.G, rem = e - c * G.G;
    const int i2 = (int)(rem % n2);
    const long long r01 = rem / n2;
    const int i1 = (int)(r01 % n1), i0 = (int)(r01 / n1);
    y[e] = (double)x[c * G.G + field_plane_off(G.tiled, n1, n2, i0) + field_col_off(G.tiled, n2, i1, i2)];
  }
}

inline unsigned blocks_for(int M) {
  const unsigned nb = (unsigned)((M + WAVES - 1) / WAVES);
  return (nb + NXCD - 1) / NXCD * NXCD;
}

}  // namespace

size_t tile_record_bytes() { return sizeof(SRec); }

// Up to four buffers cleared by one launch (the segments are walked in turn).
struct ZeroList {
  uint4* p[4];
  long long n16[4];
  int n;
};

__global__ void k_fill_zero_many(ZeroList z) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  const long long i0 = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  for (int k = 0; k < z.n; ++k)
    for (long long i = i0; i < z.n16[k]; i += stride) z.p[k][i] = make_uint4(0u, 0u, 0u, 0u);
}

int fill_zero_many(void* const* ptrs, const size_t* bytes, int n, hipStream_t s) {
  if (n < 0 || n > 4) {
    set_error("fill_zero_many: at most four buffers");
    return GDC_EINVAL;
  }
  ZeroList z{};
  long long most = 0;
  int m = 0;
  for (int k = 0; k < n; ++k) {
    if (bytes[k] == 0) continue;
    if ((bytes[k] & 15) || (reinterpret_cast<uintptr_t>(ptrs[k]) & 15)) {
      set_error("fill_zero_many: sizes and addresses must be 16-byte aligned");
      return GDC_EINVAL;
    }
    z.p[m] = reinterpret_cast<uint4*>(ptrs[k]);
    z.n16[m] = (long long)(bytes[k] / 16);
    most = std::max(most, z.n16[m]);
    ++m;
  }
  z.n = m;
  if (m == 0) return GDC_OK;
  const long long blocks = std::min<long long>((most + 255) / 256, 2048);
  hipLaunchKernelGGL(k_fill_zero_many, dim3((unsigned)blocks), dim3(256), 0, s, z);
  return check_launch("k_fill_zero_many");
}

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

template <typename R>
__global__ void k_fill_sine(GridGeom G, R* __restrict__ f, double k) {
  const long long n = 3 * G.G;
  const long long stride = (long long)gridDim.x * blockDim.x;
  const int n1 = G.n[1], n2 = G.n[2];
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) {
    const long long c = e / G.G, rem = e - c * G.G;
    const int i2 = (int)(rem % n2);
    const long long r01 = rem / n2;
    const int i1 = (int)(r01 % n1), i0 = (int)(r01 / n1);
    f[c * G.G + field_plane_off(G.tiled, n1, n2, i0) + field_col_off(G.tiled, n2, i1, i2)] =
        c == 0 ? R(sin(k * (i1 * G.dx[1]))) : R(0);
  }
}

__global__ __launch_bounds__(1024) void k_blob_dot_x(const double* __restrict__ a, const double* __restrict__ b,
                                                     int M, double* __restrict__ out) {
  __shared__ double sh[16];
  double t = 0.0;
  for (int i = threadIdx.x; i < M; i += 1024) t += a[3LL * i] * b[3LL * i];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = t;
  __syncthreads();
  if (threadIdx.x == 0) {
    double u = 0.0;
    for (int w = 0; w < 16; ++w) u += sh[w];
    *out = u;
  }
}

template <typename R>
int field_to_rowmajor(const GridGeom& g, const R* x, double* y, hipStream_t s) {
  const long long want = (3 * g.G + 255) / 256;
  hipLaunchKernelGGL((k_to_rowmajor<R>), dim3((unsigned)(want < 8192 ? (want > 0 ? want : 1) : 8192)), dim3(256),
                     0, s, g, x, y);
  return check_launch("k_to_rowmajor");
}
template int field_to_rowmajor<float>(const GridGeom&, const float*, double*, hipStream_t);

template <typename R>
int fill_sine_field(const GridGeom& g, R* f, hipStream_t s) {
  const long long want = (3 * g.G + 255) / 256;
  const double k = 2.0 * 3.14159265358979323846 / g.L[1];
  hipLaunchKernelGGL((k_fill_sine<R>), dim3((unsigned)(want < 8192 ? (want > 0 ? want : 1) : 8192)), dim3(256), 0,
                     s, g, f, k);
  return check_launch("k_fill_sine");
}
template int fill_sine_field<float>(const GridGeom&, float*, hipStream_t);
template int fill_sine_field<double>(const GridGeom&, double*, hipStream_t);

int blob_dot_x(const double* a, const double* b, int M, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_blob_dot_x, dim3(1), dim3(1024), 0, s, a, b, M, out);
  return check_launch("k_blob_dot_x");
}
template int field_to_rowmajor<double>(const GridGeom&, const double*, double*, hipStream_t);

int tile_sort(const GridGeom& g, const TileGeom& t, const double* r, int M, int* tile, int* count, int* off,
              int* cursor, void* rec, int* spos, hipStream_t s, bool zeroed) {
  if (!zeroed) GDC_TRY(fill_zero(count, tile_count_bytes(t), s));
  if (M > 0) {
    hipLaunchKernelGGL(k_tile_count, dim3((M + 255) / 256), dim3(256), 0, s, g, t, r, M, tile, count);
    GDC_TRY(check_launch("k_tile_count"));
  }
  hipLaunchKernelGGL(k_tile_scan, dim3(1), dim3(1024), 0, s, count, t.ntiles, off, cursor);
  GDC_TRY(check_launch("k_tile_scan"));
  if (M > 0) {
    SRec* sorted = (SRec*)rec;
    SRec* unordered = sorted + M;
    hipLaunchKernelGGL(k_tile_scatter, dim3((M + 255) / 256), dim3(256), 0, s, g, r, tile, M, cursor, unordered);
    GDC_TRY(check_launch("k_tile_scatter"));
    hipLaunchKernelGGL(k_tile_rank, dim3((t.ntiles + 3) / 4), dim3(256), 0, s, off, t.ntiles, unordered, sorted,
                       spos);
    GDC_TRY(check_launch("k_tile_rank"));
  }
  return GDC_OK;
}

size_t spread_table_bytes(const GridGeom& g, const TileGeom& t, int M, int precision) {
  // a stencil of P points meets at most ceil((P - 1) / T) + 2 tiles of an
  // axis (a partial last tile can add one), and never more than nt
  size_t per = 1;
  for (int d = 0; d < 3; ++d) {
    const int k = (g.P[d] - 1 + t.T[d] - 1) / t.T[d] + 2;
    per *= (size_t)std::min(k, t.nt[d]);
  }
  const size_t rec = precision == GDC_FP64
                         ? (t.wz8 ? sizeof(HitTab<double, 8>) : sizeof(HitTab<double, 32>))
                         : (t.wz8 ? sizeof(HitTab<float, 8>) : sizeof(HitTab<float, 32>));
  return per * (size_t)(M > 0 ? M : 1) * rec;
}

template <typename R>
int spread_prepare(const GridGeom& g, const TileGeom& t, const void* rec, const int* off, void* tabs,
                   int* tab_start, int* tab_count, int* order, unsigned int* claimed, hipStream_t s, bool zeroed) {
  if (t.T[0] != 8 || t.T[1] != 8 || t.T[2] > 32) {
    set_error("spread: tiles must be 8 x 8 x (up to 32)");
    return GDC_EINVAL;
  }
  if (!zeroed) GDC_TRY(fill_zero(claimed, spread_claim_bytes(), s));
  if (t.wz8)
    hipLaunchKernelGGL((k_spread_prep<R, 8>), dim3(t.ntiles), dim3(NT), 0, s, g, t, (const SRec*)rec, off,
                       (HitTab<R, 8>*)tabs, tab_start, tab_count, claimed);
  else
    hipLaunchKernelGGL((k_spread_prep<R, 32>), dim3(t.ntiles), dim3(NT), 0, s, g, t, (const SRec*)rec, off,
                       (HitTab<R, 32>*)tabs, tab_start, tab_count, claimed);
  GDC_TRY(check_launch("k_spread_prep"));
  hipLaunchKernelGGL(k_tile_order, dim3((t.ntiles + NT - 1) / NT), dim3(NT), 0, s, tab_start, tab_count, t.ntiles,
                     claimed, (int4*)order);
  return check_launch("k_tile_order");
}

void spread_describe(SpreadArgs& a, const GridGeom& g, const TileGeom& t, const void* tabs, const int* order,
                     const double* lam, const double* lam_sorted, void* f, const int* skip) {
  a.G = g;
  a.T = t;
  a.tabs = tabs;
  a.order = (const int4*)order;
  a.lam = lam;
  a.lam_sorted = lam_sorted;
  a.f = f;
  a.skip = skip;
  a.grid = LocalGrid{t.ntiles, 1, 1};
}

template <typename R>
int spread_fused(const SpreadArgs* dev_args, int ns, int wz8, const int* first, int total, hipStream_t s) {
  if (ns <= 0) return GDC_OK;
  if (wz8)
    hipLaunchKernelGGL((k_spread_tab_fused<R, 8>), dim3(total), dim3(NTS), 0, s, dev_args, first, ns);
  else
    hipLaunchKernelGGL((k_spread_tab_fused<R, 32>), dim3(total), dim3(NTS), 0, s, dev_args, first, ns);
  return check_launch("k_spread_tab_fused");
}

void interp_describe(InterpArgs& a, const GridGeom& g, const double* r, const void* u, double* v, int M,
                     double scale, const int* blob_body, const double* Y, const double* V, const int* skip,
                     const void* sorted) {
  a.G = g;
  a.r = r;
  a.u = u;
  a.v = v;
  a.M = M;
  a.scale = scale;
  a.blob_body = blob_body;
  a.Y = Y;
  a.V = V;
  a.skip = skip;
  a.rec = sorted;
  a.grid = LocalGrid{(int)blocks_for(M), 1, 1};
}

template <typename R>
int interp_fused(const InterpArgs* dev_args, int ns, const int* first, int total, hipStream_t s) {
  if (ns <= 0) return GDC_OK;
  hipLaunchKernelGGL((k_interp_fused<R>), dim3(total), dim3(NT), 0, s, dev_args, first, ns);
  return check_launch("k_interp_fused");
}

template <typename R>
int spread(const GridGeom& g, const TileGeom& t, const void* tabs, const int* order, const double* lam,
           const double* lam_sorted, R* f, hipStream_t s, const int* skip) {
  if (t.T[0] != 8 || t.T[1] != 8 || t.T[2] > 32) {
    set_error("spread: tiles must be 8 x 8 x (up to 32)");
    return GDC_EINVAL;
  }
  const ProbeEvents pe = probe_claim("spread");
#define GDC_SPREAD_(W)                                                                          \
  GDC_LAUNCH_PROBED((k_spread_tab<R, W>), dim3(t.ntiles), dim3(NTS), 0, s, pe, g, t, (const HitTab<R, W>*)tabs, \
                    (const int4*)order, lam, lam_sorted, f, skip)
  if (t.wz8)
    GDC_SPREAD_(8);
  else
    GDC_SPREAD_(32);
#undef GDC_SPREAD_
  return check_launch("k_spread_tab");
}

template <typename R>
int interp(const GridGeom& g, const double* r, const R* u, double* v, int M, double scale,
           const int* blob_body, const double* Y, const double* V, hipStream_t s, const int* skip,
           const void* sorted) {
  if (M <= 0) return GDC_OK;
  if (g.n[2] % 4 != 0) {
    set_error("interp: the grid's axis 2 must be a multiple of 4 (16-byte chunks)");
    return GDC_EINVAL;
  }
  if (g.P[2] + 2 * Component<R>::CW - 2 > 64) {
    set_error("interp: the stencil is too wide along axis 2 for the 64 per-blob factors");
    return GDC_EINVAL;
  }
  RigidTerm K{blob_body, Y, V};
  const ProbeEvents pe = probe_claim("interp");
  GDC_LAUNCH_PROBED((k_interp<R>), dim3(blocks_for(M)), dim3(NT), 0, s, pe, g, r, u, v, M, scale, K, skip,
                     (const SRec*)sorted);
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

template int spread_prepare<float>(const GridGeom&, const TileGeom&, const void*, const int*, void*, int*, int*,
                                   int*, unsigned int*, hipStream_t, bool);
template int spread_prepare<double>(const GridGeom&, const TileGeom&, const void*, const int*, void*, int*, int*,
                                    int*, unsigned int*, hipStream_t, bool);
template int spread<float>(const GridGeom&, const TileGeom&, const void*, const int*, const double*, const double*,
                           float*, hipStream_t, const int*);
template int spread<double>(const GridGeom&, const TileGeom&, const void*, const int*, const double*, const double*,
                            double*, hipStream_t, const int*);
template int spread_fused<float>(const SpreadArgs*, int, int, const int*, int, hipStream_t);
template int spread_fused<double>(const SpreadArgs*, int, int, const int*, int, hipStream_t);
template int interp_fused<float>(const InterpArgs*, int, const int*, int, hipStream_t);
template int interp_fused<double>(const InterpArgs*, int, const int*, int, hipStream_t);
template int interp<float>(const GridGeom&, const double*, const float*, double*, int, double, const int*,
                           const double*, const double*, hipStream_t, const int*, const void*);
template int interp<double>(const GridGeom&, const double*, const double*, double*, int, double, const int*,
                            const double*, const double*, hipStream_t, const int*, const void*);
template int interp_fd<float>(const GridGeom&, const double*, const double*, int, const float*, double*,
                              double*, int, hipStream_t);
template int interp_fd<double>(const GridGeom&, const double*, const double*, int, const double*, double*,
                               double*, int, hipStream_t);

}  // namespace gdc
