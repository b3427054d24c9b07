// Gaussian spreading S and averaging J = S* between blobs and the grid
// (Sec. 4.2, eq. spreading and eq. averaging).
//
// Delta_i(x) = (2 pi sigma^2)^{-3/2} exp(-|x - r_i|^2 / 2 sigma^2), set to zero
// beyond the cutoff radius rc (minimum-image distance, no renormalisation), so
// J = dV S^T exactly.  Averaging: one 64-wide wavefront per blob walks the
// blob's stencil.  Spreading: one workgroup per grid tile gathers the blobs
// that reach it (see k_spread_tiles).  Positions arrive in FP64; each blob's offset to
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

// Stencil walk in columns: lane l owns the (a1, a2) pairs l, l + 64, ... of
// the P1 x P2 cross-section and loops over a0, so consecutive lanes read
// consecutive grid points along axis 2 and no division happens in the loop.

// Rigid-body term subtracted by the averaging epilogue of the saddle operator:
// U_p + Omega_p x (r_i - Y_p) for blob i of body p.
struct RigidTerm {
  const int* blob_body;   // M
  const double* Y;        // N x 3
  const double* V;        // N x 6 (U, Omega); null: no rigid term
};

template <typename R>
__global__ __launch_bounds__(NT) void k_interp(GridGeom G, const double* __restrict__ r,
                                               const R* __restrict__ u, double* __restrict__ v, int M,
                                               double scale, RigidTerm K) {
  const int blob = blockIdx.x * WAVES + threadIdx.x / 64;
  const int lane = threadIdx.x & 63;
  if (blob >= M) return;
  const BlobBase B = blob_base(G, r + 3LL * blob, 0);
  const int P0 = G.P[0], P1 = G.P[1], P2 = G.P[2];
  const long long Gs = G.G;
  const int n0 = G.n[0], n1 = G.n[1], n2 = G.n[2];
  const R wn = R(G.wnorm), i2 = R(G.inv2s2);
  R s0 = 0, s1 = 0, s2 = 0;
  for (int pr = lane; pr < P1 * P2; pr += 64) {
    const int a1 = pr / P2, a2 = pr - a1 * P2;
    const double d1 = B.e[1] + a1 * G.dx[1], d2 = B.e[2] + a2 * G.dx[2];
    const double d12 = d1 * d1 + d2 * d2;
    if (d12 > G.rc2) continue;
    const long long col = (long long)wrap(B.g[1] + a1, n1) * n2 + wrap(B.g[2] + a2, n2);
    const long long plane = (long long)n1 * n2;
    // four points of the column per round, all loads issued before use
    for (int a0 = 0; a0 < P0; a0 += 4) {
      R wv[4];
      long long ix[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int aa = a0 + q;
        const int gg = wrap(B.g[0] + aa, n0);
        const double d0 = B.e[0] + aa * G.dx[0];
        const double dd = d0 * d0 + d12;
        const bool ok = (aa < P0) && (dd <= G.rc2);
        wv[q] = ok ? wn * gexp<R>(-R(dd) * i2) : R(0);
        ix[q] = (long long)(ok ? gg : B.g[0]) * plane + col;
      }
      R x0[4], x1[4], x2[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        x0[q] = u[ix[q]];
        x1[q] = u[Gs + ix[q]];
        x2[q] = u[2 * Gs + ix[q]];
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        s0 += wv[q] * x0[q];
        s1 += wv[q] * x1[q];
        s2 += wv[q] * x2[q];
      }
    }
  }
  s0 = wave_sum(s0);
  s1 = wave_sum(s1);
  s2 = wave_sum(s2);
  if (lane == 0) {
    double o[3] = {scale * (double)s0, scale * (double)s1, scale * (double)s2};
    if (K.V) {
      const int p = K.blob_body[blob];
      const double* Vp = K.V + 6LL * p;
      const double rel[3] = {r[3LL * blob] - K.Y[3LL * p], r[3LL * blob + 1] - K.Y[3LL * p + 1],
                             r[3LL * blob + 2] - K.Y[3LL * p + 2]};
      o[0] -= Vp[0] + (Vp[4] * rel[2] - Vp[5] * rel[1]);
      o[1] -= Vp[1] + (Vp[5] * rel[0] - Vp[3] * rel[2]);
      o[2] -= Vp[2] + (Vp[3] * rel[1] - Vp[4] * rel[0]);
    }
    v[3LL * blob] = o[0];
    v[3LL * blob + 1] = o[1];
    v[3LL * blob + 2] = o[2];
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
    const long long col = (long long)wrap(B.g[1] + a1, n1) * n2 + wrap(B.g[2] + a2, n2);
    int g0 = B.g[0];
    for (int a0 = 0; a0 < P0; ++a0, g0 = (g0 + 1 == n0) ? 0 : g0 + 1) {
      const double d0 = B.e[0] + a0 * G.dx[0];
      const double dd = d0 * d0 + d12;
      if (dd > reach2) continue;
      const bool in0 = dd <= G.rc2;
      const long long idx = (long long)g0 * n1 * n2 + col;
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
          dw = w * gexpm1<R>(R(2.0 * dot - Dr2[k]) * i2);
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
struct SRec {
  double e[3];
  int g;
  int blob;
};

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
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int t = blockIdx.x * 4 + w;
  if (t >= ntiles) return;   // whole wave leaves together; no block barrier below
  const int lo = off[t], hi = off[t + 1];
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

// Spreading by gathering: one workgroup per tile of 8 x 8 x 32 points; thread
// (j0, j1, b) owns the 8 points (j0, j1, 8b..8b+7) and keeps their three
// force components in registers.  The blobs that reach the tile are collected
// in LDS in candidate order (tiles are sorted by blob index), then every
// thread adds each blob's Gaussian to its points: no atomics, one coalesced
// write of the tile, and a fixed summation order.
template <typename R>
__global__ __launch_bounds__(NT) void k_spread_gather(GridGeom G, TileGeom T, const SRec* __restrict__ rec,
                                                      const int* __restrict__ off, const double* __restrict__ lam,
                                                      const double* __restrict__ lam_sorted, R* __restrict__ f) {
  constexpr int HMAX = 2 * NT;
  __shared__ int nb_base[125], nb_pref[126];
  __shared__ double hit_e[HMAX][3];
  __shared__ R hit_l[HMAX][3];
  __shared__ int hit_g[HMAX];
  __shared__ int wave_cnt[2 * WAVES];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int tl = blockIdx.x;
  const int t2 = tl % T.nt[2], t1 = (tl / T.nt[2]) % T.nt[1], t0 = tl / (T.nt[1] * T.nt[2]);
  const int tt[3] = {t0, t1, t2};
  const int ts[3] = {t0 * T.T[0], t1 * T.T[1], t2 * T.T[2]};
  const int te[3] = {min(T.T[0], G.n[0] - ts[0]), min(T.T[1], G.n[1] - ts[1]), min(T.T[2], G.n[2] - ts[2])};
  int c[3], st[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    c[d] = min(2 * T.H[d] + 1, T.nt[d]);
    st[d] = (c[d] == T.nt[d]) ? 0 : tt[d] - T.H[d];
  }
  const int nnb = c[0] * c[1] * c[2];
  if (tid < nnb) {
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
    for (int k = 1; k <= nnb; ++k) nb_pref[k] += nb_pref[k - 1];
  }
  __syncthreads();
  const int total = nb_pref[nnb];
  // this thread's points
  const int j0 = tid >> 5, j1 = (tid >> 2) & 7, zb = tid & 3;
  const bool live = j0 < te[0] && j1 < te[1] && zb * 8 < te[2];
  const R wn = R(G.wnorm), i2 = R(G.inv2s2);
  R acc[8][3];
#pragma unroll
  for (int k = 0; k < 8; ++k) acc[k][0] = acc[k][1] = acc[k][2] = R(0);
  for (int base = 0; base < total; base += HMAX) {
    // compact the hits of this round in candidate order
    int hslot[2];
    bool hflag[2];
    SRec hx[2];
    double hl[2][3];
#pragma unroll
    for (int half = 0; half < 2; ++half) {
      const int ci = base + half * NT + tid;
      hflag[half] = false;
      if (ci < total) {
        int k = 0;
        while (nb_pref[k + 1] <= ci) ++k;
        const int pos = nb_base[k] + (ci - nb_pref[k]);
        hx[half] = rec[pos];
        const SRec& x = hx[half];
        if (lam_sorted) {
          hl[half][0] = lam_sorted[3LL * pos];
          hl[half][1] = lam_sorted[3LL * pos + 1];
          hl[half][2] = lam_sorted[3LL * pos + 2];
        } else {
          hl[half][0] = lam[3LL * x.blob];
          hl[half][1] = lam[3LL * x.blob + 1];
          hl[half][2] = lam[3LL * x.blob + 2];
        }
        const int gb[3] = {x.g & 1023, (x.g >> 10) & 1023, (x.g >> 20) & 1023};
        bool hit = true;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          const Ranges Rg = axis_ranges(gb[d], ts[d], te[d], G.n[d], G.P[d]);
          hit = hit && (Rg.l1 + Rg.l2 > 0);
        }
        hflag[half] = hit;
      }
      const unsigned long long m = __ballot(hflag[half]);
      hslot[half] = __popcll(m & ((1ull << lane) - 1ull));
      if (lane == 0) wave_cnt[half * WAVES + wave] = __popcll(m);
    }
    __syncthreads();
    int nh = 0;
#pragma unroll
    for (int half = 0; half < 2; ++half) {
      int before = nh;
      for (int w = 0; w < WAVES; ++w) {
        if (w < wave) before += wave_cnt[half * WAVES + w];
        nh += wave_cnt[half * WAVES + w];
      }
      if (hflag[half]) {
        const int slot = before + hslot[half];
        hit_e[slot][0] = hx[half].e[0];
        hit_e[slot][1] = hx[half].e[1];
        hit_e[slot][2] = hx[half].e[2];
        hit_g[slot] = hx[half].g;
        hit_l[slot][0] = R(hl[half][0]);
        hit_l[slot][1] = R(hl[half][1]);
        hit_l[slot][2] = R(hl[half][2]);
      }
    }
    __syncthreads();
    if (live) {
      for (int h = 0; h < nh; ++h) {
        const int g = hit_g[h];
        int a0 = ts[0] + j0 - (g & 1023);
        a0 += (a0 < 0) ? G.n[0] : 0;
        int a1 = ts[1] + j1 - ((g >> 10) & 1023);
        a1 += (a1 < 0) ? G.n[1] : 0;
        if (a0 >= G.P[0] || a1 >= G.P[1]) continue;
        const double d0 = hit_e[h][0] + a0 * G.dx[0];
        const double d1 = hit_e[h][1] + a1 * G.dx[1];
        const double d01 = d0 * d0 + d1 * d1;
        if (d01 > G.rc2) continue;
        int a2 = ts[2] + zb * 8 - ((g >> 20) & 1023);
        a2 += (a2 < 0) ? G.n[2] : 0;
        const double e2 = hit_e[h][2];
        const R l0 = hit_l[h][0], l1 = hit_l[h][1], l2 = hit_l[h][2];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const int ak = (a2 + k >= G.n[2]) ? a2 + k - G.n[2] : a2 + k;
          const double dz = e2 + ak * G.dx[2];
          const double dd = d01 + dz * dz;
          if (ak < G.P[2] && dd <= G.rc2) {
            const R w = wn * gexp<R>(-R(dd) * i2);
            acc[k][0] += w * l0;
            acc[k][1] += w * l1;
            acc[k][2] += w * l2;
          }
        }
      }
    }
    __syncthreads();
  }
  if (live) {
    const long long Gs = G.G;
    const long long row = ((long long)(ts[0] + j0) * G.n[1] + (ts[1] + j1)) * G.n[2] + ts[2] + zb * 8;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      if (zb * 8 + k < te[2]) {
        f[row + k] = acc[k][0];
        f[Gs + row + k] = acc[k][1];
        f[2 * Gs + row + k] = acc[k][2];
      }
    }
  }
}

// One workgroup per tile.  MODE 0 (spreading): the tile's field starts at
// zero in LDS, every blob that reaches the tile adds its Gaussian with LDS
// atomics, and the tile is written once.  MODE 1 (averaging): the tile's field
// is read once into LDS with coalesced loads, every blob that reaches the tile
// forms its partial sum over the tile from LDS, and the partial sums are added
// to the blob velocities with one FP64 global atomic per blob, tile and
// component.  LDS rows are padded by one element so that lanes walking a
// stencil cross-section hit distinct banks.
template <typename R, int MODE>
__global__ __launch_bounds__(NT) void k_tile_op(GridGeom G, TileGeom T, const SRec* __restrict__ rec,
                                                const int* __restrict__ off, const double* __restrict__ lam,
                                                const double* __restrict__ lam_sorted, R* __restrict__ f,
                                                const R* __restrict__ u, double* __restrict__ v, double scale) {
  extern __shared__ __align__(16) unsigned char smem[];
  R* acc = reinterpret_cast<R*>(smem);
  const int RS = T.T[2] + 1, PS = T.T[1] * RS, CS = T.T[0] * PS;
  const int TP = T.T[0] * T.T[1] * T.T[2];
  __shared__ int nb_base[125], nb_pref[126];
  constexpr int HMAX = 2 * NT;   // candidates tested per round
  __shared__ double hit_e[HMAX][3];
  __shared__ double hit_l[HMAX][3];
  __shared__ int hit_g[HMAX];
  __shared__ int hit_b[HMAX];
  __shared__ int nhit;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int tl = blockIdx.x;
  const int t2 = tl % T.nt[2], t1 = (tl / T.nt[2]) % T.nt[1], t0 = tl / (T.nt[1] * T.nt[2]);
  const int tt[3] = {t0, t1, t2};
  const int ts[3] = {t0 * T.T[0], t1 * T.T[1], t2 * T.T[2]};
  const int te[3] = {min(T.T[0], G.n[0] - ts[0]), min(T.T[1], G.n[1] - ts[1]), min(T.T[2], G.n[2] - ts[2])};
  const long long Gs = G.G;
  int c[3], st[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    c[d] = min(2 * T.H[d] + 1, T.nt[d]);
    st[d] = (c[d] == T.nt[d]) ? 0 : tt[d] - T.H[d];
  }
  const int nnb = c[0] * c[1] * c[2];
  for (int p = tid; p < TP; p += NT) {
    const int j2 = p % T.T[2], j1 = (p / T.T[2]) % T.T[1], j0 = p / (T.T[1] * T.T[2]);
    const int q = j0 * PS + j1 * RS + j2;
    if (MODE == 0) {
      acc[q] = R(0);
      acc[CS + q] = R(0);
      acc[2 * CS + q] = R(0);
    } else {
      R x0 = 0, x1 = 0, x2 = 0;
      if (j0 < te[0] && j1 < te[1] && j2 < te[2]) {
        const long long idx = ((long long)(ts[0] + j0) * G.n[1] + (ts[1] + j1)) * G.n[2] + ts[2] + j2;
        x0 = u[idx];
        x1 = u[Gs + idx];
        x2 = u[2 * Gs + idx];
      }
      acc[q] = x0;
      acc[CS + q] = x1;
      acc[2 * CS + q] = x2;
    }
  }
  if (tid < nnb) {
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
    for (int k = 1; k <= nnb; ++k) nb_pref[k] += nb_pref[k - 1];
  }
  __syncthreads();
  const int total = nb_pref[nnb];
  const R wn = R(G.wnorm), i2 = R(G.inv2s2);
  for (int base = 0; base < total; base += HMAX) {
    if (tid == 0) nhit = 0;
    __syncthreads();
    // each thread tests two candidates; a hit's record (and forces) go to LDS
#pragma unroll
    for (int half = 0; half < HMAX / NT; ++half) {
      const int ci = base + half * NT + tid;
      if (ci < total) {
        int k = 0;
        while (nb_pref[k + 1] <= ci) ++k;
        const int pos = nb_base[k] + (ci - nb_pref[k]);
        const SRec x = rec[pos];
        double la = 0, lb = 0, lc = 0;
        if (MODE == 0) {
          if (lam_sorted) {
            la = lam_sorted[3LL * pos];
            lb = lam_sorted[3LL * pos + 1];
            lc = lam_sorted[3LL * pos + 2];
          } else {
            la = lam[3LL * x.blob];
            lb = lam[3LL * x.blob + 1];
            lc = lam[3LL * x.blob + 2];
          }
        }
        const int gb[3] = {x.g & 1023, (x.g >> 10) & 1023, (x.g >> 20) & 1023};
        bool hit = true;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          const Ranges Rg = axis_ranges(gb[d], ts[d], te[d], G.n[d], G.P[d]);
          hit = hit && (Rg.l1 + Rg.l2 > 0);
        }
        if (hit) {
          const int slot = atomicAdd(&nhit, 1);
          hit_e[slot][0] = x.e[0];
          hit_e[slot][1] = x.e[1];
          hit_e[slot][2] = x.e[2];
          hit_g[slot] = x.g;
          hit_b[slot] = x.blob;
          hit_l[slot][0] = la;
          hit_l[slot][1] = lb;
          hit_l[slot][2] = lc;
        }
      }
    }
    __syncthreads();
    // work items (hit, stencil column): item = hit * S + pair, pair < c1 c2,
    // spread over all threads of the block
    const int nh = nhit;
    const int S = T.S;
    for (int it = tid; it < nh * S; it += NT) {
      const int h = it / S, pr = it - h * S;
      const int g = hit_g[h];
      const int gb1 = (g >> 10) & 1023, gb2 = (g >> 20) & 1023;
      const Ranges R1 = axis_ranges(gb1, ts[1], te[1], G.n[1], G.P[1]);
      const Ranges R2 = axis_ranges(gb2, ts[2], te[2], G.n[2], G.P[2]);
      const int c1 = R1.l1 + R1.l2, c2 = R2.l1 + R2.l2;
      if (pr >= c1 * c2) continue;
      const int gb0 = g & 1023;
      const Ranges R0 = axis_ranges(gb0, ts[0], te[0], G.n[0], G.P[0]);
      const int c0 = R0.l1 + R0.l2;
      const int i1 = pr / c2, i2c = pr - i1 * c2;
      const int j1 = i1 < R1.l1 ? R1.s1 + i1 : R1.s2 + (i1 - R1.l1);
      const int j2 = i2c < R2.l1 ? R2.s1 + i2c : R2.s2 + (i2c - R2.l1);
      int a1 = ts[1] + j1 - gb1;
      a1 += (a1 < 0) ? G.n[1] : 0;
      int a2 = ts[2] + j2 - gb2;
      a2 += (a2 < 0) ? G.n[2] : 0;
      const double d1 = hit_e[h][1] + a1 * G.dx[1], d2 = hit_e[h][2] + a2 * G.dx[2];
      const double d12 = d1 * d1 + d2 * d2;
      if (d12 > G.rc2) continue;
      const double e0 = hit_e[h][0];
      R s0 = 0, s1 = 0, s2 = 0;
      const R l0 = R(hit_l[h][0]), l1 = R(hit_l[h][1]), l2 = R(hit_l[h][2]);
      for (int i0 = 0; i0 < c0; ++i0) {
        const int j0 = i0 < R0.l1 ? R0.s1 + i0 : R0.s2 + (i0 - R0.l1);
        int a0 = ts[0] + j0 - gb0;
        a0 += (a0 < 0) ? G.n[0] : 0;
        const double d0 = e0 + a0 * G.dx[0];
        const double dd = d0 * d0 + d12;
        if (dd <= G.rc2) {
          const R w = wn * gexp<R>(-R(dd) * i2);
          const int q = j0 * PS + j1 * RS + j2;
          if (MODE == 0) {
            atomicAdd(acc + q, w * l0);
            atomicAdd(acc + CS + q, w * l1);
            atomicAdd(acc + 2 * CS + q, w * l2);
          } else {
            s0 += w * acc[q];
            s1 += w * acc[CS + q];
            s2 += w * acc[2 * CS + q];
          }
        }
      }
      if (MODE == 1) {
        atomicAdd(&hit_l[h][0], (double)s0);
        atomicAdd(&hit_l[h][1], (double)s1);
        atomicAdd(&hit_l[h][2], (double)s2);
      }
    }
    if (MODE == 1) {
      __syncthreads();
      for (int h = tid; h < nh; h += NT) {
        const int b = hit_b[h];
        atomicAdd(v + 3LL * b, scale * hit_l[h][0]);
        atomicAdd(v + 3LL * b + 1, scale * hit_l[h][1]);
        atomicAdd(v + 3LL * b + 2, scale * hit_l[h][2]);
      }
    }
    __syncthreads();
  }
  if (MODE == 0) {
    for (int p = tid; p < TP; p += NT) {
      const int j2 = p % T.T[2], j1 = (p / T.T[2]) % T.T[1], j0 = p / (T.T[1] * T.T[2]);
      if (j0 < te[0] && j1 < te[1] && j2 < te[2]) {
        const long long idx = ((long long)(ts[0] + j0) * G.n[1] + (ts[1] + j1)) * G.n[2] + ts[2] + j2;
        const int q = j0 * PS + j1 * RS + j2;
        f[idx] = acc[q];
        f[Gs + idx] = acc[CS + q];
        f[2 * Gs + idx] = acc[2 * CS + q];
      }
    }
  }
}

// v_i = -(U_p + Omega_p x (r_i - Y_p)) (rigid term of the saddle operator),
// or 0; the tiled averaging then adds dV J u.
__global__ void k_interp_init(const double* __restrict__ r, int M, RigidTerm K, double* __restrict__ v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= M) return;
  double o[3] = {0.0, 0.0, 0.0};
  if (K.V) {
    const int p = K.blob_body[i];
    const double* Vp = K.V + 6LL * p;
    const double rel[3] = {r[3LL * i] - K.Y[3LL * p], r[3LL * i + 1] - K.Y[3LL * p + 1], r[3LL * i + 2] - K.Y[3LL * p + 2]};
    o[0] = -(Vp[0] + (Vp[4] * rel[2] - Vp[5] * rel[1]));
    o[1] = -(Vp[1] + (Vp[5] * rel[0] - Vp[3] * rel[2]));
    o[2] = -(Vp[2] + (Vp[3] * rel[1] - Vp[4] * rel[0]));
  }
  v[3LL * i] = o[0];
  v[3LL * i + 1] = o[1];
  v[3LL * i + 2] = o[2];
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

size_t tile_record_bytes() { return sizeof(SRec); }

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

int tile_sort(const GridGeom& g, const TileGeom& t, const double* r, int M, int* tile, int* count, int* off,
              int* cursor, void* rec, int* spos, hipStream_t s) {
  GDC_TRY(fill_zero(count, ((size_t)t.ntiles * sizeof(int) + 15) / 16 * 16, s));
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

template <typename R>
size_t tile_lds_bytes(const TileGeom& t) {
  return 3 * (size_t)t.T[0] * t.T[1] * (t.T[2] + 1) * sizeof(R);
}

template <typename R>
int spread(const GridGeom& g, const TileGeom& t, const void* rec, const double* lam, const double* lam_sorted,
           const int* off, R* f, hipStream_t s) {
  if (t.T[0] > 8 || t.T[1] > 8 || t.T[2] > 32) {
    set_error("spread: tiles larger than 8 x 8 x 32");
    return GDC_EINVAL;
  }
  ProbeScope ps("spread", s);
  hipLaunchKernelGGL((k_spread_gather<R>), dim3(t.ntiles), dim3(NT), 0, s, g, t, (const SRec*)rec, off, lam,
                     lam_sorted, f);
  return check_launch("k_spread_gather");
}

template <typename R>
int interp_tiles(const GridGeom& g, const TileGeom& t, const void* rec, const int* off, const double* r,
                 const R* u, double* v, int M, double scale, const int* blob_body, const double* Y,
                 const double* V, hipStream_t s) {
  if (M <= 0) return GDC_OK;
  RigidTerm K{blob_body, Y, V};
  hipLaunchKernelGGL(k_interp_init, dim3((M + 255) / 256), dim3(256), 0, s, r, M, K, v);
  GDC_TRY(check_launch("k_interp_init"));
  hipLaunchKernelGGL((k_tile_op<R, 1>), dim3(t.ntiles), dim3(NT), tile_lds_bytes<R>(t), s, g, t, (const SRec*)rec,
                     off, (const double*)nullptr, (const double*)nullptr, (R*)nullptr, u, v, scale);
  return check_launch("k_tile_op<interp>");
}

template <typename R>
int interp(const GridGeom& g, const double* r, const R* u, double* v, int M, double scale,
           const int* blob_body, const double* Y, const double* V, hipStream_t s) {
  if (M <= 0) return GDC_OK;
  RigidTerm K{blob_body, Y, V};
  ProbeScope ps("interp", s);
  hipLaunchKernelGGL((k_interp<R>), dim3(blocks_for(M)), dim3(NT), 0, s, g, r, u, v, M, scale, K);
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

template int spread<float>(const GridGeom&, const TileGeom&, const void*, const double*, const double*, const int*,
                           float*, hipStream_t);
template int spread<double>(const GridGeom&, const TileGeom&, const void*, const double*, const double*, const int*,
                            double*, hipStream_t);
template int interp<float>(const GridGeom&, const double*, const float*, double*, int, double, const int*,
                           const double*, const double*, hipStream_t);
template int interp_tiles<float>(const GridGeom&, const TileGeom&, const void*, const int*, const double*,
                                 const float*, double*, int, double, const int*, const double*, const double*,
                                 hipStream_t);
template int interp_tiles<double>(const GridGeom&, const TileGeom&, const void*, const int*, const double*,
                                  const double*, double*, int, double, const int*, const double*, const double*,
                                  hipStream_t);
template int interp<double>(const GridGeom&, const double*, const double*, double*, int, double, const int*,
                            const double*, const double*, hipStream_t);
template int interp_fd<float>(const GridGeom&, const double*, const double*, int, const float*, double*,
                              double*, int, hipStream_t);
template int interp_fd<double>(const GridGeom&, const double*, const double*, int, const double*, double*,
                               double*, int, hipStream_t);

}  // namespace gdc
