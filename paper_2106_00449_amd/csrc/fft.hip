// Spectral Stokes solve and fluctuating-stress field on gfx950.
//
// The periodic Stokes problem of Sec. 4.2 is solved in Fourier space:
// u_hat = (I - k k^T/|k|^2) f_hat / (eta |k|^2), with the k = 0 mode and every
// mode with an index at n_d/2 removed.  The 3-D real transforms are done as
// five LDS-resident passes over lines, each a full read and write of the
// field with coalesced or 128-byte-segment access, and each pass writing its
// output transposed so that the next pass reads contiguous lines:
//
//   A  real [c][i0][i1][i2]   --R2C along axis 2-->  X [c][i0][k2][i1]
//   B  X                      --FFT along axis 1-->  Y [c][k2][k1][i0]
//   C  Y (3 components)  --FFT axis 0, project, inverse FFT axis 0-->  Y
//   B' Y                      --iFFT along axis 1--> X
//   A' X                      --C2R along axis 2-->  real
//
// Only k2 < n2/2 is stored: the Nyquist plane is zeroed by the solver, so the
// half spectrum has exactly the real field's size and the three buffers can
// ping-pong.  The random velocity field needs no forward transforms: pass C
// draws the stress spectrum from Philox counters, takes its divergence and
// projects it in place of a load (noise fused with the projection).
//
// Each 1-D transform is a Stockham autosort FFT with radix-4/2/3 stages,
// fully unrolled per line length, running on several lines per workgroup in
// LDS with twiddles e^{-2 pi i k/N} from a table computed on the host.

#include <hip/hip_ext.h>

#include "gdc_internal.h"
#include "noise_dev.h"

// No automatic multiply-add contraction in this file: every instantiation of
// a pass (each workgroup size the autotuner may pick) then performs the same
// roundings, and the transforms give the same bits whatever the launch shape.
#pragma clang fp contract(off)

#include <array>
#include <cmath>
#include <initializer_list>
#include <map>
#include <mutex>

namespace gdc {
namespace {

constexpr int NT = 256;

template <typename R>
struct Tiles {
  // Lines per workgroup in passes A, B, B', A' (128-byte segments in the
  // transposed accesses) and per component in pass C.
  static constexpr int TL = sizeof(R) == 4 ? 16 : 8;
  static constexpr int TC = sizeof(R) == 4 ? 8 : 2;
};

constexpr int next_radix(int n) {
  return (n % 4 == 0) ? 4 : (n % 2 == 0) ? 2 : (n % 3 == 0) ? 3 : 0;
}

// Radix-R DFT in registers, V[s] = sum_r v[r] w^{rs}, w = e^{-+2 pi i/R}.
template <typename R, int RAD, bool INV>
struct Bfly;

template <typename R, bool INV>
struct Bfly<R, 2, INV> {
  __device__ __forceinline__ static void run(Cx<R>* v) {
    const Cx<R> a = v[0], b = v[1];
    v[0] = Cx<R>{a.x + b.x, a.y + b.y};
    v[1] = Cx<R>{a.x - b.x, a.y - b.y};
  }
};

template <typename R, bool INV>
struct Bfly<R, 4, INV> {
  __device__ __forceinline__ static void run(Cx<R>* v) {
    const Cx<R> a{v[0].x + v[2].x, v[0].y + v[2].y};
    const Cx<R> b{v[0].x - v[2].x, v[0].y - v[2].y};
    const Cx<R> c{v[1].x + v[3].x, v[1].y + v[3].y};
    const Cx<R> d{v[1].x - v[3].x, v[1].y - v[3].y};
    v[0] = Cx<R>{a.x + c.x, a.y + c.y};
    v[2] = Cx<R>{a.x - c.x, a.y - c.y};
    if (!INV) {  // w = -i
      v[1] = Cx<R>{b.x + d.y, b.y - d.x};
      v[3] = Cx<R>{b.x - d.y, b.y + d.x};
    } else {
      v[1] = Cx<R>{b.x - d.y, b.y + d.x};
      v[3] = Cx<R>{b.x + d.y, b.y - d.x};
    }
  }
};

template <typename R, bool INV>
struct Bfly<R, 3, INV> {
  __device__ __forceinline__ static void run(Cx<R>* v) {
    constexpr R h = R(0.86602540378443864676);  // sqrt(3)/2
    const Cx<R> s{v[1].x + v[2].x, v[1].y + v[2].y};
    const Cx<R> t{v[1].x - v[2].x, v[1].y - v[2].y};
    const Cx<R> m{v[0].x - R(0.5) * s.x, v[0].y - R(0.5) * s.y};
    // forward: w = -i h t ; inverse: w = +i h t
    const Cx<R> w = INV ? Cx<R>{-h * t.y, h * t.x} : Cx<R>{h * t.y, -h * t.x};
    v[0] = Cx<R>{v[0].x + s.x, v[0].y + s.y};
    v[1] = Cx<R>{m.x + w.x, m.y + w.y};
    v[2] = Cx<R>{m.x - w.x, m.y - w.y};
  }
};

// ------------------------------------------------------------ line transforms
// A length-N line transform runs as the four-step factorisation N = A B:
//   step 1: for each b < B, an A-point DFT of x[b + B a] (a < A) in
//           registers, times w_N^{b k1}, written back to the same places;
//   step 2: for each k1 < A, a B-point DFT of the B consecutive values
//           y[B k1 + b] in registers, giving X[k1 + A k2].
// Step 1 is in place per thread; step 2 reads everything before any write.
// Three barriers per transform.  Threads take tasks line-fastest, so lanes
// walk across lines whose padded stride spreads them over the LDS banks.
// Small DFTs in registers recurse on radix 4/2/3 with twiddles read from the
// line's table (w_A^e = w_N^{e N/A}).

template <typename R, bool INV>
__device__ __forceinline__ Cx<R> twiddle(const Cx<R>* tw, int e) {
  Cx<R> w = tw[e];
  if (INV) w.y = -w.y;
  return w;
}

// cos and sin of 2 pi e / n (0 <= e < n), for twiddles whose index is known
// when the code is compiled (the in-register DFTs below, fully unrolled):
// the angle is reduced to [0, pi/4] by quarter turns and the octant
// symmetry, and the Taylor series of cos and sin there is summed in FP64 to
// far below FP64 rounding; quarter turns come out exactly 0 and +-1.
struct CosSin {
  double c, s;
};
__host__ __device__ constexpr CosSin cos_sin_turn(int e, int n) {
  e %= n;
  const int q = (4 * e) / n, r = 4 * e - q * n;   // e / n = (q + r / n) / 4
  const bool mirror = 2 * r > n;                   // past an eighth turn
  const double phi = 1.57079632679489661923 * (double)(mirror ? n - r : r) / (double)n;
  double c = 0.0, s = 0.0, tc = 1.0, ts = phi;
  for (int j = 0; j < 12; ++j) {    // terms phi^(2j) / (2j)! and phi^(2j+1) / (2j+1)!
    c += tc;
    s += ts;
    tc *= -phi * phi / (double)((2 * j + 1) * (2 * j + 2));
    ts *= -phi * phi / (double)((2 * j + 2) * (2 * j + 3));
  }
  if (mirror) {
    const double t = c;
    c = s;
    s = t;
  }
  for (int j = 0; j < q; ++j) {     // a quarter turn: (c, s) -> (-s, c)
    const double t = c;
    c = -s;
    s = t;
  }
  return CosSin{c, s};
}

// a times w_n^e = e^{-+2 pi i e/n} (forward / inverse) with e and n known at
// compile time: multiplications by 0 and +-1 are left out.
template <typename R, bool INV>
__device__ __forceinline__ Cx<R> cmul_turn(Cx<R> a, int e, int n) {
  const CosSin w = cos_sin_turn(e, n);
  const double wr = w.c, wi = INV ? w.s : -w.s;
  if (wi == 0.0) {
    if (wr == 1.0) return a;
    if (wr == -1.0) return Cx<R>{-a.x, -a.y};
  }
  if (wr == 0.0) {
    if (wi == 1.0) return Cx<R>{-a.y, a.x};
    if (wi == -1.0) return Cx<R>{a.y, -a.x};
  }
  return cmul(a, Cx<R>{R(wr), R(wi)});
}

// In-register DFT of A values v[j] (natural order in and out); tw is the
// e^{-2 pi i k/N} table of the full line length N (A divides N); the
// twiddles inside the DFT (powers of w_A) are compile-time constants.
template <typename R, int A, int N, bool INV>
struct RegDFT {
  static constexpr int RAD = next_radix(A), S = A / RAD;
  __device__ __forceinline__ static void run(Cx<R>* v, const Cx<R>* tw) {
    Cx<R> sub[RAD][S];
#pragma unroll
    for (int p = 0; p < RAD; ++p)
#pragma unroll
      for (int j = 0; j < S; ++j) sub[p][j] = v[j * RAD + p];
#pragma unroll
    for (int p = 0; p < RAD; ++p) RegDFT<R, S, N, INV>::run(sub[p], tw);
#pragma unroll
    for (int k = 0; k < S; ++k) {
      Cx<R> t[RAD];
#pragma unroll
      for (int p = 0; p < RAD; ++p)
        t[p] = (p * k == 0) ? sub[p][k] : cmul_turn<R, INV>(sub[p][k], (p * k) % A, A);
      Bfly<R, RAD, INV>::run(t);
#pragma unroll
      for (int q = 0; q < RAD; ++q) v[k + S * q] = t[q];
    }
  }
};
template <typename R, int N, bool INV>
struct RegDFT<R, 1, N, INV> {
  __device__ __forceinline__ static void run(Cx<R>*, const Cx<R>*) {}
};
template <typename R, int N, bool INV>
struct RegDFT<R, 2, N, INV> {
  __device__ __forceinline__ static void run(Cx<R>* v, const Cx<R>*) { Bfly<R, 2, INV>::run(v); }
};
template <typename R, int N, bool INV>
struct RegDFT<R, 3, N, INV> {
  __device__ __forceinline__ static void run(Cx<R>* v, const Cx<R>*) { Bfly<R, 3, INV>::run(v); }
};
template <typename R, int N, bool INV>
struct RegDFT<R, 4, N, INV> {
  __device__ __forceinline__ static void run(Cx<R>* v, const Cx<R>*) { Bfly<R, 4, INV>::run(v); }
};

// N = A B with A the largest divisor of N not above 16.
constexpr int split_a(int n) {
  int a = 1;
  for (int d = 1; d <= 16; ++d)
    if (n % d == 0) a = d;
  return a;
}

// Unnormalised forward (e^{-i}) or inverse (e^{+i}) transforms of NL lines
// of length N (line stride LS) in LDS by a workgroup of NTH threads.
template <typename R, int N, int NL, int LS, bool INV, int NTH = NT>
__device__ __forceinline__ void fft_lines(Cx<R>* buf, const Cx<R>* tw) {
  constexpr int A = split_a(N), B = N / A;
  static_assert(A * B == N, "line length");
  const int tid = threadIdx.x;
  // step 1
  for (int task = tid; task < NL * B; task += NTH) {
    const int t = task % NL, b = task / NL;
    Cx<R>* line = buf + t * LS;
    Cx<R> v[A];
#pragma unroll
    for (int a = 0; a < A; ++a) v[a] = line[b + B * a];
    RegDFT<R, A, N, INV>::run(v, tw);
#pragma unroll
    for (int k1 = 0; k1 < A; ++k1) {
      // b k1 <= (B - 1)(A - 1) < N: the index needs no reduction
      const Cx<R> w = (B > 1 && k1 > 0 && b > 0) ? cmul(v[k1], twiddle<R, INV>(tw, b * k1)) : v[k1];
      line[b + B * k1] = w;
    }
  }
  __syncthreads();
  if (B > 1) {
    constexpr int TOT = NL * A, PER = (TOT + NTH - 1) / NTH;
    Cx<R> u[PER][B];
#pragma unroll
    for (int m = 0; m < PER; ++m) {
      const int task = tid + m * NTH;
      if ((TOT % NTH == 0) || task < TOT) {
        const int t = task % NL, k1 = task / NL;
        const Cx<R>* line = buf + t * LS;
#pragma unroll
        for (int b = 0; b < B; ++b) u[m][b] = line[B * k1 + b];
        RegDFT<R, B, N, INV>::run(u[m], tw);
      }
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < PER; ++m) {
      const int task = tid + m * NTH;
      if ((TOT % NTH == 0) || task < TOT) {
        const int t = task % NL, k1 = task / NL;
        Cx<R>* line = buf + t * LS;
#pragma unroll
        for (int k2 = 0; k2 < B; ++k2) line[k1 + A * k2] = u[m][k2];
      }
    }
    __syncthreads();
  }
}

template <typename R, int N, int NTH = NT>
__device__ __forceinline__ void load_twiddles(Cx<R>* tw, const Cx<R>* __restrict__ twg) {
  for (int k = threadIdx.x; k < N; k += NTH) tw[k] = twg[k];
}

// Moves ITEMS items e = tid, tid + NTH, ... from ld(e) to st(e, value) with
// the loads of a chunk issued before any of its stores, so that a thread has
// up to 128 bytes of global loads in flight instead of one at a time.
template <int ITEMS, int NTH, typename Ld, typename St>
__device__ __forceinline__ void staged_copy(Ld ld, St st) {
  using T = decltype(ld(0));
  constexpr int PER = (ITEMS + NTH - 1) / NTH;
  constexpr int CH0 = 128 / (int)sizeof(T) > 0 ? 128 / (int)sizeof(T) : 1;
  constexpr int CH = CH0 < PER ? CH0 : PER;
  const int tid = threadIdx.x;
#pragma unroll
  for (int m0 = 0; m0 < PER; m0 += CH) {
    T v[CH];
#pragma unroll
    for (int m = 0; m < CH; ++m) {
      const int e = tid + (m0 + m) * NTH;
      if (m0 + m < PER && (ITEMS % NTH == 0 || e < ITEMS)) v[m] = ld(e);
    }
#pragma unroll
    for (int m = 0; m < CH; ++m) {
      const int e = tid + (m0 + m) * NTH;
      if (m0 + m < PER && (ITEMS % NTH == 0 || e < ITEMS)) st(e, v[m]);
    }
  }
}

// FP32 lines whose length N is a multiple of 128 move between HBM and a
// workgroup's LDS lines (stride LS) in whole-wave runs: 128 consecutive values
// of one line per wave, two per lane (one 16-byte access).  Line l of the NL
// lines sits at (l / TC) cstride + (l % TC) lstride values from g.  A run's
// line and address are wave-uniform, so the per-value index arithmetic is
// scalar.  Lines at l % TC >= nl load as zeros and are not stored.
template <int N, int NL, int TC, int LS, int NTH, bool STORE>
__device__ __forceinline__ void move_runs(Cx<float>* buf, Cx<float>* g, long long cstride, long long lstride,
                                          int nl) {
  typedef float F4 __attribute__((ext_vector_type(4)));
  constexpr int W = NTH / 64, RPL = N / 128, NR = NL * RPL, PW = NR / W;
  static_assert(N % 128 == 0 && NR % W == 0, "runs per wave");
  const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (!STORE) {
    F4 v[PW];
#pragma unroll
    for (int m = 0; m < PW; ++m) {
      const int run = wv + m * W, l = run / RPL, x = (run - l * RPL) * 128 + 2 * lane;
      const int c = l / TC, t = l - c * TC;
      v[m] = t < nl ? *reinterpret_cast<const F4*>(g + c * cstride + t * lstride + x) : F4{0.f, 0.f, 0.f, 0.f};
    }
#pragma unroll
    for (int m = 0; m < PW; ++m) {
      const int run = wv + m * W, l = run / RPL, x = (run - l * RPL) * 128 + 2 * lane;
      Cx<float>* p = buf + l * LS + x;
      p[0] = Cx<float>{v[m].x, v[m].y};
      p[1] = Cx<float>{v[m].z, v[m].w};
    }
  } else {
#pragma unroll
    for (int m = 0; m < PW; ++m) {
      const int run = wv + m * W, l = run / RPL, x = (run - l * RPL) * 128 + 2 * lane;
      const int c = l / TC, t = l - c * TC;
      if (t < nl) {
        const Cx<float>* p = buf + l * LS + x;
        const Cx<float> a = p[0], b = p[1];
        *reinterpret_cast<F4*>(g + c * cstride + t * lstride + x) = F4{a.x, a.y, b.x, b.y};
      }
    }
  }
}

// The transposed side of the axis-1 passes and of the plane projection
// (FP32, 16 lines per component and workgroup): value k of line t of
// component c sits at g[c gcs + k cs + t] (the 16 lines' values of one k are
// one 128-byte segment) and at buf[c bcs + t LS + k] in LDS.  A wave moves 4
// consecutive k of the 16 lines of one component per run, one value per lane
// (lanes across lines, as the generic loops): the lane's offset is fixed and
// a run adds a wave-uniform base.  The loads of a move go into registers
// (cols_fetch) apart from their LDS writes (cols_put), so that a workgroup
// can fetch its next block of lines while it works on the current one.
template <int N, int NC, int NTH>
struct ColsRegs {
  static constexpr int W = NTH / 64, RPC = N / 4, NR = NC * RPC, PW = NR / W;
  static_assert(N % 4 == 0 && NR % W == 0, "runs per wave");
  Cx<float> v[PW];
};

template <int N, int NC, int NTH>
__device__ __forceinline__ void cols_fetch(ColsRegs<N, NC, NTH>& r, const Cx<float>* g, int cs, long long gcs,
                                           int nl) {
  using C = ColsRegs<N, NC, NTH>;
  const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int t = lane & 15, kl = lane >> 4;
  const int goff = kl * cs + t;
  const bool in = t < nl;
#pragma unroll
  for (int m = 0; m < C::PW; ++m) {
    const int run = wv + m * C::W, c = run / C::RPC, k0 = 4 * (run - c * C::RPC);
    r.v[m] = in ? g[c * gcs + k0 * cs + goff] : Cx<float>{0.f, 0.f};
  }
}

template <int N, int NC, int LS, int NTH>
__device__ __forceinline__ void cols_put(Cx<float>* buf, const ColsRegs<N, NC, NTH>& r, int bcs) {
  using C = ColsRegs<N, NC, NTH>;
  const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int t = lane & 15, kl = lane >> 4;
#pragma unroll
  for (int m = 0; m < C::PW; ++m) {
    const int run = wv + m * C::W, c = run / C::RPC, k0 = 4 * (run - c * C::RPC);
    buf[c * bcs + t * LS + k0 + kl] = r.v[m];
  }
}

template <int N, int NC, int LS, int NTH, bool STORE>
__device__ __forceinline__ void move_cols(Cx<float>* buf, Cx<float>* g, int cs, long long gcs, int bcs, int nl) {
  constexpr int W = NTH / 64, RPC = N / 4, NR = NC * RPC, PW = NR / W;
  static_assert(N % 4 == 0 && NR % W == 0, "runs per wave");
  const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int t = lane & 15, kl = lane >> 4;
  const int goff = kl * cs + t;
  const bool in = t < nl;
  if (!STORE) {
    ColsRegs<N, NC, NTH> r;
    cols_fetch<N, NC, NTH>(r, g, cs, gcs, nl);
    cols_put<N, NC, LS, NTH>(buf, r, bcs);
  } else {
#pragma unroll
    for (int m = 0; m < PW; ++m) {
      const int run = wv + m * W, c = run / RPC, k0 = 4 * (run - c * RPC);
      if (in) g[c * gcs + k0 * cs + goff] = buf[c * bcs + t * LS + k0 + kl];
    }
  }
}

// Offset of a lane's two points in a 128-point run of a real row: point
// 128 jr + 2 lane of row i1 sits at field_col_off(i1, 128 jr) plus this (in
// the tiled layout a row's runs of 32 points are 2048 values apart).
__device__ __forceinline__ int run_lane_off(int tiled, int lane) {
  return tiled ? ((lane >> 4) << 11) + 2 * (lane & 15) : 2 * lane;
}

// ------------------------------------------------------------ pass A: R2C, axis 2
// Two real lines packed as one complex line z = a + i b; after the FFT,
// A(k) = (Z(k) + conj Z(N-k))/2 and B(k) = (Z(k) - conj Z(N-k))/(2i).
template <typename R, int N2, int NTH>
__global__ __launch_bounds__(NTH) void k_r2c_axis2(const R* __restrict__ in, Cx<R>* __restrict__ X,
                                                  const Cx<R>* __restrict__ twg, int n0, int n1, int tiled,
                                                  const int* __restrict__ skip) {
  if (skip && *skip) return;
  constexpr int TL = Tiles<R>::TL, NLc = TL / 2, LS = N2 + 1, H = N2 / 2;
  __shared__ Cx<R> buf[NLc * LS];
  __shared__ Cx<R> tw[N2];
  const int tid = threadIdx.x;
  const int c = blockIdx.z, i0 = blockIdx.y, i1b = blockIdx.x * TL;
  const int nl = min(TL, n1 - i1b);
  load_twiddles<R, N2, NTH>(tw, twg);
  const R* src = in + (long long)c * n0 * n1 * N2 + field_plane_off(tiled, n1, N2, i0);
  // items of four consecutive points of both lines of a pair (N2 is a
  // multiple of 4, and of 32 in the tiled layout: a row's runs of 32 points
  // are contiguous), one 4-vector load per line
  typedef R R4 __attribute__((ext_vector_type(4)));
  typedef R R8 __attribute__((ext_vector_type(8)));
  Cx<R>* dst = X + ((long long)c * n0 + i0) * H * n1 + i1b;
  if constexpr (sizeof(R) == 4 && N2 % 128 == 0) {
    // whole-wave runs: 128 points of both rows of a line pair per run, two
    // per lane; the transposed store of the split spectra four k (all 16
    // lines) per run, lanes across the lines
    typedef float F2 __attribute__((ext_vector_type(2)));
    constexpr int W = NTH / 64, RPL = N2 / 128, NR = NLc * RPL, PW = NR / W, PK = H / 4 / W;
    static_assert(NR % W == 0 && (H / 4) % W == 0, "runs per wave");
    const int lane = tid & 63, wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lo = run_lane_off(tiled, lane);
    F2 va[PW], vb[PW];
#pragma unroll
    for (int m = 0; m < PW; ++m) {
      const int run = wv + m * W, p = run / RPL, jr = run - p * RPL, i1 = i1b + 2 * p;
      va[m] = 2 * p < nl ? *reinterpret_cast<const F2*>(src + field_col_off(tiled, N2, i1, 128 * jr) + lo)
                         : F2{0.f, 0.f};
      vb[m] = 2 * p + 1 < nl ? *reinterpret_cast<const F2*>(src + field_col_off(tiled, N2, i1 + 1, 128 * jr) + lo)
                             : F2{0.f, 0.f};
    }
#pragma unroll
    for (int m = 0; m < PW; ++m) {
      const int run = wv + m * W, p = run / RPL, jr = run - p * RPL;
      Cx<R>* d = buf + p * LS + 128 * jr + 2 * lane;
      d[0] = Cx<R>{va[m].x, vb[m].x};
      d[1] = Cx<R>{va[m].y, vb[m].y};
    }
    __syncthreads();
    fft_lines<R, N2, NLc, LS, false, NTH>(buf, tw);
    const int t = lane & 15, kl = lane >> 4, q = t >> 1, goff = kl * n1 + t;
#pragma unroll
    for (int m = 0; m < PK; ++m) {
      const int k0 = 4 * (wv + m * W), k = k0 + kl;
      if (t < nl) {
        const Cx<R> z = buf[q * LS + k];
        const Cx<R> zc = buf[q * LS + (k == 0 ? 0 : N2 - k)];
        dst[k0 * n1 + goff] = (t & 1) ? Cx<R>{R(0.5) * (z.y + zc.y), R(0.5) * (zc.x - z.x)}
                                      : Cx<R>{R(0.5) * (z.x + zc.x), R(0.5) * (z.y - zc.y)};
      }
    }
    return;
  }
  constexpr int Q = N2 / 4;
  staged_copy<NLc * Q, NTH>(
      [&](int g) {
        const int p = g / Q, x = (g - p * Q) * 4;
        const R4 z4 = {R(0), R(0), R(0), R(0)};
        const R4 a = (2 * p < nl) ? *reinterpret_cast<const R4*>(src + field_col_off(tiled, N2, i1b + 2 * p, x)) : z4;
        const R4 b =
            (2 * p + 1 < nl) ? *reinterpret_cast<const R4*>(src + field_col_off(tiled, N2, i1b + 2 * p + 1, x)) : z4;
        return R8{a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
      },
      [&](int g, R8 v) {
        const int p = g / Q, x = (g - p * Q) * 4;
        Cx<R>* d = buf + p * LS + x;
        d[0] = Cx<R>{v.s0, v.s4};
        d[1] = Cx<R>{v.s1, v.s5};
        d[2] = Cx<R>{v.s2, v.s6};
        d[3] = Cx<R>{v.s3, v.s7};
      });
  __syncthreads();
  fft_lines<R, N2, NLc, LS, false, NTH>(buf, tw);
  for (int e = tid; e < H * TL; e += NTH) {
    const int k = e / TL, t = e - k * TL;
    if (t < nl) {
      const int p = t >> 1;
      const Cx<R> z = buf[p * LS + k];
      const Cx<R> zc = buf[p * LS + ((N2 - k) % N2)];
      Cx<R> a;
      if ((t & 1) == 0)
        a = Cx<R>{R(0.5) * (z.x + zc.x), R(0.5) * (z.y - zc.y)};
      else
        a = Cx<R>{R(0.5) * (z.y + zc.y), R(0.5) * (zc.x - z.x)};
      dst[(long long)k * n1 + t] = a;
    }
  }
}

// ------------------------------------------------------------ pass B: FFT, axis 1
template <typename R, int N1, int NTH>
__global__ __launch_bounds__(NTH) void k_fwd_axis1(const Cx<R>* __restrict__ X, Cx<R>* __restrict__ Y,
                                                  const Cx<R>* __restrict__ twg, int n0, int H,
                                                  const int* __restrict__ skip) {
  if (skip && *skip) return;
  constexpr int TL = Tiles<R>::TL, LS = N1 + 1;
  __shared__ Cx<R> buf[TL * LS];
  __shared__ Cx<R> tw[N1];
  const int tid = threadIdx.x;
  const int c = blockIdx.z, k2 = blockIdx.y, i0b = blockIdx.x * TL;
  const int nl = min(TL, n0 - i0b);
  load_twiddles<R, N1, NTH>(tw, twg);
  // line t of the workgroup starts H N1 values after line t - 1; element
  // e = t N1 + x sits at e + t (H - 1) N1 there and at e + t (LS - N1) in LDS
  const Cx<R>* Xl = X + (((long long)c * n0 + i0b) * H + k2) * N1;
  Cx<R>* Yl = Y + ((long long)c * H + k2) * N1 * n0 + i0b;
  if constexpr (sizeof(R) == 4 && N1 % 128 == 0) {
    move_runs<N1, TL, TL, LS, NTH, false>(buf, const_cast<Cx<R>*>(Xl), 0, (long long)H * N1, nl);
    __syncthreads();
    fft_lines<R, N1, TL, LS, false, NTH>(buf, tw);
    move_cols<N1, 1, LS, NTH, true>(buf, Yl, n0, 0, 0, nl);
    return;
  }
  const long long gap = (long long)(H - 1) * N1;
  staged_copy<TL * N1, NTH>(
      [&](int e) {
        const int t = e / N1;
        return (t < nl) ? Xl[e + t * gap] : Cx<R>{R(0), R(0)};
      },
      [&](int e, Cx<R> z) { buf[e + (e / N1) * (LS - N1)] = z; });
  __syncthreads();
  fft_lines<R, N1, TL, LS, false, NTH>(buf, tw);
  for (int e = tid; e < N1 * TL; e += NTH) {
    const int k1 = e / TL, t = e - k1 * TL;
    if (t < nl) Yl[(long long)k1 * n0 + t] = buf[t * LS + k1];
  }
}

// Tiles of Tiles<R>::TL lines per workgroup of the inverse axis-1 pass: two
// on the FP32 run path (the second fetched during the first's transform).
template <typename R, int N1>
constexpr int inv1_tiles() {
  return (sizeof(R) == 4 && N1 % 128 == 0) ? 2 : 1;
}

// ------------------------------------------------------------ pass B': iFFT, axis 1
template <typename R, int N1, int NTH>
__global__ __launch_bounds__(NTH) void k_inv_axis1(const Cx<R>* __restrict__ Y, Cx<R>* __restrict__ X,
                                                  const Cx<R>* __restrict__ twg, int n0, int H,
                                                  const int* __restrict__ skip) {
  if (skip && *skip) return;
  constexpr int TL = Tiles<R>::TL, LS = N1 + 1;
  __shared__ Cx<R> buf[TL * LS];
  __shared__ Cx<R> tw[N1];
  const int tid = threadIdx.x;
  const int c = blockIdx.z, k2 = blockIdx.y, i0b = blockIdx.x * TL;
  const int nl = min(TL, n0 - i0b);
  load_twiddles<R, N1, NTH>(tw, twg);
  const Cx<R>* Yl = Y + ((long long)c * H + k2) * N1 * n0 + i0b;
  Cx<R>* Xl = X + (((long long)c * n0 + i0b) * H + k2) * N1;
  if constexpr (inv1_tiles<R, N1>() == 2) {
    // two tiles of TL lines per workgroup (i0 blocks 2 x and 2 x + 1): the
    // second tile's loads go to registers before the first tile's
    // transform, so that their latency overlaps that work
    const int i0a = blockIdx.x * 2 * TL, i0c = i0a + TL;
    const int nla = min(TL, n0 - i0a), nlc = min(TL, n0 - i0c);
    const Cx<R>* Ya = Y + ((long long)c * H + k2) * N1 * n0 + i0a;
    ColsRegs<N1, 1, NTH> next;
    move_cols<N1, 1, LS, NTH, false>(buf, const_cast<Cx<R>*>(Ya), n0, 0, 0, nla);
    if (nlc > 0) cols_fetch<N1, 1, NTH>(next, Ya + TL, n0, 0, nlc);
    __syncthreads();
    fft_lines<R, N1, TL, LS, true, NTH>(buf, tw);
    move_runs<N1, TL, TL, LS, NTH, true>(buf, X + (((long long)c * n0 + i0a) * H + k2) * N1, 0, (long long)H * N1,
                                         nla);
    if (nlc <= 0) return;
    __syncthreads();
    cols_put<N1, 1, LS, NTH>(buf, next, 0);
    __syncthreads();
    fft_lines<R, N1, TL, LS, true, NTH>(buf, tw);
    move_runs<N1, TL, TL, LS, NTH, true>(buf, X + (((long long)c * n0 + i0c) * H + k2) * N1, 0, (long long)H * N1,
                                         nlc);
    return;
  }
  staged_copy<N1 * TL, NTH>(
      [&](int e) {
        const int k1 = e / TL, t = e - k1 * TL;
        return (t < nl) ? Yl[(long long)k1 * n0 + t] : Cx<R>{R(0), R(0)};
      },
      [&](int e, Cx<R> z) {
        const int k1 = e / TL, t = e - k1 * TL;
        buf[t * LS + k1] = z;
      });
  __syncthreads();
  fft_lines<R, N1, TL, LS, true, NTH>(buf, tw);
  // as the loads of pass B: element e = t N1 + x at e + t (H - 1) N1
  const long long gap = (long long)(H - 1) * N1;
  for (int e = tid; e < TL * N1; e += NTH) {
    const int t = e / N1;
    if (t < nl) Xl[e + t * gap] = buf[e + t * (LS - N1)];
  }
}

// Blocks of Tiles<R>::TL lines per workgroup of the C2R pass: two on the
// FP32 run path (the second fetched during the first's transform).
template <typename R, int N2>
constexpr int c2r_tiles() {
  return (sizeof(R) == 4 && N2 % 128 == 0) ? 2 : 1;
}

// ------------------------------------------------------------ pass A': C2R, axis 2
// Z(k) = A(k) + i B(k) with the Hermitian extension A(N-k) = conj A(k); the
// k = 0 term keeps only real parts (as a real inverse transform does) and the
// Nyquist term is zero.
template <typename R, int N2, int NTH>
__global__ __launch_bounds__(NTH) void k_c2r_axis2(const Cx<R>* __restrict__ X, R* __restrict__ out,
                                                  const Cx<R>* __restrict__ twg, int n0, int n1, int tiled,
                                                  const int* __restrict__ skip) {
  if (skip && *skip) return;
  constexpr int TL = Tiles<R>::TL, NLc = TL / 2, LS = N2 + 1, H = N2 / 2;
  __shared__ Cx<R> buf[NLc * LS];
  __shared__ Cx<R> tw[N2];
  const int tid = threadIdx.x;
  const int c = blockIdx.z, i0 = blockIdx.y, i1b = blockIdx.x * TL;
  const int nl = min(TL, n1 - i1b);
  load_twiddles<R, N2, NTH>(tw, twg);
  const Cx<R>* src = X + ((long long)c * n0 + i0) * H * n1 + i1b;
  const Cx<R> zero{R(0), R(0)};
  // the two values of an item as one native 4-vector (kept in registers)
  typedef R R4 __attribute__((ext_vector_type(4)));
  R* dst = out + (long long)c * n0 * n1 * N2 + field_plane_off(tiled, n1, N2, i0);
  if constexpr (c2r_tiles<R, N2>() == 2) {
    // the transposed load eight k (all 8 line pairs) per run, a lane's pair
    // in one 16-byte load; the real rows in whole-wave runs of 128 points of
    // both rows of a pair, two per lane.  Two blocks of TL lines per
    // workgroup (2 x and 2 x + 1 along axis 1): the second block's loads go
    // to registers before the first block's transform, so that their
    // latency overlaps that work.
    typedef float F2 __attribute__((ext_vector_type(2)));
    constexpr int W = NTH / 64, PK = H / 8 / W, RPL = N2 / 128, NR = NLc * RPL, PW = NR / W;
    static_assert((H / 8) % W == 0 && NR % W == 0, "runs per wave");
    const int lane = tid & 63, wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int q = lane & 7, kl = lane >> 3, goff = kl * n1 + 2 * q;
    const int i1a = blockIdx.x * 2 * TL, i1c = i1a + TL;
    const int nla = min(TL, n1 - i1a), nlc = min(TL, n1 - i1c);
    const Cx<R>* srca = X + ((long long)c * n0 + i0) * H * n1 + i1a;
    auto fetch = [&](R4* v, const Cx<R>* sb, int nlb) {
#pragma unroll
      for (int m = 0; m < PK; ++m) {
        const Cx<R>* sp = sb + 8 * (wv + m * W) * n1 + goff;
        v[m] = 2 * q + 1 < nlb ? *reinterpret_cast<const R4*>(sp)
                               : (2 * q < nlb ? R4{sp[0].x, sp[0].y, R(0), R(0)} : R4{R(0), R(0), R(0), R(0)});
      }
    };
    auto put = [&](const R4* v) {
#pragma unroll
      for (int m = 0; m < PK; ++m) {
        const int k = 8 * (wv + m * W) + kl;
        const Cx<R> a{v[m].x, v[m].y}, b{v[m].z, v[m].w};
        if (k == 0) {
          buf[q * LS] = Cx<R>{a.x, b.x};
          buf[q * LS + H] = zero;
        } else {
          buf[q * LS + k] = Cx<R>{a.x - b.y, a.y + b.x};
          buf[q * LS + N2 - k] = Cx<R>{a.x + b.y, b.x - a.y};
        }
      }
    };
    const int lo = run_lane_off(tiled, lane);
    auto store = [&](int i1s, int nlb) {
#pragma unroll
      for (int m = 0; m < PW; ++m) {
        const int run = wv + m * W, p = run / RPL, jr = run - p * RPL, i1 = i1s + 2 * p;
        const Cx<R>* s2 = buf + p * LS + 128 * jr + 2 * lane;
        const Cx<R> z0 = s2[0], z1 = s2[1];
        if (2 * p < nlb) *reinterpret_cast<F2*>(dst + field_col_off(tiled, N2, i1, 128 * jr) + lo) = F2{z0.x, z1.x};
        if (2 * p + 1 < nlb)
          *reinterpret_cast<F2*>(dst + field_col_off(tiled, N2, i1 + 1, 128 * jr) + lo) = F2{z0.y, z1.y};
      }
    };
    R4 va[PK], vc[PK];
    fetch(va, srca, nla);
    put(va);
    if (nlc > 0) fetch(vc, srca + TL, nlc);
    __syncthreads();
    fft_lines<R, N2, NLc, LS, true, NTH>(buf, tw);
    store(i1a, nla);
    if (nlc <= 0) return;
    __syncthreads();
    put(vc);
    __syncthreads();
    fft_lines<R, N2, NLc, LS, true, NTH>(buf, tw);
    store(i1c, nlc);
    return;
  }
  staged_copy<H * NLc, NTH>(
      [&](int e) {
        const int k = e / NLc, p = e - k * NLc;
        // select values, not references (a reference to `zero` would put it in scratch memory)
        const Cx<R> a = (2 * p < nl) ? Cx<R>(src[(long long)k * n1 + 2 * p]) : Cx<R>{R(0), R(0)};
        const Cx<R> b = (2 * p + 1 < nl) ? Cx<R>(src[(long long)k * n1 + 2 * p + 1]) : Cx<R>{R(0), R(0)};
        return R4{a.x, a.y, b.x, b.y};
      },
      [&](int e, R4 v) {
        const int k = e / NLc, p = e - k * NLc;
        const Cx<R> a{v.x, v.y}, b{v.z, v.w};
        if (k == 0) {
          buf[p * LS] = Cx<R>{a.x, b.x};
          buf[p * LS + H] = zero;
        } else {
          buf[p * LS + k] = Cx<R>{a.x - b.y, a.y + b.x};
          buf[p * LS + N2 - k] = Cx<R>{a.x + b.y, b.x - a.y};
        }
      });
  __syncthreads();
  fft_lines<R, N2, NLc, LS, true, NTH>(buf, tw);
  // four consecutive points of both lines of a pair per item, one 4-vector
  // store per line (as the loads of pass A)
  typedef R R4v __attribute__((ext_vector_type(4)));
  constexpr int Q = N2 / 4;
  for (int g = tid; g < NLc * Q; g += NTH) {
    const int p = g / Q, x = (g - p * Q) * 4;
    const Cx<R>* s4 = buf + p * LS + x;
    const Cx<R> z0 = s4[0], z1 = s4[1], z2 = s4[2], z3 = s4[3];
    if (2 * p < nl)
      *reinterpret_cast<R4v*>(dst + field_col_off(tiled, N2, i1b + 2 * p, x)) = R4v{z0.x, z1.x, z2.x, z3.x};
    if (2 * p + 1 < nl)
      *reinterpret_cast<R4v*>(dst + field_col_off(tiled, N2, i1b + 2 * p + 1, x)) = R4v{z0.y, z1.y, z2.y, z3.y};
  }
}

__global__ void k_philox_normals(uint64_t seed, uint32_t c1, uint64_t step, uint32_t c0_begin,
                                 int count, double* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  double z[4];
  four_normals(seed, c0_begin + (uint32_t)i, c1, step, z);
#pragma unroll
  for (int k = 0; k < 4; ++k) out[4 * (long long)i + k] = z[k];
}

// ------------------------------------------------------------ pass C
__device__ __forceinline__ int signed_index(int j, int n) { return j < n / 2 ? j : j - n; }

// The stress spectrum W(k) at stored mode (j0, j1, j2) (not a removed one):
// Philox normals of the canonical member of the mode's +/-k pair (the
// conjugate on the k2 = 0 plane when the mode is not canonical), scaled;
// components xx, yy, zz, xy, xz, yz.
__device__ __forceinline__ void stress_mode(const ProjParams& P, int j0, int j1, int j2, double wr[6], double wi[6]) {
  const int n0 = P.n0, n1 = P.n1;
  const int m0 = signed_index(j0, n0), m1 = signed_index(j1, n1);
  int c0 = j0, c1 = j1;
  bool conj = false;
  if (j2 == 0 && !(m1 > 0 || (m1 == 0 && m0 > 0))) {
    c0 = (n0 - j0) % n0;
    c1 = (n1 - j1) % n1;
    conj = true;
  }
  const uint32_t idx = (uint32_t)(((long long)c0 * n1 + c1) * P.n2h + j2);
  const uint64_t step = P.step_ptr ? *P.step_ptr : P.step;
  double z[12];
#pragma unroll
  for (int call = 0; call < 3; ++call) four_normals(P.seed, idx, (uint32_t)call, step, z + 4 * call);
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    const double sc = c < 3 ? P.sdiag : P.soff;
    wr[c] = sc * z[2 * c];
    wi[c] = conj ? -sc * z[2 * c + 1] : sc * z[2 * c + 1];
  }
}

// Velocity spectrum of the stress noise at stored mode (j0, j1, j2), already
// projected and scaled by 1/(eta |k|^2 G).  Returns false for removed modes.
// In the slip channel the stress is W'(k) = (W(k) + R W(k') R) / sqrt(2),
// k' = (k0, -k1, k2) the mirror mode and R W R the stress with its xy and yz
// components negated: the Fourier form of adding, in real space, the
// reflection of the stress about the walls (Sec. 6.3), which keeps the
// velocity mirror-symmetric with Cov(J u) = (2 kT/dt) M of the channel.
__device__ bool noise_mode(const ProjParams& P, int j0, int j1, int j2, double ur[3], double ui[3]) {
  const int n0 = P.n0, n1 = P.n1;
  if (j0 == n0 / 2 || j1 == n1 / 2 || (j0 == 0 && j1 == 0 && j2 == 0)) return false;
  const int m0 = signed_index(j0, n0), m1 = signed_index(j1, n1);
  double wr[6], wi[6];
  stress_mode(P, j0, j1, j2, wr, wi);
  if (P.channel) {
    double vr[6], vi[6];
    stress_mode(P, j0, (n1 - j1) % n1, j2, vr, vi);
    constexpr double h = 0.70710678118654752440;   // 1/sqrt(2)
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      const double sg = (c == 3 || c == 5) ? -1.0 : 1.0;
      wr[c] = (wr[c] + sg * vr[c]) * h;
      wi[c] = (wi[c] + sg * vi[c]) * h;
    }
  }
  const double k[3] = {P.kf0 * m0, P.kf1 * m1, P.kf2 * j2};
  // g_a = i sum_b k_b W_ab
  const double sr[3] = {k[0] * wr[0] + k[1] * wr[3] + k[2] * wr[4],
                        k[0] * wr[3] + k[1] * wr[1] + k[2] * wr[5],
                        k[0] * wr[4] + k[1] * wr[5] + k[2] * wr[2]};
  const double si[3] = {k[0] * wi[0] + k[1] * wi[3] + k[2] * wi[4],
                        k[0] * wi[3] + k[1] * wi[1] + k[2] * wi[5],
                        k[0] * wi[4] + k[1] * wi[5] + k[2] * wi[2]};
  double gr[3], gi[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    gr[a] = -si[a];
    gi[a] = sr[a];
  }
  const double k2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
  const double kgr = (k[0] * gr[0] + k[1] * gr[1] + k[2] * gr[2]) / k2;
  const double kgi = (k[0] * gi[0] + k[1] * gi[1] + k[2] * gi[2]) / k2;
  const double sc = P.inv_eta * P.invG / k2;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    ur[a] = sc * (gr[a] - k[a] * kgr);
    ui[a] = sc * (gi[a] - k[a] * kgi);
  }
  return true;
}

// The Stokes projection of the TC spectrum lines in LDS (FP32, N0 a multiple
// of 64), in whole-wave runs of 64 modes of one line: a run's j1, its k_y and
// the tests for removed modes along axis 1 are wave-uniform, and so is its
// first signed index along axis 0 when N0 is a multiple of 128 (a run then
// lies within one half of the line).  u = (c/k^2) (f - k (k.f)/k^2),
// c = 1/(eta G), with 1/k^2 from the hardware reciprocal (1 ulp); removed
// modes (Nyquist along axis 0 or 1, k = 0) and lines past n1 get a zero
// factor.
template <int N0, int TC, int LS, int NTH>
__device__ __forceinline__ void project_runs(Cx<float>* buf, const ProjParams& P, int k2, int k1b, int nl) {
  constexpr int W = NTH / 64, RPL = N0 / 64, NR = TC * RPL;
  static_assert(N0 % 64 == 0 && NR % W == 0, "runs per wave");
  const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int n1 = P.n1;
  const float fl = (float)lane, kz = float(P.kf2) * float(k2), c0 = float(P.inv_eta * P.invG);
  const float kf0 = float(P.kf0), kf1 = float(P.kf1);
#pragma unroll
  for (int m = 0; m < NR / W; ++m) {
    const int run = wv + m * W, t = run / RPL, jr = run - t * RPL, j1 = k1b + t;
    const float ky = kf1 * float(signed_index(j1, n1));
    float kx;
    bool nyq;
    if constexpr (N0 % 128 == 0) {
      const int m0 = jr < RPL / 2 ? 64 * jr : 64 * jr - N0;
      kx = kf0 * (fl + float(m0));   // the sum is an exact small integer
      nyq = lane == 0 && jr == RPL / 2;
    } else {
      const int j0 = 64 * jr + lane;
      kx = kf0 * float(j0 < N0 / 2 ? j0 : j0 - N0);
      nyq = j0 == N0 / 2;
    }
    const float kk = fused_ma(kx, kx, fused_ma(ky, ky, kz * kz));
    const bool drop = t >= nl || j1 == n1 / 2 || nyq || (lane == 0 && jr == 0 && j1 == 0 && k2 == 0);
    const float ik = drop ? 0.f : __builtin_amdgcn_rcpf(kk);
    const float s1 = c0 * ik, s2 = s1 * ik;
    Cx<float>* p = buf + t * LS + 64 * jr + lane;
    const Cx<float> f0 = p[0], f1 = p[TC * LS], f2 = p[2 * TC * LS];
    const float dr = fused_ma(kx, f0.x, fused_ma(ky, f1.x, kz * f2.x)) * s2;
    const float di = fused_ma(kx, f0.y, fused_ma(ky, f1.y, kz * f2.y)) * s2;
    p[0] = Cx<float>{fused_ma(-kx, dr, s1 * f0.x), fused_ma(-kx, di, s1 * f0.y)};
    p[TC * LS] = Cx<float>{fused_ma(-ky, dr, s1 * f1.x), fused_ma(-ky, di, s1 * f1.y)};
    p[2 * TC * LS] = Cx<float>{fused_ma(-kz, dr, s1 * f2.x), fused_ma(-kz, di, s1 * f2.y)};
  }
}

template <typename R, int N0, bool NOISE, int NTH>
__global__ __launch_bounds__(NTH) void k_axis0_project(Cx<R>* __restrict__ Y, const Cx<R>* __restrict__ twg,
                                                      ProjParams P, const int* __restrict__ skip) {
  if (skip && *skip) return;
  constexpr int TC = Tiles<R>::TC, NLn = 3 * TC, LS = N0 + 1;
  constexpr bool RUNS = sizeof(R) == 4 && N0 % 128 == 0;
  __shared__ Cx<R> buf[NLn * LS];
  __shared__ Cx<R> tw[N0];
  const int tid = threadIdx.x;
  const int k2 = blockIdx.y, k1b = blockIdx.x * TC;
  const int nl = min(TC, P.n1 - k1b);
  const int H = P.n2h, n1 = P.n1;
  load_twiddles<R, N0, NTH>(tw, twg);
  // component c's TC lines are one contiguous run of TC N0 values
  const long long cstride = (long long)H * n1 * N0;
  const Cx<R>* Yk = Y + ((long long)k2 * n1 + k1b) * N0;
  if constexpr (RUNS && !NOISE) {
    move_runs<N0, 3 * TC, TC, LS, NTH, false>(buf, Y + ((long long)k2 * n1 + k1b) * N0, cstride, N0, nl);
    __syncthreads();
    fft_lines<R, N0, NLn, LS, false, NTH>(buf, tw);
    __syncthreads();
    project_runs<N0, TC, LS, NTH>(buf, P, k2, k1b, nl);
    __syncthreads();
    fft_lines<R, N0, NLn, LS, true, NTH>(buf, tw);
    move_runs<N0, 3 * TC, TC, LS, NTH, true>(buf, Y + ((long long)k2 * n1 + k1b) * N0, cstride, N0, nl);
    return;
  }
  if (!NOISE) {
    staged_copy<NLn * N0, NTH>(
        [&](int e) {
          const int c = e / (TC * N0), r = e - c * (TC * N0);   // r = t N0 + x
          return (r < nl * N0) ? Yk[c * cstride + r] : Cx<R>{R(0), R(0)};
        },
        [&](int e, Cx<R> z) {
          // l LS + x with l = e / N0, x = e - l N0
          buf[e + (e / N0) * (LS - N0)] = z;
        });
    __syncthreads();
    fft_lines<R, N0, NLn, LS, false, NTH>(buf, tw);
  } else {
    __syncthreads();
  }
  for (int e = tid; e < TC * N0; e += NTH) {
    const int t = e / N0, j0 = e - t * N0;
    const int j1 = k1b + t;
    Cx<R> u[3] = {{R(0), R(0)}, {R(0), R(0)}, {R(0), R(0)}};
    if (t < nl) {
      if (NOISE) {
        double ur[3], ui[3];
        if (noise_mode(P, j0, j1, k2, ur, ui)) {
#pragma unroll
          for (int a = 0; a < 3; ++a) u[a] = Cx<R>{R(ur[a]), R(ui[a])};
        }
      } else if (!(j0 == N0 / 2 || j1 == n1 / 2 || (j0 == 0 && j1 == 0 && k2 == 0))) {
        const R kx = R(P.kf0) * R(signed_index(j0, N0));
        const R ky = R(P.kf1) * R(signed_index(j1, n1));
        const R kz = R(P.kf2) * R(k2);
        const R kk = kx * kx + ky * ky + kz * kz;
        const Cx<R> f0 = buf[(0 * TC + t) * LS + j0];
        const Cx<R> f1 = buf[(1 * TC + t) * LS + j0];
        const Cx<R> f2 = buf[(2 * TC + t) * LS + j0];
        const R ikk = R(1) / kk;
        const R dr = (kx * f0.x + ky * f1.x + kz * f2.x) * ikk;
        const R di = (kx * f0.y + ky * f1.y + kz * f2.y) * ikk;
        const R sc = R(P.inv_eta * P.invG) * ikk;
        u[0] = Cx<R>{sc * (f0.x - kx * dr), sc * (f0.y - kx * di)};
        u[1] = Cx<R>{sc * (f1.x - ky * dr), sc * (f1.y - ky * di)};
        u[2] = Cx<R>{sc * (f2.x - kz * dr), sc * (f2.y - kz * di)};
      }
    }
    // Each (t, j0) is read and written by the same thread only.
#pragma unroll
    for (int a = 0; a < 3; ++a) buf[(a * TC + t) * LS + j0] = u[a];
  }
  __syncthreads();
  fft_lines<R, N0, NLn, LS, true, NTH>(buf, tw);
  Cx<R>* Yo = Y + ((long long)k2 * n1 + k1b) * N0;
  if constexpr (RUNS) {
    move_runs<N0, 3 * TC, TC, LS, NTH, true>(buf, Yo, cstride, N0, nl);
  } else {
    for (int e = tid; e < NLn * N0; e += NTH) {
      const int c = e / (TC * N0), r = e - c * (TC * N0);
      if (r < nl * N0) Yo[c * cstride + r] = buf[e + (e / N0) * (LS - N0)];
    }
  }
}


// ------------------------------------------------------------ three-pass layout
// For FP32 grids with n1 = n2 <= 128 a whole (component, axis-0) plane of
// the half spectrum fits in LDS (n1 x n2/2 complex values, 66 KB at 128), so
// the two passes on each side of pass C merge into one:
//
//   P  real [c][i0][i1][i2]  --R2C axis 2, FFT axis 1-->   Z [c][i0][k2][k1]
//   C  Z (3 components)  --FFT axis 0, project, inverse FFT axis 0-->  Z
//   P' Z                     --iFFT axis 1, C2R axis 2-->   real
//
// P and P' read and write whole planes contiguously; pass C reads 16
// consecutive k1 of each (c, i0, k2) line, one 128-byte segment.


template <int N1, int N2>
struct PlaneLds {
  static constexpr int LA = N2 + 1, LB = N1 + 1;    // padded line strides
  static constexpr int H = N2 / 2;
  static constexpr int A = (N1 / 2) * LA, B = H * LB;
  static constexpr int SIZE = A > B ? A : B;
};

// Two real rows (2p, 2p+1) of length N2 as one complex line; after its FFT
// Z, row 2p has A(k) = (Z(k) + conj Z(N2-k))/2 and row 2p+1 has
// B(k) = (Z(k) - conj Z(N2-k))/(2i), k < N2/2.  Then FFT along axis 1.
template <typename R, int N1, int N2, int NTH>
__device__ __forceinline__ void plane_fwd_body(const R* __restrict__ in, Cx<R>* __restrict__ Z,
                                               const Cx<R>* __restrict__ tw1g, const Cx<R>* __restrict__ tw2g,
                                               int n0, int tiled, const int* __restrict__ skip, const BlockIx& bi) {
  if (skip && *skip) return;
  using L = PlaneLds<N1, N2>;
  constexpr int H = L::H, NP = N1 / 2;
  __shared__ Cx<R> buf[L::SIZE];
  __shared__ Cx<R> tw1[N1], tw2[N2];
  const int tid = threadIdx.x;
  const int i0 = bi.x, c = bi.y;
  load_twiddles<R, N1, NTH>(tw1, tw1g);
  load_twiddles<R, N2, NTH>(tw2, tw2g);
  const R* src = in + (long long)c * n0 * N1 * N2 + field_plane_off(tiled, N1, N2, i0);
  // four consecutive points of both rows of a pair per item (as pass A)
  typedef R R4 __attribute__((ext_vector_type(4)));
  typedef R R8 __attribute__((ext_vector_type(8)));
  constexpr int Q = N2 / 4;
  staged_copy<NP * Q, NTH>(
      [&](int g) {
        const int p = g / Q, x = (g - p * Q) * 4;
        const R4 a = *reinterpret_cast<const R4*>(src + field_col_off(tiled, N2, 2 * p, x));
        const R4 b = *reinterpret_cast<const R4*>(src + field_col_off(tiled, N2, 2 * p + 1, x));
        return R8{a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
      },
      [&](int g, R8 v) {
        const int p = g / Q, x = (g - p * Q) * 4;
        Cx<R>* d = buf + p * L::LA + x;
        d[0] = Cx<R>{v.s0, v.s4};
        d[1] = Cx<R>{v.s1, v.s5};
        d[2] = Cx<R>{v.s2, v.s6};
        d[3] = Cx<R>{v.s3, v.s7};
      });
  __syncthreads();
  fft_lines<R, N2, NP, L::LA, false, NTH>(buf, tw2);
  // unpack into lines k2 (length N1, index i1)
  constexpr int ITEMS = NP * H, PER = (ITEMS + NTH - 1) / NTH;
  Cx<R> ra[PER], rb[PER];
#pragma unroll
  for (int m = 0; m < PER; ++m) {
    const int e = tid + m * NTH;
    if (e < ITEMS) {
      const int p = e / H, k = e - p * H;
      const Cx<R> z = buf[p * L::LA + k];
      const Cx<R> zc = buf[p * L::LA + ((N2 - k) % N2)];
      ra[m] = Cx<R>{R(0.5) * (z.x + zc.x), R(0.5) * (z.y - zc.y)};
      rb[m] = Cx<R>{R(0.5) * (z.y + zc.y), R(0.5) * (zc.x - z.x)};
    }
  }
  __syncthreads();
#pragma unroll
  for (int m = 0; m < PER; ++m) {
    const int e = tid + m * NTH;
    if (e < ITEMS) {
      const int p = e / H, k = e - p * H;
      buf[k * L::LB + 2 * p] = ra[m];
      buf[k * L::LB + 2 * p + 1] = rb[m];
    }
  }
  __syncthreads();
  fft_lines<R, N1, H, L::LB, false, NTH>(buf, tw1);
  Cx<R>* dst = Z + ((long long)c * n0 + i0) * H * N1;
  // line k of element e = k N1 + x starts LB - N1 values later per line in LDS
  staged_copy<H * N1, NTH>([&](int e) { return buf[e + (e / N1) * (L::LB - N1)]; },
                           [&](int e, Cx<R> z) { dst[e] = z; });
}

// Inverse of k_plane_fwd: iFFT along axis 1, then rows (2p, 2p+1) rebuilt as
// one complex line Z(k) = A(k) + i B(k) with the Hermitian extensions (the
// k = 0 term keeps real parts, the Nyquist term is zero) and inverse FFT.
template <typename R, int N1, int N2, int NTH>
__global__ __launch_bounds__(NTH) void k_plane_fwd(const R* __restrict__ in, Cx<R>* __restrict__ Z,
                                                   const Cx<R>* __restrict__ tw1g, const Cx<R>* __restrict__ tw2g,
                                                   int n0, int tiled, const int* __restrict__ skip) {
  plane_fwd_body<R, N1, N2, NTH>(in, Z, tw1g, tw2g, n0, tiled, skip, hw_block());
}

template <typename R, int N1, int N2, int NTH>
__global__ __launch_bounds__(NTH) void k_plane_fwd_fused(const PlaneArgs* __restrict__ a,
                                                         const int* __restrict__ first, int ns) {
  const int sidx = fused_suspension(first, ns, blockIdx.x);
  const PlaneArgs& A = a[sidx];
  plane_fwd_body<R, N1, N2, NTH>((const R*)A.in, (Cx<R>*)A.out, (const Cx<R>*)A.tw1, (const Cx<R>*)A.tw2, A.n0,
                                 A.tiled, A.skip, fused_block(A.grid, (int)blockIdx.x - first[sidx]));
}

template <typename R, int N1, int N2, int NTH>
__device__ __forceinline__ void plane_inv_body(const Cx<R>* __restrict__ Z, R* __restrict__ out,
                                               const Cx<R>* __restrict__ tw1g, const Cx<R>* __restrict__ tw2g,
                                               int n0, int tiled, const int* __restrict__ skip, const BlockIx& bi) {
  if (skip && *skip) return;
  using L = PlaneLds<N1, N2>;
  constexpr int H = L::H, NP = N1 / 2;
  __shared__ Cx<R> buf[L::SIZE];
  __shared__ Cx<R> tw1[N1], tw2[N2];
  const int tid = threadIdx.x;
  const int i0 = bi.x, c = bi.y;
  load_twiddles<R, N1, NTH>(tw1, tw1g);
  load_twiddles<R, N2, NTH>(tw2, tw2g);
  const Cx<R>* src = Z + ((long long)c * n0 + i0) * H * N1;
  staged_copy<H * N1, NTH>([&](int e) { return src[e]; },
                           [&](int e, Cx<R> z) { buf[e + (e / N1) * (L::LB - N1)] = z; });
  __syncthreads();
  fft_lines<R, N1, H, L::LB, true, NTH>(buf, tw1);
  constexpr int ITEMS = NP * H, PER = (ITEMS + NTH - 1) / NTH;
  Cx<R> ra[PER], rb[PER];
#pragma unroll
  for (int m = 0; m < PER; ++m) {
    const int e = tid + m * NTH;
    if (e < ITEMS) {
      const int p = e / H, k = e - p * H;
      ra[m] = buf[k * L::LB + 2 * p];
      rb[m] = buf[k * L::LB + 2 * p + 1];
    }
  }
  __syncthreads();
  const Cx<R> zero{R(0), R(0)};
#pragma unroll
  for (int m = 0; m < PER; ++m) {
    const int e = tid + m * NTH;
    if (e < ITEMS) {
      const int p = e / H, k = e - p * H;
      const Cx<R> a = ra[m], b = rb[m];
      if (k == 0) {
        buf[p * L::LA] = Cx<R>{a.x, b.x};
        buf[p * L::LA + H] = zero;
      } else {
        buf[p * L::LA + k] = Cx<R>{a.x - b.y, a.y + b.x};
        buf[p * L::LA + N2 - k] = Cx<R>{a.x + b.y, b.x - a.y};
      }
    }
  }
  __syncthreads();
  fft_lines<R, N2, NP, L::LA, true, NTH>(buf, tw2);
  R* dst = out + (long long)c * n0 * N1 * N2 + field_plane_off(tiled, N1, N2, i0);
  // four consecutive points of both rows of a pair per item (as pass A')
  typedef R R8 __attribute__((ext_vector_type(8)));
  typedef R R4v __attribute__((ext_vector_type(4)));
  constexpr int Q = N2 / 4;
  staged_copy<NP * Q, NTH>(
      [&](int g) {
        const int p = g / Q, x = (g - p * Q) * 4;
        const Cx<R>* s4 = buf + p * L::LA + x;
        const Cx<R> z0 = s4[0], z1 = s4[1], z2 = s4[2], z3 = s4[3];
        return R8{z0.x, z1.x, z2.x, z3.x, z0.y, z1.y, z2.y, z3.y};
      },
      [&](int g, R8 v) {
        const int p = g / Q, x = (g - p * Q) * 4;
        *reinterpret_cast<R4v*>(dst + field_col_off(tiled, N2, 2 * p, x)) = R4v{v.s0, v.s1, v.s2, v.s3};
        *reinterpret_cast<R4v*>(dst + field_col_off(tiled, N2, 2 * p + 1, x)) = R4v{v.s4, v.s5, v.s6, v.s7};
      });
}

// Pass C on the plane layout Z[c][i0][k2][k1]: TCP consecutive k1 lines of
// each component per workgroup.
constexpr int TCP = 16;

template <typename R, int N1, int N2, int NTH>
__global__ __launch_bounds__(NTH) void k_plane_inv(const Cx<R>* __restrict__ Z, R* __restrict__ out,
                                                   const Cx<R>* __restrict__ tw1g, const Cx<R>* __restrict__ tw2g,
                                                   int n0, int tiled, const int* __restrict__ skip) {
  plane_inv_body<R, N1, N2, NTH>(Z, out, tw1g, tw2g, n0, tiled, skip, hw_block());
}

template <typename R, int N1, int N2, int NTH>
__global__ __launch_bounds__(NTH) void k_plane_inv_fused(const PlaneArgs* __restrict__ a,
                                                         const int* __restrict__ first, int ns) {
  const int sidx = fused_suspension(first, ns, blockIdx.x);
  const PlaneArgs& A = a[sidx];
  plane_inv_body<R, N1, N2, NTH>((const Cx<R>*)A.in, (R*)A.out, (const Cx<R>*)A.tw1, (const Cx<R>*)A.tw2, A.n0,
                                 A.tiled, A.skip, fused_block(A.grid, (int)blockIdx.x - first[sidx]));
}

template <typename R, int N0, bool NOISE, int NTH>
__device__ __forceinline__ void axis0_plane_body(Cx<R>* __restrict__ Z, const Cx<R>* __restrict__ twg,
                                                 const ProjParams& P, const int* __restrict__ skip,
                                                 const BlockIx& bi) {
  if (skip && *skip) return;
  constexpr int NLn = 3 * TCP, LS = N0 + 1;
  __shared__ Cx<R> buf[NLn * LS];
  __shared__ Cx<R> tw[N0];
  const int tid = threadIdx.x;
  const int k2 = bi.y, k1b = bi.x * TCP;
  const int nl = min(TCP, P.n1 - k1b);
  const int H = P.n2h, n1 = P.n1;
  load_twiddles<R, N0, NTH>(tw, twg);
  // element e = (c N0 + x) TCP + t: in Z at Zk[(c N0 + x) H n1 + t], in LDS
  // at (c TCP + t) LS + x
  Cx<R>* Zk = Z + (long long)k2 * n1 + k1b;
  const long long hs = (long long)H * n1;
  auto lds_at = [&](int rest, int t) { return rest + t * LS + (rest / N0) * (TCP * LS - N0); };
  // FP32 lines of a length that splits into runs: the moves in whole-wave
  // runs, and the projection in runs of 64 modes when 64 divides the length
  constexpr bool COLS = sizeof(R) == 4 && N0 % 32 == 0;
  constexpr bool PRUNS = sizeof(R) == 4 && N0 % 64 == 0;
  if constexpr (COLS && !NOISE) {
    move_cols<N0, 3, LS, NTH, false>(buf, Zk, (int)hs, N0 * hs, TCP * LS, nl);
    __syncthreads();
    fft_lines<R, N0, NLn, LS, false, NTH>(buf, tw);
  } else if (!NOISE) {
    staged_copy<NLn * N0, NTH>(
        [&](int e) {
          const int t = e % TCP, rest = e / TCP;
          return (t < nl) ? Zk[rest * hs + t] : Cx<R>{R(0), R(0)};
        },
        [&](int e, Cx<R> z) { buf[lds_at(e / TCP, e % TCP)] = z; });
    __syncthreads();
    fft_lines<R, N0, NLn, LS, false, NTH>(buf, tw);
  } else {
    __syncthreads();
  }
  if constexpr (PRUNS && !NOISE) {
    project_runs<N0, TCP, LS, NTH>(buf, P, k2, k1b, nl);
  } else {
  for (int e = tid; e < TCP * N0; e += NTH) {
    const int t = e / N0, j0 = e - t * N0;
    const int j1 = k1b + t;
    Cx<R> u[3] = {{R(0), R(0)}, {R(0), R(0)}, {R(0), R(0)}};
    if (t < nl) {
      if (NOISE) {
        double ur[3], ui[3];
        if (noise_mode(P, j0, j1, k2, ur, ui)) {
#pragma unroll
          for (int a = 0; a < 3; ++a) u[a] = Cx<R>{R(ur[a]), R(ui[a])};
        }
      } else if (!(j0 == N0 / 2 || j1 == n1 / 2 || (j0 == 0 && j1 == 0 && k2 == 0))) {
        const R kx = R(P.kf0) * R(signed_index(j0, N0));
        const R ky = R(P.kf1) * R(signed_index(j1, n1));
        const R kz = R(P.kf2) * R(k2);
        const R kk = kx * kx + ky * ky + kz * kz;
        const Cx<R> f0 = buf[(0 * TCP + t) * LS + j0];
        const Cx<R> f1 = buf[(1 * TCP + t) * LS + j0];
        const Cx<R> f2 = buf[(2 * TCP + t) * LS + j0];
        const R ikk = R(1) / kk;
        const R dr = (kx * f0.x + ky * f1.x + kz * f2.x) * ikk;
        const R di = (kx * f0.y + ky * f1.y + kz * f2.y) * ikk;
        const R sc = R(P.inv_eta * P.invG) * ikk;
        u[0] = Cx<R>{sc * (f0.x - kx * dr), sc * (f0.y - kx * di)};
        u[1] = Cx<R>{sc * (f1.x - ky * dr), sc * (f1.y - ky * di)};
        u[2] = Cx<R>{sc * (f2.x - kz * dr), sc * (f2.y - kz * di)};
      }
    }
    // Each (t, j0) is read and written by the same thread only.
#pragma unroll
    for (int a = 0; a < 3; ++a) buf[(a * TCP + t) * LS + j0] = u[a];
  }
  }
  __syncthreads();
  fft_lines<R, N0, NLn, LS, true, NTH>(buf, tw);
  if constexpr (COLS) {
    move_cols<N0, 3, LS, NTH, true>(buf, Zk, (int)hs, N0 * hs, TCP * LS, nl);
  } else {
    staged_copy<NLn * N0, NTH>([&](int e) { return buf[lds_at(e / TCP, e % TCP)]; },
                               [&](int e, Cx<R> z) {
                                 const int t = e % TCP;
                                 if (t < nl) Zk[(e / TCP) * hs + t] = z;
                               });
  }
}

template <typename R, int N0, bool NOISE, int NTH>
__global__ __launch_bounds__(NTH) void k_axis0_plane(Cx<R>* __restrict__ Z, const Cx<R>* __restrict__ twg,
                                                    ProjParams P, const int* __restrict__ skip) {
  axis0_plane_body<R, N0, NOISE, NTH>(Z, twg, P, skip, hw_block());
}

template <typename R, int N0, int NTH>
__global__ __launch_bounds__(NTH) void k_axis0_plane_fused(const ProjPlaneArgs* __restrict__ a,
                                                           const int* __restrict__ first, int ns) {
  const int sidx = fused_suspension(first, ns, blockIdx.x);
  const ProjPlaneArgs& A = a[sidx];
  axis0_plane_body<R, N0, false, NTH>((Cx<R>*)A.Z, (const Cx<R>*)A.tw, A.P, A.skip,
                                      fused_block(A.grid, (int)blockIdx.x - first[sidx]));
}

// ------------------------------------------------------------ dispatch

#define GDC_FFT_SIZES(X) X(8) X(12) X(16) X(24) X(32) X(48) X(64) X(96) X(128) X(192) X(256) X(384)

// Every pass takes its workgroup size (threads) at run time from the grid's
// FftShape; the instantiated sizes are 256 and 512 (and 1024 for the plane
// passes).  The size only changes how the same line transforms are shared
// out, so every choice gives the same results bit for bit.
bool nth_ok(int nth, bool allow_1024) {
  if (nth == 256 || nth == 512 || (allow_1024 && nth == 1024)) return true;
  set_error("unsupported FFT workgroup size");
  return false;
}

template <typename R>
int launch_r2c(int n2, const R* in, Cx<R>* X, const Cx<R>* tw, int n0, int n1, int tiled, int nth, hipStream_t s,
               const int* skip) {
  if (!nth_ok(nth, false)) return GDC_EINVAL;
  dim3 grid((n1 + Tiles<R>::TL - 1) / Tiles<R>::TL, n0, 3);
  const ProbeEvents pe = probe_claim("fft_r2c");
#define L_(N, T) GDC_LAUNCH_PROBED((k_r2c_axis2<R, N, T>), grid, dim3(T), 0, s, pe, in, X, tw, n0, n1, tiled, skip)
  switch (n2) {
#define X_(N) case N: if (nth == 512) L_(N, 512); else L_(N, 256); break;
    GDC_FFT_SIZES(X_)
#undef X_
    default: set_error("unsupported grid size"); return GDC_EINVAL;
  }
#undef L_
  return check_launch("k_r2c_axis2");
}

template <typename R>
int launch_fwd1(int n1, const Cx<R>* X, Cx<R>* Y, const Cx<R>* tw, int n0, int H, int nth, hipStream_t s,
                const int* skip) {
  if (!nth_ok(nth, false)) return GDC_EINVAL;
  dim3 grid((n0 + Tiles<R>::TL - 1) / Tiles<R>::TL, H, 3);
  const ProbeEvents pe = probe_claim("fft_fwd1");
#define L_(N, T) GDC_LAUNCH_PROBED((k_fwd_axis1<R, N, T>), grid, dim3(T), 0, s, pe, X, Y, tw, n0, H, skip)
  switch (n1) {
#define X_(N) case N: if (nth == 512) L_(N, 512); else L_(N, 256); break;
    GDC_FFT_SIZES(X_)
#undef X_
    default: set_error("unsupported grid size"); return GDC_EINVAL;
  }
#undef L_
  return check_launch("k_fwd_axis1");
}

template <typename R>
int launch_inv1(int n1, const Cx<R>* Y, Cx<R>* X, const Cx<R>* tw, int n0, int H, int nth, hipStream_t s,
                const int* skip) {
  if (!nth_ok(nth, false)) return GDC_EINVAL;
  const int tiles = (n0 + Tiles<R>::TL - 1) / Tiles<R>::TL;
  const ProbeEvents pe = probe_claim("fft_inv1");
#define L_(N, T)                                                                                           \
  GDC_LAUNCH_PROBED((k_inv_axis1<R, N, T>), dim3((tiles + inv1_tiles<R, N>() - 1) / inv1_tiles<R, N>(), H, 3), \
                    dim3(T), 0, s, pe, Y, X, tw, n0, H, skip)
  switch (n1) {
#define X_(N) case N: if (nth == 512) L_(N, 512); else L_(N, 256); break;
    GDC_FFT_SIZES(X_)
#undef X_
    default: set_error("unsupported grid size"); return GDC_EINVAL;
  }
#undef L_
  return check_launch("k_inv_axis1");
}

template <typename R>
int launch_c2r(int n2, const Cx<R>* X, R* out, const Cx<R>* tw, int n0, int n1, int tiled, int nth, hipStream_t s,
               const int* skip) {
  if (!nth_ok(nth, false)) return GDC_EINVAL;
  const int tiles = (n1 + Tiles<R>::TL - 1) / Tiles<R>::TL;
  const ProbeEvents pe = probe_claim("fft_c2r");
#define L_(N, T)                                                                                          \
  GDC_LAUNCH_PROBED((k_c2r_axis2<R, N, T>), dim3((tiles + c2r_tiles<R, N>() - 1) / c2r_tiles<R, N>(), n0, 3), \
                    dim3(T), 0, s, pe, X, out, tw, n0, n1, tiled, skip)
  switch (n2) {
#define X_(N) case N: if (nth == 512) L_(N, 512); else L_(N, 256); break;
    GDC_FFT_SIZES(X_)
#undef X_
    default: set_error("unsupported grid size"); return GDC_EINVAL;
  }
#undef L_
  return check_launch("k_c2r_axis2");
}

template <typename R, bool NOISE>
int launch_proj(int n0, Cx<R>* Y, const Cx<R>* tw, const ProjParams& P, int nth, hipStream_t s, const int* skip) {
  if (!nth_ok(nth, false)) return GDC_EINVAL;
  dim3 grid((P.n1 + Tiles<R>::TC - 1) / Tiles<R>::TC, P.n2h, 1);
  const ProbeEvents pe = probe_claim(NOISE ? "fft_noise" : "fft_project");
#define L_(N, T) GDC_LAUNCH_PROBED((k_axis0_project<R, N, NOISE, T>), grid, dim3(T), 0, s, pe, Y, tw, P, skip)
  switch (n0) {
#define X_(N) case N: if (nth == 512) L_(N, 512); else L_(N, 256); break;
    GDC_FFT_SIZES(X_)
#undef X_
    default: set_error("unsupported grid size"); return GDC_EINVAL;
  }
#undef L_
  return check_launch("k_axis0_project");
}


// Plane sizes: n1 = n2 and n0 in this list (FP32 only).
#define GDC_PLANE_SIZES(X) X(8) X(12) X(16) X(24) X(32) X(48) X(64) X(96) X(128)

bool plane_size(int n) {
  switch (n) {
#define X_(N) case N: return true;
    GDC_PLANE_SIZES(X_)
#undef X_
    default: return false;
  }
}

template <typename R>
bool plane_path(const GridGeom& g) {
  return sizeof(R) == 4 && g.n[1] == g.n[2] && plane_size(g.n[1]) && plane_size(g.n[0]);
}

template <typename R>
int launch_plane(bool inverse, int n, const void* in, void* out, const Cx<R>* tw1, const Cx<R>* tw2, int n0,
                 int tiled, int nth, hipStream_t s, const int* skip) {
  if (!nth_ok(nth, true)) return GDC_EINVAL;
  dim3 grid(n0, 3);
  const ProbeEvents pe = probe_claim(inverse ? "fft_plane_inv" : "fft_plane_fwd");
  if constexpr (sizeof(R) != 4) {
    set_error("plane transforms are FP32 only");
    return GDC_EINVAL;
  } else {
    if (!inverse) {
#define L_(N, T) GDC_LAUNCH_PROBED((k_plane_fwd<R, N, N, T>), grid, dim3(T), 0, s, pe, (const R*)in, (Cx<R>*)out, tw1, tw2, n0, tiled, skip)
      switch (n) {
#define X_(N) case N: if (nth == 1024) L_(N, 1024); else if (nth == 512) L_(N, 512); else L_(N, 256); break;
        GDC_PLANE_SIZES(X_)
#undef X_
        default: set_error("unsupported plane size"); return GDC_EINVAL;
      }
#undef L_
      return check_launch("k_plane_fwd");
    }
#define L_(N, T) GDC_LAUNCH_PROBED((k_plane_inv<R, N, N, T>), grid, dim3(T), 0, s, pe, (const Cx<R>*)in, (R*)out, tw1, tw2, n0, tiled, skip)
    switch (n) {
#define X_(N) case N: if (nth == 1024) L_(N, 1024); else if (nth == 512) L_(N, 512); else L_(N, 256); break;
      GDC_PLANE_SIZES(X_)
#undef X_
      default: set_error("unsupported plane size"); return GDC_EINVAL;
    }
#undef L_
    return check_launch("k_plane_inv");
  }
}

template <typename R, bool NOISE>
int launch_proj_plane(int n0, Cx<R>* Z, const Cx<R>* tw, const ProjParams& P, int nth, hipStream_t s,
                      const int* skip) {
  if (!nth_ok(nth, false)) return GDC_EINVAL;
  dim3 grid((P.n1 + TCP - 1) / TCP, P.n2h, 1);
  const ProbeEvents pe = probe_claim(NOISE ? "fft_noise" : "fft_project");
  if constexpr (sizeof(R) != 4) {
    set_error("plane transforms are FP32 only");
    return GDC_EINVAL;
  } else {
#define L_(N, T) GDC_LAUNCH_PROBED((k_axis0_plane<R, N, NOISE, T>), grid, dim3(T), 0, s, pe, Z, tw, P, skip)
    switch (n0) {
#define X_(N) case N: if (nth == 512) L_(N, 512); else L_(N, 256); break;
      GDC_PLANE_SIZES(X_)
#undef X_
      default: set_error("unsupported grid size"); return GDC_EINVAL;
    }
#undef L_
    return check_launch("k_axis0_plane");
  }
}

ProjParams proj_params(const GridGeom& g) {
  ProjParams P{};
  P.n0 = g.n[0];
  P.n1 = g.n[1];
  P.n2h = g.n2h;
  constexpr double kTwoPi = 6.283185307179586476925;
  P.kf0 = kTwoPi / g.L[0];
  P.kf1 = kTwoPi / g.L[1];
  P.kf2 = kTwoPi / g.L[2];
  P.inv_eta = 1.0 / g.eta;
  P.invG = 1.0 / (double)g.G;
  return P;
}

}  // namespace

bool fft_size_supported(int n) {
  switch (n) {
#define X_(N) case N: return true;
    GDC_FFT_SIZES(X_)
#undef X_
    default: return false;
  }
}

template <typename R>
int stokes_solve(const GridGeom& g, const Cx<R>* const tw[3], R* real, Cx<R>* X, Cx<R>* Y,
                 hipStream_t s, const int* skip) {
  const int n0 = g.n[0], n1 = g.n[1], n2 = g.n[2], H = g.n2h;
  const FftShape& f = g.fft;
  if (plane_path<R>(g)) {
    GDC_TRY(launch_plane<R>(false, n1, real, X, tw[1], tw[2], n0, g.tiled, f.plane_fwd, s, skip));
    GDC_TRY((launch_proj_plane<R, false>(n0, X, tw[0], proj_params(g), f.proj_plane, s, skip)));
    return launch_plane<R>(true, n1, X, real, tw[1], tw[2], n0, g.tiled, f.plane_inv, s, skip);
  }
  GDC_TRY(launch_r2c<R>(n2, real, X, tw[2], n0, n1, g.tiled, f.r2c, s, skip));
  GDC_TRY(launch_fwd1<R>(n1, X, Y, tw[1], n0, H, f.fwd1, s, skip));
  GDC_TRY((launch_proj<R, false>(n0, Y, tw[0], proj_params(g), f.proj, s, skip)));
  GDC_TRY(launch_inv1<R>(n1, Y, X, tw[1], n0, H, f.inv1, s, skip));
  GDC_TRY(launch_c2r<R>(n2, X, real, tw[2], n0, n1, g.tiled, f.c2r, s, skip));
  return GDC_OK;
}

bool stokes_fusable(const GridGeom& g, int precision) {
  return precision != GDC_FP64 && plane_path<float>(g);
}

void stokes_describe(StokesArgs& a, const GridGeom& g, const void* const tw[3], void* real, void* X,
                     const int* skip) {
  const int n0 = g.n[0];
  a.fwd = PlaneArgs{real, X, tw[1], tw[2], n0, g.tiled, skip, LocalGrid{n0, 3, 1}};
  a.proj = ProjPlaneArgs{X, tw[0], proj_params(g), skip, LocalGrid{(g.n[1] + TCP - 1) / TCP, g.n2h, 1}};
  a.inv = PlaneArgs{X, real, tw[1], tw[2], n0, g.tiled, skip, LocalGrid{n0, 3, 1}};
}

int stokes_fused(const GridGeom& g, const PlaneArgs* fwd, const ProjPlaneArgs* proj, const PlaneArgs* inv, int ns,
                 const int* first_plane, int tot_plane, const int* first_proj, int tot_proj, hipStream_t s) {
  if (ns <= 0) return GDC_OK;
  using R = float;
  const FftShape& f = g.fft;
  const int n = g.n[1];
  if (!plane_path<R>(g) || !nth_ok(f.plane_fwd, true) || !nth_ok(f.plane_inv, true) || !nth_ok(f.proj_plane, false))
    return GDC_EINVAL;
  const dim3 gp(tot_plane), gq(tot_proj);
#define L_(K, N, T, ARGS, FIRST) hipLaunchKernelGGL((K<R, N, N, T>), (FIRST == first_plane ? gp : gq), dim3(T), 0, s, ARGS, FIRST, ns)
#define SW_(K, NTH, ARGS, FIRST)                                                        \
  switch (n) {                                                                          \
    GDC_PLANE_SIZES(X_)                                                                 \
    default: set_error("unsupported plane size"); return GDC_EINVAL;                    \
  }
#define X_(N) case N: if (f.plane_fwd == 1024) L_(k_plane_fwd_fused, N, 1024, fwd, first_plane); \
                      else if (f.plane_fwd == 512) L_(k_plane_fwd_fused, N, 512, fwd, first_plane); \
                      else L_(k_plane_fwd_fused, N, 256, fwd, first_plane); break;
  SW_(k_plane_fwd_fused, f.plane_fwd, fwd, first_plane)
#undef X_
  GDC_TRY(check_launch("k_plane_fwd_fused"));
#define X_(N) case N: if (f.proj_plane == 512) hipLaunchKernelGGL((k_axis0_plane_fused<R, N, 512>), gq, dim3(512), 0, s, proj, first_proj, ns); \
                      else hipLaunchKernelGGL((k_axis0_plane_fused<R, N, 256>), gq, dim3(256), 0, s, proj, first_proj, ns); break;
  SW_(k_axis0_plane_fused, f.proj_plane, proj, first_proj)
#undef X_
  GDC_TRY(check_launch("k_axis0_plane_fused"));
#define X_(N) case N: if (f.plane_inv == 1024) L_(k_plane_inv_fused, N, 1024, inv, first_plane); \
                      else if (f.plane_inv == 512) L_(k_plane_inv_fused, N, 512, inv, first_plane); \
                      else L_(k_plane_inv_fused, N, 256, inv, first_plane); break;
  SW_(k_plane_inv_fused, f.plane_inv, inv, first_plane)
#undef X_
#undef SW_
#undef L_
  return check_launch("k_plane_inv_fused");
}

template <typename R>
int fluct_field(const GridGeom& g, const Cx<R>* const tw[3], R* real, Cx<R>* X, Cx<R>* Y,
                uint64_t seed, uint64_t step, double kT, double dt, hipStream_t s, const uint64_t* step_ptr) {
  const int n0 = g.n[0], n1 = g.n[1], n2 = g.n[2], H = g.n2h;
  const FftShape& f = g.fft;
  ProjParams P = proj_params(g);
  P.seed = seed;
  P.step = step;
  P.step_ptr = step_ptr;
  // real-space variances 4 kT eta/(dV dt) (diagonal) and 2 kT eta/(dV dt)
  // (off-diagonal) of the stress at a grid point; per stored mode, real and
  // imaginary parts each carry G var / 2.
  const double base = kT * g.eta / (g.dV * dt);
  P.sdiag = std::sqrt((double)g.G * 4.0 * base / 2.0);
  P.soff = std::sqrt((double)g.G * 2.0 * base / 2.0);
  P.channel = g.channel;
  if (plane_path<R>(g)) {
    GDC_TRY((launch_proj_plane<R, true>(n0, X, tw[0], P, f.proj_plane, s, nullptr)));
    return launch_plane<R>(true, n1, X, real, tw[1], tw[2], n0, g.tiled, f.plane_inv, s, nullptr);
  }
  GDC_TRY((launch_proj<R, true>(n0, Y, tw[0], P, f.proj, s, nullptr)));
  GDC_TRY(launch_inv1<R>(n1, Y, X, tw[1], n0, H, f.inv1, s, nullptr));
  GDC_TRY(launch_c2r<R>(n2, X, real, tw[2], n0, n1, g.tiled, f.c2r, s, nullptr));
  return GDC_OK;
}

// Autotuner: for every pass of this grid's transform, time each workgroup
// size (one warm-up launch, then the mean of three) on the handle's own
// buffers and keep the fastest.  The buffers are zeroed first; the choice is
// cached per (grid, precision) for the process.
namespace {
template <typename F>
int time_launches(hipStream_t s, F launch, float& us) {
  hipEvent_t a = nullptr, b = nullptr;
  GDC_HIP(hipEventCreate(&a));
  GDC_HIP(hipEventCreate(&b));
  int rc = launch();
  if (rc == GDC_OK && hipEventRecord(a, s) != hipSuccess) rc = GDC_EDEVICE;
  for (int k = 0; k < 3 && rc == GDC_OK; ++k) rc = launch();
  if (rc == GDC_OK && hipEventRecord(b, s) != hipSuccess) rc = GDC_EDEVICE;
  float ms = 0.f;
  if (rc == GDC_OK && (hipEventSynchronize(b) != hipSuccess || hipEventElapsedTime(&ms, a, b) != hipSuccess))
    rc = GDC_EDEVICE;
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (rc == GDC_EDEVICE) set_error("autotuner timing failed");
  us = ms * 1e3f / 3.f;
  return rc;
}

// Two rounds over the sizes, interleaved, keeping each size's faster round:
// a transient slowdown of one measurement does not decide the pick.
template <typename F>
int pick(hipStream_t s, std::initializer_list<int> sizes, F launch_with, int& best) {
  constexpr int MAXS = 4;
  float t[MAXS] = {0.f, 0.f, 0.f, 0.f};
  for (int round = 0; round < 2; ++round) {
    int i = 0;
    for (int nth : sizes) {
      float us = 0.f;
      GDC_TRY(time_launches(s, [&] { return launch_with(nth); }, us));
      if (i < MAXS) t[i] = round == 0 ? us : (us < t[i] ? us : t[i]);
      ++i;
    }
  }
  float best_us = 0.f;
  best = 0;
  int i = 0;
  for (int nth : sizes) {
    if (i < MAXS && (best == 0 || t[i] < best_us)) {
      best = nth;
      best_us = t[i];
    }
    ++i;
  }
  return GDC_OK;
}

std::mutex g_tune_mutex;
std::map<std::array<int, 4>, FftShape> g_tuned;
}  // namespace

template <typename R>
int fft_autotune(GridGeom& g, const Cx<R>* const tw[3], R* real, Cx<R>* X, Cx<R>* Y, hipStream_t s) {
  const std::array<int, 4> key{g.n[0], g.n[1], g.n[2], (int)sizeof(R)};
  {
    std::lock_guard<std::mutex> lk(g_tune_mutex);
    auto it = g_tuned.find(key);
    if (it != g_tuned.end()) {
      g.fft = it->second;
      return GDC_OK;
    }
  }
  const int n0 = g.n[0], n1 = g.n[1], n2 = g.n[2], H = g.n2h;
  GDC_TRY(fill_zero(real, 3 * (size_t)g.G * sizeof(R), s));
  GDC_TRY(fill_zero(X, 3 * (size_t)g.G * sizeof(R), s));
  GDC_TRY(fill_zero(Y, 3 * (size_t)g.G * sizeof(R), s));
  FftShape f = g.fft;
  const ProjParams P = proj_params(g);
  if (plane_path<R>(g)) {
    GDC_TRY(pick(s, {256, 512, 1024}, [&](int t) {
      return launch_plane<R>(false, n1, real, X, tw[1], tw[2], n0, g.tiled, t, s, nullptr); }, f.plane_fwd));
    GDC_TRY(pick(s, {256, 512}, [&](int t) {
      return launch_proj_plane<R, false>(n0, X, tw[0], P, t, s, nullptr); }, f.proj_plane));
    GDC_TRY(pick(s, {256, 512, 1024}, [&](int t) {
      return launch_plane<R>(true, n1, X, real, tw[1], tw[2], n0, g.tiled, t, s, nullptr); }, f.plane_inv));
  } else {
    GDC_TRY(pick(s, {256, 512}, [&](int t) {
      return launch_r2c<R>(n2, real, X, tw[2], n0, n1, g.tiled, t, s, nullptr); }, f.r2c));
    GDC_TRY(pick(s, {256, 512}, [&](int t) { return launch_fwd1<R>(n1, X, Y, tw[1], n0, H, t, s, nullptr); },
                 f.fwd1));
    GDC_TRY(pick(s, {256, 512}, [&](int t) {
      return launch_proj<R, false>(n0, Y, tw[0], P, t, s, nullptr); }, f.proj));
    GDC_TRY(pick(s, {256, 512}, [&](int t) { return launch_inv1<R>(n1, Y, X, tw[1], n0, H, t, s, nullptr); },
                 f.inv1));
    GDC_TRY(pick(s, {256, 512}, [&](int t) {
      return launch_c2r<R>(n2, X, real, tw[2], n0, n1, g.tiled, t, s, nullptr); }, f.c2r));
  }
  g.fft = f;
  std::lock_guard<std::mutex> lk(g_tune_mutex);
  g_tuned[key] = f;
  return GDC_OK;
}

int philox_normals_dev(uint64_t seed, uint32_t c1, uint64_t step, uint32_t c0_begin, int count,
                       double* out_dev, hipStream_t s) {
  if (count <= 0) return GDC_OK;
  hipLaunchKernelGGL(k_philox_normals, dim3((count + 255) / 256), dim3(256), 0, s, seed, c1, step,
                     c0_begin, count, out_dev);
  return check_launch("k_philox_normals");
}

template int stokes_solve<float>(const GridGeom&, const Cx<float>* const[3], float*, Cx<float>*,
                                   Cx<float>*, hipStream_t, const int*);
template int stokes_solve<double>(const GridGeom&, const Cx<double>* const[3], double*, Cx<double>*,
                                   Cx<double>*, hipStream_t, const int*);
template int fluct_field<float>(const GridGeom&, const Cx<float>* const[3], float*, Cx<float>*,
                                Cx<float>*, uint64_t, uint64_t, double, double, hipStream_t, const uint64_t*);
template int fluct_field<double>(const GridGeom&, const Cx<double>* const[3], double*, Cx<double>*,
                                 Cx<double>*, uint64_t, uint64_t, double, double, hipStream_t,
                                 const uint64_t*);
template int fft_autotune<float>(GridGeom&, const Cx<float>* const[3], float*, Cx<float>*, Cx<float>*,
                                 hipStream_t);
template int fft_autotune<double>(GridGeom&, const Cx<double>* const[3], double*, Cx<double>*, Cx<double>*,
                                  hipStream_t);

}  // namespace gdc
