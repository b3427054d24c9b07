// Per-body kernels of the gDC step and of the rigid saddle-point operator
// (Sec. 2.2, Sec. 3), FP64 throughout.
//
// Body-frame tables are built once per shape on the host: (K^T K)^+, the
// projector onto null(K) (spin of a straight rod, rotation of a one-blob
// body), and the inverse of the block preconditioner.  K, M's RPY self block
// and the least-squares operator are covariant under rotation, so in the lab
// frame a body only needs R(q): (K^T K)^+_lab = Q^T (K^T K)^+_body Q with
// Q = diag(R^T, R^T), and likewise for the other tables.

#include "gdc_internal.h"
#include "noise_dev.h"

namespace gdc {
namespace {

constexpr int NT = 256;

inline unsigned nblk(long long n, int nt = NT) { return (unsigned)((n + nt - 1) / nt); }

__device__ __forceinline__ void load3(const double* p, double* x) {
  x[0] = p[0];
  x[1] = p[1];
  x[2] = p[2];
}

// y = Q^T A Q x for a body-frame 6x6 A (row-major), Q = diag(R^T, R^T).
__device__ void rotate_6x6(const double* A, const double* R, const double* x, double* y) {
  double xb[6], yb[6];
  matTvec3(R, x, xb);
  matTvec3(R, x + 3, xb + 3);
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < 6; ++j) s += A[6 * i + j] * xb[j];
    yb[i] = s;
  }
  matvec3(R, yb, y);
  matvec3(R, yb + 3, y + 3);
}

// ------------------------------------------------------------ geometry

__global__ void k_blob_positions(BodyTables B, const double* __restrict__ Y, const double* __restrict__ q,
                                 double* __restrict__ r) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= B.M) return;
  const int p = B.blob_body[i], s = B.body_shape[p];
  double R[9], b[3], x[3];
  rotmat(q + 4LL * p, R);
  load3(B.shape_b + 3LL * (B.shape_boff[s] + B.blob_local[i]), b);
  matvec3(R, b, x);
  r[3LL * i] = Y[3LL * p] + x[0];
  r[3LL * i + 1] = Y[3LL * p + 1] + x[1];
  r[3LL * i + 2] = Y[3LL * p + 2] + x[2];
}

// ------------------------------------------------------------ block preconditioner
// One wavefront per body: gather (x_i for its blobs, x_V), rotate to the body
// frame, multiply by the shape's dense inverse of [[M_RPY, -K], [-K^T, -Pi]]
// (stored transposed, so lanes read consecutive entries), rotate back.  When
// yV is given the same kernel also forms the body rows of the saddle operator
// at z = P^-1 x, yV = -K^T z_lam - Pi z_V, in the body frame (K, Pi are
// rotation covariant) before rotating them to the lab frame.
typedef double dbl4 __attribute__((ext_vector_type(4)));

// The same preconditioner on the matrix cores: one workgroup (4 waves) per
// group of up to 16 bodies of one shape, each wave one 16-row block.  The body-frame vectors x_b = Q^T x of the group
// are the columns of X (D x 16, LDS); Y = P_s^-1 X by FP64 MFMA
// (v_mfma_f64_16x16x4f64: 16-row blocks of P_s^-1, K in steps of 4; lane l
// passes A[16 rb + l % 16][4 t + l / 16] and X[4 t + l / 16][l % 16] and gets
// Y[16 rb + l / 16 + 4 r][l % 16], r < 4); then rotated back and scattered
// exactly as k_precond does.  D = 3 n_b + 6 <= PREC_MFMA_MAXDIM.
__device__ __forceinline__ void precond_mfma_body(const BodyTables& B, const double* __restrict__ q,
                                                  const double* __restrict__ x, double* __restrict__ z,
                                                  double* __restrict__ yV, const int* __restrict__ spos,
                                                  double* __restrict__ zs, const int* __restrict__ skip,
                                                  int mirror, const BlockIx& bi) {
  if (skip && *skip) return;
  constexpr int DP = PREC_MFMA_MAXDIM;
  __shared__ double X[DP][16];
  __shared__ double Yl[DP][16];
  __shared__ double As[DP * DP];   // the shape's block, staged once
  __shared__ double Rm[16][9];
  __shared__ double Tb[16][6];
  __shared__ int pb[16];
  const int g = bi.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int s = B.group_shape[g], first = B.group_first[g], cnt = B.group_count[g];
  const int off_s = B.shape_boff[s], nb = B.shape_boff[s + 1] - off_s;
  const int D = 3 * nb + 6, nv = nb + 2;
  const long long Mx3 = 3LL * B.M;
  // the shape's block first: its loads do not depend on the bodies, so they
  // are in flight while the body indices, orientations and vectors arrive
  const double* AT = B.shape_precT + B.shape_prec_off[s];   // AT[k D + i] = (P_s^-1)[i][k]
  for (int e0 = 0; e0 < D * D; e0 += 8 * 256) {   // eight loads per thread in flight
    double v[8];
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      const int e = e0 + tid + 256 * m;
      v[m] = e < D * D ? AT[e] : 0.0;
    }
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      const int e = e0 + tid + 256 * m;
      if (e < D * D) As[e] = v[m];
    }
  }
  if (tid < 16) {
    const int p = tid < cnt ? B.group_body[first + tid] : -1;
    pb[tid] = p;
    if (p >= 0) rotmat(q + 4LL * p, &Rm[tid][0]);
  }
  __syncthreads();
  for (int t = tid; t < nv * 16; t += 256) {
    const int v = t >> 4, j = t & 15;
    const int p = pb[j];
    double w[3] = {0.0, 0.0, 0.0};
    if (p >= 0) {
      const double* src = v < nb ? x + 3LL * (B.body_off[p] + v) : x + Mx3 + 6LL * p + 3 * (v - nb);
      double xv[3];
      load3(src, xv);
      matTvec3(&Rm[j][0], xv, w);
    }
    X[3 * v][j] = w[0];
    X[3 * v + 1][j] = w[1];
    X[3 * v + 2][j] = w[2];
  }
  for (int t = tid; t < (DP - D) * 16; t += 256) X[D + (t >> 4)][t & 15] = 0.0;
  __syncthreads();
  const int il = lane & 15, kq = lane >> 4;
  const int nrb = (D + 15) / 16, nk = (D + 3) / 4;
  for (int rb = wave; rb < nrb; rb += 4) {   // one 16-row block per wave
    dbl4 acc = {0.0, 0.0, 0.0, 0.0};
    const int i = 16 * rb + il;
    for (int t = 0; t < nk; ++t) {
      const int k = 4 * t + kq;
      const double a = (i < D && k < D) ? As[k * D + i] : 0.0;
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, X[k][il], acc, 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) Yl[16 * rb + kq + 4 * r][il] = acc[r];
  }
  __syncthreads();
  for (int t = tid; t < nv * 16; t += 256) {
    const int v = t >> 4, j = t & 15;
    const int p = pb[j];
    if (p < 0) continue;
    const double yv[3] = {Yl[3 * v][j], Yl[3 * v + 1][j], Yl[3 * v + 2][j]};
    double w[3];
    matvec3(&Rm[j][0], yv, w);
    const int off = B.body_off[p];
    double* dst = v < nb ? z + 3LL * (off + v) : z + Mx3 + 6LL * p + 3 * (v - nb);
    dst[0] = w[0];
    dst[1] = w[1];
    dst[2] = w[2];
    if (zs && v < nb) {
      double* d2 = zs + 3LL * spos[off + v];
      d2[0] = w[0];
      d2[1] = w[1];
      d2[2] = w[2];
      if (mirror) {   // the image's force R w
        double* d3 = zs + 3LL * spos[mirror + off + v];
        d3[0] = w[0];
        d3[1] = -w[1];
        d3[2] = w[2];
      }
    }
  }
  if (!yV) return;
  const double* bb = B.shape_b + 3LL * off_s;
  for (int t = tid; t < 16 * 6; t += 256) {
    const int j = t / 6, c = t % 6;
    if (pb[j] < 0) continue;
    double acc = 0.0;
    for (int i = 0; i < nb; ++i) {
      if (c < 3) {
        acc += Yl[3 * i + c][j];
      } else {
        const int cc = c - 3, c1 = (cc + 1) % 3, c2 = (cc + 2) % 3;
        acc += bb[3 * i + c1] * Yl[3 * i + c2][j] - bb[3 * i + c2] * Yl[3 * i + c1][j];
      }
    }
    const double* Pi = B.shape_null + 36LL * s + 6 * c;
    double pz = 0.0;
    for (int m = 0; m < 6; ++m) pz += Pi[m] * Yl[3 * nb + m][j];
    Tb[j][c] = -acc - pz;
  }
  __syncthreads();
  if (tid < 32) {
    const int j = tid >> 1, half = tid & 1;
    const int p = pb[j];
    if (p >= 0) {
      double w[3];
      matvec3(&Rm[j][0], &Tb[j][3 * half], w);
      double* dst = yV + 6LL * p + 3 * half;
      dst[0] = w[0];
      dst[1] = w[1];
      dst[2] = w[2];
    }
  }
}

__global__ __launch_bounds__(256) void k_precond_mfma(BodyTables B, const double* __restrict__ q,
                                                     const double* __restrict__ x, double* __restrict__ z,
                                                     double* __restrict__ yV, const int* __restrict__ spos,
                                                     double* __restrict__ zs, const int* __restrict__ skip,
                                                     int mirror) {
  precond_mfma_body(B, q, x, z, yV, spos, zs, skip, mirror, hw_block());
}

// The same, fused over several suspensions (one PrecondArgs each).
__global__ __launch_bounds__(256) void k_precond_mfma_fused(const PrecondArgs* __restrict__ a,
                                                           const int* __restrict__ first, int ns) {
  const int sidx = fused_suspension(first, ns, blockIdx.x);
  const PrecondArgs& A = a[sidx];
  precond_mfma_body(A.B, A.q, A.x, A.z, A.yV, A.spos, A.zs, A.skip, A.mirror,
                    fused_block(A.grid, (int)blockIdx.x - first[sidx]));
}

__global__ __launch_bounds__(64) void k_precond(BodyTables B, const double* __restrict__ q,
                                                const double* __restrict__ x, double* __restrict__ z,
                                                double* __restrict__ yV, const int* __restrict__ spos,
                                                double* __restrict__ zs, const int* __restrict__ skip,
                                                int mirror) {
  if (skip && *skip) return;
  extern __shared__ double sh[];
  const int p = blockIdx.x;
  const int lane = threadIdx.x;
  const int s = B.body_shape[p];
  const int off = B.body_off[p], nb = B.body_off[p + 1] - off;
  const int D = 3 * nb + 6;
  double* xb = sh;
  double* yb = sh + D;
  double* tb = sh + 2 * D;
  double R[9];
  rotmat(q + 4LL * p, R);
  const long long Mx3 = 3LL * B.M;
  for (int k = lane; k < nb + 2; k += 64) {
    const double* src = k < nb ? x + 3LL * (off + k) : x + Mx3 + 6LL * p + 3 * (k - nb);
    double v[3], w[3];
    load3(src, v);
    matTvec3(R, v, w);
    xb[3 * k] = w[0];
    xb[3 * k + 1] = w[1];
    xb[3 * k + 2] = w[2];
  }
  __syncthreads();
  const double* AT = B.shape_precT + B.shape_prec_off[s];
  for (int i = lane; i < D; i += 64) {
    double acc = 0.0;
    for (int j = 0; j < D; ++j) acc += AT[(long long)j * D + i] * xb[j];
    yb[i] = acc;
  }
  __syncthreads();
  for (int k = lane; k < nb + 2; k += 64) {
    double* dst = k < nb ? z + 3LL * (off + k) : z + Mx3 + 6LL * p + 3 * (k - nb);
    double v[3] = {yb[3 * k], yb[3 * k + 1], yb[3 * k + 2]}, w[3];
    matvec3(R, v, w);
    dst[0] = w[0];
    dst[1] = w[1];
    dst[2] = w[2];
    if (zs && k < nb) {
      double* d2 = zs + 3LL * spos[off + k];
      d2[0] = w[0];
      d2[1] = w[1];
      d2[2] = w[2];
      if (mirror) {   // the image's force R w
        double* d3 = zs + 3LL * spos[mirror + off + k];
        d3[0] = w[0];
        d3[1] = -w[1];
        d3[2] = w[2];
      }
    }
  }
  if (!yV) return;
  if (lane < 6) {
    double t = 0.0;
    const double* bb = B.shape_b + 3LL * B.shape_boff[s];
    for (int i = 0; i < nb; ++i) {
      const double* zi = yb + 3 * i;
      if (lane < 3) {
        t += zi[lane];
      } else {
        const double* bi = bb + 3 * i;
        const int c = lane - 3, c1 = (c + 1) % 3, c2 = (c + 2) % 3;
        t += bi[c1] * zi[c2] - bi[c2] * zi[c1];
      }
    }
    const double* Pi = B.shape_null + 36LL * s + 6 * lane;
    double pz = 0.0;
    for (int j = 0; j < 6; ++j) pz += Pi[j] * yb[3 * nb + j];
    tb[lane] = -t - pz;
  }
  __syncthreads();
  if (lane < 2) {
    double w[3];
    matvec3(R, tb + 3 * lane, w);
    double* dst = yV + 6LL * p + 3 * lane;
    dst[0] = w[0];
    dst[1] = w[1];
    dst[2] = w[2];
  }
}

// ------------------------------------------------------------ step 3 perturbations
// mode 0 (finite differences, eq. FD): six displacements per blob,
//   k = 0..2: delta L_p e_k (translation), k = 3..5: (R(exp(delta e_{k-3}) . q) - R(q)) b_i.
// mode 1 (random finite differences, eq. rfd_div): one displacement
//   delta L_p W_U + (R(exp(delta W_Omega) . q) - R(q)) b_i with W ~ N(0,1)^6 from
//   Philox (stage 1, c0 = body, calls 0 and 1, first six normals).
// With Y given, the blob positions r_i = Y_p + R(q_p) b_i are written too
// (the rotation is at hand).
__global__ void k_fd_displacements(BodyTables B, const double* __restrict__ q, double delta, int mode,
                                   uint64_t seed, uint64_t step, double* __restrict__ dr,
                                   double* __restrict__ wrfd, const double* __restrict__ Y,
                                   double* __restrict__ r, const uint64_t* __restrict__ step_ptr) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= B.M) return;
  if (step_ptr) step = *step_ptr;
  const int p = B.blob_body[i], s = B.body_shape[p];
  const double Lp = B.shape_Lp[s];
  double b[3], R[9];
  load3(B.shape_b + 3LL * (B.shape_boff[s] + B.blob_local[i]), b);
  const double* qp = q + 4LL * p;
  rotmat(qp, R);
  if (Y) {
    double x[3];
    matvec3(R, b, x);
    r[3LL * i] = Y[3LL * p] + x[0];
    r[3LL * i + 1] = Y[3LL * p + 1] + x[1];
    r[3LL * i + 2] = Y[3LL * p + 2] + x[2];
  }
  if (mode == 0) {
    double* o = dr + 18LL * i;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      o[3 * k] = k == 0 ? delta * Lp : 0.0;
      o[3 * k + 1] = k == 1 ? delta * Lp : 0.0;
      o[3 * k + 2] = k == 2 ? delta * Lp : 0.0;
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      double u[3] = {0, 0, 0}, e[4], q2[4], R2[9], D[9];
      u[a] = delta;
      qexp(u, e);
      qmul(e, qp, q2);
      rotmat(q2, R2);
#pragma unroll
      for (int k = 0; k < 9; ++k) D[k] = R2[k] - R[k];
      double x[3];
      matvec3(D, b, x);
      o[9 + 3 * a] = x[0];
      o[9 + 3 * a + 1] = x[1];
      o[9 + 3 * a + 2] = x[2];
    }
  } else {
    double z[8];
    four_normals(seed, (uint32_t)p, 16u, step, z);
    four_normals(seed, (uint32_t)p, 17u, step, z + 4);
    double u[3] = {delta * z[3], delta * z[4], delta * z[5]}, e[4], q2[4], R2[9], D[9], x[3];
    qexp(u, e);
    qmul(e, qp, q2);
    rotmat(q2, R2);
#pragma unroll
    for (int k = 0; k < 9; ++k) D[k] = R2[k] - R[k];
    matvec3(D, b, x);
    dr[3LL * i] = delta * Lp * z[0] + x[0];
    dr[3LL * i + 1] = delta * Lp * z[1] + x[1];
    dr[3LL * i + 2] = delta * Lp * z[2] + x[2];
    if (B.blob_local[i] == 0) {
#pragma unroll
      for (int k = 0; k < 6; ++k) wrfd[6LL * p + k] = z[k];
    }
  }
}

// calV = Q^T (K^T K)^+_body Q K^T v with lab-frame offsets R b_i (eq. sol_unconst).
__device__ void lsq_body(const BodyTables& B, int p, int s, const double* R, const double* v,
                         long long vstride, const double* vadd, long long astride, double* out) {
  double F[6] = {0, 0, 0, 0, 0, 0};
  const int off = B.body_off[p], nb = B.body_off[p + 1] - off;
  for (int k = 0; k < nb; ++k) {
    double b[3], rel[3], w[3], t[3];
    load3(B.shape_b + 3LL * (B.shape_boff[s] + k), b);
    matvec3(R, b, rel);
    const double* vi = v + vstride * (off + k);
    w[0] = vi[0];
    w[1] = vi[1];
    w[2] = vi[2];
    if (vadd) {
      const double* ai = vadd + astride * (off + k);
      w[0] += ai[0];
      w[1] += ai[1];
      w[2] += ai[2];
    }
    cross3(rel, w, t);
    F[0] += w[0]; F[1] += w[1]; F[2] += w[2];
    F[3] += t[0]; F[4] += t[1]; F[5] += t[2];
  }
  rotate_6x6(B.shape_pinv + 36LL * s, R, F, out);
}

// Per body: calV_p and d_p (eq. FD or the term inside the expectation of
// eq. rfd_div), so that nu = 1 + dt/2 sum_p d_p.  A body takes 8 lanes: lane
// 0 solves at the unperturbed state; with forward differences lanes 1-3
// solve with the translated velocities and lanes 4-6 at the rotated
// orientations, with RFD lane 1 at the random displacement.  Lane 0 adds the
// quotients in the order translations, then rotations.
constexpr int LSQ_LANES = 8;

__device__ void lsq_div_body(const BodyTables& B, int p, int j, const double* __restrict__ q,
                             const double* __restrict__ v, const double* __restrict__ vd,
                             const double* __restrict__ wrfd, double delta, int mode, double* __restrict__ calV,
                             double* __restrict__ d) {
  const int s = B.body_shape[p];
  const double Lp = B.shape_Lp[s];
  const double* qp = q + 4LL * p;
  double R[9], V[6] = {0, 0, 0, 0, 0, 0};
  rotmat(qp, R);
  if (j == 0) {
    lsq_body(B, p, s, R, v, 3, nullptr, 0, V);
  } else if (mode == 0 && j <= 3) {   // translation: K unchanged, difference of v only
    lsq_body(B, p, s, R, vd + 3 * (j - 1), 18, nullptr, 0, V);
  } else if ((mode == 0 && j <= 6) || (mode != 0 && j == 1)) {   // rotation: K and v both change
    double u[3] = {0, 0, 0}, e[4], q2[4], R2[9];
    if (mode == 0) {
      u[j - 4] = delta;
    } else {
      const double* z = wrfd + 6LL * p;
      u[0] = delta * z[3];
      u[1] = delta * z[4];
      u[2] = delta * z[5];
    }
    qexp(u, e);
    qmul(e, qp, q2);
    rotmat(q2, R2);
    lsq_body(B, p, s, R2, v, 3, mode == 0 ? vd + 9 + 3 * (j - 4) : vd, mode == 0 ? 18 : 3, V);
  }
  double V0[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) V0[k] = __shfl(V[k], 0, LSQ_LANES);
  if (j == 0) {
#pragma unroll
    for (int k = 0; k < 6; ++k) calV[6LL * p + k] = V0[k];
  }
  if (mode == 0) {
    double c = 0.0;
    if (j >= 1 && j <= 3) {
      const double dv = j == 1 ? V[0] : j == 2 ? V[1] : V[2];
      c = dv / (delta * Lp);
    } else if (j >= 4 && j <= 6) {
      const double v1 = j == 4 ? V[3] : j == 5 ? V[4] : V[5];
      const double v0 = j == 4 ? V0[3] : j == 5 ? V0[4] : V0[5];
      c = (v1 - v0) / delta;
    }
    double acc = 0.0;
#pragma unroll
    for (int t = 1; t <= 6; ++t) acc += __shfl(c, t, LSQ_LANES);
    if (j == 0) d[p] = acc;
  } else if (j == 1) {
    const double* z = wrfd + 6LL * p;
    d[p] = (z[0] * (V[0] - V0[0]) + z[1] * (V[1] - V0[1]) + z[2] * (V[2] - V0[2])) / (delta * Lp) +
           (z[3] * (V[3] - V0[3]) + z[4] * (V[4] - V0[4]) + z[5] * (V[5] - V0[5])) / delta;
  }
}

// The per-body work above, then nu = 1 + half_dt sum_p d_p by the last block
// to finish (counter zero on entry and left at zero): thread t adds d_t,
// d_{t+64}, ... in order, then the wave adds across lanes.  Fixed order, no
// atomics on the data.
__global__ __launch_bounds__(64) void k_body_lsq_div(BodyTables B, const double* __restrict__ q,
                                                     const double* __restrict__ v, const double* __restrict__ vd,
                                                     const double* __restrict__ wrfd, double delta, int mode,
                                                     double* __restrict__ calV, double* __restrict__ d,
                                                     unsigned int* __restrict__ counter, double half_dt,
                                                     double* __restrict__ nu) {
  __shared__ bool last;
  const int p = (blockIdx.x * blockDim.x + threadIdx.x) / LSQ_LANES;
  const int j = threadIdx.x % LSQ_LANES;
  if (p < B.N) lsq_div_body(B, p, j, q, v, vd, wrfd, delta, mode, calV, d);   // a body's 8 lanes together
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) last = atomicAdd(counter, 1u) == gridDim.x - 1;
  __syncthreads();
  if (!last) return;
  __threadfence();
  const volatile double* dv = d;
  double sum = 0.0;
  for (int i = threadIdx.x; i < B.N; i += 64) sum += dv[i];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) sum += __shfl_xor(sum, o, 64);
  if (threadIdx.x == 0) {
    nu[0] = 1.0 + half_dt * sum;
    *counter = 0u;
  }
}


// Step 4 and the midpoint blob positions in one pass, one thread per blob:
// each blob forms its body's Y^m, q^m (the body's first blob stores them)
// and r^m_i = Y^m + R(q^m) b_i.
__global__ void k_midpoint_blobs(BodyTables B, const double* __restrict__ Y, const double* __restrict__ q,
                                 const double* __restrict__ calV, double h, double* __restrict__ Ym,
                                 double* __restrict__ qm, double* __restrict__ rm) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= B.M) return;
  const int p = B.blob_body[i], s = B.body_shape[p];
  const double* V = calV + 6LL * p;
  const double y[3] = {Y[3LL * p] + h * V[0], Y[3LL * p + 1] + h * V[1], Y[3LL * p + 2] + h * V[2]};
  double u[3] = {h * V[3], h * V[4], h * V[5]}, e[4], qq[4];
  qexp(u, e);
  qmul(e, q + 4LL * p, qq);
  if (B.blob_local[i] == 0) {
    Ym[3LL * p] = y[0];
    Ym[3LL * p + 1] = y[1];
    Ym[3LL * p + 2] = y[2];
#pragma unroll
    for (int k = 0; k < 4; ++k) qm[4LL * p + k] = qq[k];
  }
  double R[9], b[3], x[3];
  rotmat(qq, R);
  load3(B.shape_b + 3LL * (B.shape_boff[s] + B.blob_local[i]), b);
  matvec3(R, b, x);
  rm[3LL * i] = y[0] + x[0];
  rm[3LL * i + 1] = y[1] + x[1];
  rm[3LL * i + 2] = y[2] + x[2];
}

// Step 6: Y += nu dt V_U, q = exp(nu dt V_Omega) . q (nu on the device).
__global__ void k_update(int N, double* __restrict__ Y, double* __restrict__ q, const double* __restrict__ V,
                         const double* __restrict__ nu, double dt, int* __restrict__ nonfinite) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= N) return;
  const double h = (nu ? nu[0] : 1.0) * dt;
  const double* Vp = V + 6LL * p;
  Y[3LL * p] += h * Vp[0];
  Y[3LL * p + 1] += h * Vp[1];
  Y[3LL * p + 2] += h * Vp[2];
  double u[3] = {h * Vp[3], h * Vp[4], h * Vp[5]}, e[4], qn[4];
  qexp(u, e);
  qmul(e, q + 4LL * p, qn);
  q[4LL * p] = qn[0];
  q[4LL * p + 1] = qn[1];
  q[4LL * p + 2] = qn[2];
  q[4LL * p + 3] = qn[3];
  if (nonfinite) {
    bool ok = isfinite(qn[0]) && isfinite(qn[1]) && isfinite(qn[2]) && isfinite(qn[3]);
    for (int c = 0; c < 3; ++c) ok = ok && isfinite(Y[3LL * p + c]);
    if (!ok) atomicMax(nonfinite, 1);
  }
}

// Right-hand side [-(v_slip + u_inf); -(I - Pi) F] of the saddle problem.
__device__ __forceinline__ void rhs_blob(const BodyTables& B, int i, const double* __restrict__ Y,
                                         const double* __restrict__ r, const double* __restrict__ vslip,
                                         const double* __restrict__ vbg, double cbg, double shear, double Ly,
                                         double* __restrict__ rhs) {
  double ux = vbg ? cbg * vbg[3LL * i] : 0.0;
  if (shear != 0.0) {
    const int p = B.blob_body[i];
    const double yc = Y[3LL * p + 1];
    const double yw = yc - Ly * floor(yc / Ly);
    ux += shear * (yw + (r[3LL * i + 1] - yc) - 0.5 * Ly);
  }
  rhs[3LL * i] = -((vslip ? vslip[3LL * i] : 0.0) + ux);
  rhs[3LL * i + 1] = -(vslip ? vslip[3LL * i + 1] : 0.0);
  rhs[3LL * i + 2] = -(vslip ? vslip[3LL * i + 2] : 0.0);
}

__device__ __forceinline__ void rhs_body(const BodyTables& B, int p, const double* __restrict__ q,
                                         const double* __restrict__ F, double* __restrict__ rhsV) {
  double R[9], f[6], pf[6];
  rotmat(q + 4LL * p, R);
#pragma unroll
  for (int k = 0; k < 6; ++k) f[k] = F ? F[6LL * p + k] : 0.0;
  rotate_6x6(B.shape_null + 36LL * B.body_shape[p], R, f, pf);
#pragma unroll
  for (int k = 0; k < 6; ++k) rhsV[6LL * p + k] = -(f[k] - pf[k]);
}

// Both parts of the right-hand side in one launch: threads [0, M) the blob
// rows, threads [M, M + N) the body rows.
__global__ void k_rhs(BodyTables B, const double* __restrict__ Y, const double* __restrict__ r,
                      const double* __restrict__ vslip, const double* __restrict__ vbg, double cbg, double shear,
                      double Ly, const double* __restrict__ q, const double* __restrict__ F,
                      double* __restrict__ rhs) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < B.M)
    rhs_blob(B, i, Y, r, vslip, vbg, cbg, shear, Ly, rhs);
  else if (i < B.M + B.N)
    rhs_body(B, i - B.M, q, F, rhs + 3LL * B.M);
}

// ------------------------------------------------------------ pair forces
struct CellGrid {
  int nc[3];
  double csz[3];
  double L[3];
};

__device__ __forceinline__ int cell_of(const CellGrid& C, const double* x, double* xw) {
  int c[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    xw[d] = x[d] - C.L[d] * floor(x[d] / C.L[d]);
    const double kf = xw[d] / C.csz[d];
    int k = (kf >= 0.0 && kf < 1e9) ? (int)kf : 0;
    c[d] = k < 0 ? 0 : (k >= C.nc[d] ? C.nc[d] - 1 : k);
  }
  return (c[0] * C.nc[1] + c[1]) * C.nc[2] + c[2];
}

__global__ void k_bin_blobs(CellGrid C, int M, const double* __restrict__ r, int* __restrict__ count,
                            int* __restrict__ list, int cap, int* __restrict__ overflow) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= M) return;
  double xw[3];
  const int c = cell_of(C, r + 3LL * i, xw);
  const int slot = atomicAdd(count + c, 1);
  if (slot < cap)
    list[(long long)c * cap + slot] = i;
  else
    atomicMax(overflow, 1);
}

// Harmonic repulsion V = k/2 (r - b)^2 for r < b between blobs of different
// bodies; each blob sums its own force (no atomics).  A blob takes 32 lanes,
// lane c < 27 scanning neighbour cell c of its 3 x 3 x 3 block, and the
// lanes' partial forces are added across the half wave.
constexpr int STERIC_LANES = 32;

__global__ __launch_bounds__(NT) void k_steric(CellGrid C, BodyTables B, const double* __restrict__ r,
                                               const int* __restrict__ count, const int* __restrict__ list, int cap,
                                               double kk, double b, double* __restrict__ f) {
  const int i = (blockIdx.x * blockDim.x + threadIdx.x) / STERIC_LANES;
  const int lane = threadIdx.x % STERIC_LANES;
  if (i >= B.M) return;   // whole half waves leave together
  double xi[3];
  const int ci = cell_of(C, r + 3LL * i, xi);
  double fx = 0, fy = 0, fz = 0;
  if (lane < 27) {
    const int c3[3] = {ci / (C.nc[1] * C.nc[2]), (ci / C.nc[2]) % C.nc[1], ci % C.nc[2]};
    const int a0 = (c3[0] + lane / 9 - 1 + C.nc[0]) % C.nc[0];
    const int a1 = (c3[1] + (lane / 3) % 3 - 1 + C.nc[1]) % C.nc[1];
    const int a2 = (c3[2] + lane % 3 - 1 + C.nc[2]) % C.nc[2];
    const int cc = (a0 * C.nc[1] + a1) * C.nc[2] + a2;
    const int n = min(count[cc], cap);
    const int bi = B.blob_body[i];
    for (int s = 0; s < n; ++s) {
      const int j = list[(long long)cc * cap + s];
      if (j == i || B.blob_body[j] == bi) continue;
      double d[3];
#pragma unroll
      for (int e = 0; e < 3; ++e) {
        const double xj = r[3LL * j + e] - C.L[e] * floor(r[3LL * j + e] / C.L[e]);
        double t = xi[e] - xj;
        t -= C.L[e] * rint(t / C.L[e]);
        d[e] = t;
      }
      const double dist2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
      if (dist2 < b * b && dist2 > 0.0) {
        const double dist = sqrt(dist2);
        const double m = kk * (b - dist) / dist;
        fx += m * d[0];
        fy += m * d[1];
        fz += m * d[2];
      }
    }
  }
#pragma unroll
  for (int o = STERIC_LANES / 2; o > 0; o >>= 1) {
    fx += __shfl_xor(fx, o, STERIC_LANES);
    fy += __shfl_xor(fy, o, STERIC_LANES);
    fz += __shfl_xor(fz, o, STERIC_LANES);
  }
  if (lane == 0) {
    f[3LL * i] = fx;
    f[3LL * i + 1] = fy;
    f[3LL * i + 2] = fz;
  }
}

__global__ void k_body_forces(BodyTables B, const double* __restrict__ Y, const double* __restrict__ r,
                              const double* __restrict__ fblob, const double* __restrict__ cf,
                              double* __restrict__ F) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= B.N) return;
  double acc[6] = {cf[0], cf[1], cf[2], cf[3], cf[4], cf[5]};
  if (fblob) {
    for (int i = B.body_off[p]; i < B.body_off[p + 1]; ++i) {
      double rel[3] = {r[3LL * i] - Y[3LL * p], r[3LL * i + 1] - Y[3LL * p + 1], r[3LL * i + 2] - Y[3LL * p + 2]};
      double fi[3], t[3];
      load3(fblob + 3LL * i, fi);
      cross3(rel, fi, t);
      acc[0] += fi[0]; acc[1] += fi[1]; acc[2] += fi[2];
      acc[3] += t[0]; acc[4] += t[1]; acc[5] += t[2];
    }
  }
#pragma unroll
  for (int k = 0; k < 6; ++k) F[6LL * p + k] = acc[k];
}

__global__ void k_check_finite(const double* __restrict__ x, long long n, int* __restrict__ flag) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long stride = (long long)gridDim.x * blockDim.x;
  bool bad = false;
  for (long long k = i; k < n; k += stride) bad |= !isfinite(x[k]);
  if (bad) atomicMax(flag, 1);
}

// A caller's state on the device: flag[0] = 1 if some Y is not finite,
// flag[1] = 1 if some |q| differs from 1 by more than qtol (or is not finite).
__global__ void k_check_state(const double* __restrict__ Y, const double* __restrict__ q, int N, double qtol,
                              int* __restrict__ flag) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= N) return;
  const double* y = Y + 3LL * p;
  if (!(isfinite(y[0]) && isfinite(y[1]) && isfinite(y[2]))) atomicMax(flag, 1);
  const double* qp = q + 4LL * p;
  const double nrm = sqrt(qp[0] * qp[0] + qp[1] * qp[1] + qp[2] * qp[2] + qp[3] * qp[3]);
  if (!(fabs(nrm - 1.0) <= qtol)) atomicMax(flag + 1, 1);
}

// Slip channel: rs = [r; sigma(r)], the image of blob i at (x, L1 - y, z).
__global__ void k_mirror_positions(const double* __restrict__ r, int M, double L1, double* __restrict__ rs) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= M) return;
  const double x = r[3LL * i], y = r[3LL * i + 1], z = r[3LL * i + 2];
  rs[3LL * i] = x;
  rs[3LL * i + 1] = y;
  rs[3LL * i + 2] = z;
  rs[3LL * (M + i)] = x;
  rs[3LL * (M + i) + 1] = L1 - y;
  rs[3LL * (M + i) + 2] = z;
}

__global__ void k_sort_forces(const double* __restrict__ lam, const int* __restrict__ spos, int M, int mirror,
                              double* __restrict__ zs) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= M) return;
  const double l0 = lam[3LL * i], l1 = lam[3LL * i + 1], l2 = lam[3LL * i + 2];
  double* d = zs + 3LL * spos[i];
  d[0] = l0;
  d[1] = l1;
  d[2] = l2;
  if (mirror) {
    double* e = zs + 3LL * spos[mirror + i];
    e[0] = l0;
    e[1] = -l1;
    e[2] = l2;
  }
}

// Harmonic blob-wall repulsion (Sec. 6.3), y component of each blob force.
__global__ void k_wall_forces(const double* __restrict__ r, int M, double H, double k, double b,
                              double* __restrict__ f, int add) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= M) return;
  const double y = r[3LL * i + 1];
  double fy = 0.0;
  if (y < b) fy += k * (b - y);
  if (H - y < b) fy -= k * (b - (H - y));
  if (add) {
    f[3LL * i + 1] += fy;
  } else {
    f[3LL * i] = 0.0;
    f[3LL * i + 1] = fy;
    f[3LL * i + 2] = 0.0;
  }
}

}  // namespace

int check_state(const double* Y, const double* q, int N, double qtol, int* flag, hipStream_t s) {
  if (N <= 0) return GDC_OK;
  hipLaunchKernelGGL(k_check_state, dim3((N + 255) / 256), dim3(256), 0, s, Y, q, N, qtol, flag);
  return check_launch("k_check_state");
}

int blob_positions(const BodyTables& b, const double* Y, const double* q, double* r, hipStream_t s) {
  if (b.M == 0) return GDC_OK;
  hipLaunchKernelGGL(k_blob_positions, dim3(nblk(b.M)), dim3(NT), 0, s, b, Y, q, r);
  return check_launch("k_blob_positions");
}

bool precond_fusable(const BodyTables& b, int maxdim) { return b.mfma && maxdim <= PREC_MFMA_MAXDIM; }

void precond_describe(PrecondArgs& a, const BodyTables& b, const double* q, const double* x, double* z, double* yV,
                      const int* spos, double* zs, const int* skip, int mirror) {
  a.B = b;
  a.q = q;
  a.x = x;
  a.z = z;
  a.yV = yV;
  a.spos = spos;
  a.zs = zs;
  a.skip = skip;
  a.mirror = mirror;
  a.grid = LocalGrid{b.n_groups, 1, 1};
}

int precond_fused(const PrecondArgs* dev_args, int ns, const int* first, int total, hipStream_t s) {
  if (ns <= 0) return GDC_OK;
  hipLaunchKernelGGL(k_precond_mfma_fused, dim3(total), dim3(256), 0, s, dev_args, first, ns);
  return check_launch("k_precond_mfma_fused");
}

int precond_apply(const BodyTables& b, const double* q, const double* x, double* z, double* yV, const int* spos,
                  double* zs, int maxdim, hipStream_t s, const int* skip, int mirror) {
  if (precond_fusable(b, maxdim)) {
    hipLaunchKernelGGL(k_precond_mfma, dim3(b.n_groups), dim3(256), 0, s, b, q, x, z, yV, spos, zs, skip, mirror);
    return check_launch("k_precond_mfma");
  }
  const size_t shm = (2 * (size_t)maxdim + 8) * sizeof(double);
  hipLaunchKernelGGL(k_precond, dim3(b.N), dim3(64), shm, s, b, q, x, z, yV, spos, zs, skip, mirror);
  return check_launch("k_precond");
}

int mirror_positions(const double* r, int M, double L1, double* rs, hipStream_t s) {
  if (M <= 0) return GDC_OK;
  hipLaunchKernelGGL(k_mirror_positions, dim3(nblk(M)), dim3(NT), 0, s, r, M, L1, rs);
  return check_launch("k_mirror_positions");
}

int sort_forces(const double* lam, const int* spos, int M, int mirror, double* zs, hipStream_t s) {
  if (M <= 0) return GDC_OK;
  hipLaunchKernelGGL(k_sort_forces, dim3(nblk(M)), dim3(NT), 0, s, lam, spos, M, mirror, zs);
  return check_launch("k_sort_forces");
}

int wall_forces(const double* r, int M, double H, double k, double b, double* fblob, bool add, hipStream_t s) {
  if (M <= 0) return GDC_OK;
  hipLaunchKernelGGL(k_wall_forces, dim3(nblk(M)), dim3(NT), 0, s, r, M, H, k, b, fblob, add ? 1 : 0);
  return check_launch("k_wall_forces");
}

int fd_displacements(const BodyTables& b, const double* q, double delta, int mode, uint64_t seed,
                     uint64_t step, double* dr, double* wrfd, hipStream_t s, const double* Y, double* r,
                     const uint64_t* step_ptr) {
  hipLaunchKernelGGL(k_fd_displacements, dim3(nblk(b.M)), dim3(NT), 0, s, b, q, delta, mode, seed, step, dr, wrfd,
                     Y, r, step_ptr);
  return check_launch("k_fd_displacements");
}

__global__ void k_step_counter(uint64_t* __restrict__ c, uint64_t v, int bump) {
  if (threadIdx.x == 0) *c = bump ? *c + 1 : v;
}

int step_counter_set(uint64_t* c, uint64_t v, hipStream_t s) {
  hipLaunchKernelGGL(k_step_counter, dim3(1), dim3(64), 0, s, c, v, 0);
  return check_launch("k_step_counter");
}

int step_counter_bump(uint64_t* c, hipStream_t s) {
  hipLaunchKernelGGL(k_step_counter, dim3(1), dim3(64), 0, s, c, (uint64_t)0, 1);
  return check_launch("k_step_counter");
}

int body_lsq_div(const BodyTables& b, const double* q, const double* v, const double* vd, const double* wrfd,
                 double delta, int mode, double* calV, double* d, unsigned int* counter, double half_dt, double* nu,
                 hipStream_t s) {
  hipLaunchKernelGGL(k_body_lsq_div, dim3(nblk((long long)b.N * LSQ_LANES, 64)), dim3(64), 0, s, b, q, v, vd, wrfd,
                     delta, mode, calV, d, counter, half_dt, nu);
  return check_launch("k_body_lsq_div");
}


int midpoint_positions(const BodyTables& b, const double* Y, const double* q, const double* calV, double h,
                       double* Ym, double* qm, double* rm, hipStream_t s) {
  hipLaunchKernelGGL(k_midpoint_blobs, dim3(nblk(b.M)), dim3(NT), 0, s, b, Y, q, calV, h, Ym, qm, rm);
  return check_launch("k_midpoint_blobs");
}

int update(const BodyTables& b, double* Y, double* q, const double* V, const double* nu, double dt, int* nonfinite,
           hipStream_t s) {
  hipLaunchKernelGGL(k_update, dim3(nblk(b.N)), dim3(NT), 0, s, b.N, Y, q, V, nu, dt, nonfinite);
  return check_launch("k_update");
}

int rhs_build(const BodyTables& b, const double* q, const double* Y, const double* r, const double* vslip,
              const double* vbg, double cbg, const double* F, double shear, double Ly, double* rhs,
              hipStream_t s) {
  hipLaunchKernelGGL(k_rhs, dim3(nblk((long long)b.M + b.N)), dim3(NT), 0, s, b, Y, r, vslip, vbg, cbg, shear, Ly, q,
                     F, rhs);
  return check_launch("k_rhs");
}

int steric_forces(const BodyTables& b, const GridGeom& g, const double* r, double k, double cutoff,
                  int* cell_count, int* cell_list, int cap, const int nc[3], int* overflow, double* fblob,
                  hipStream_t s, bool zeroed) {
  CellGrid C;
  for (int d = 0; d < 3; ++d) {
    C.nc[d] = nc[d];
    C.L[d] = g.L[d];
    C.csz[d] = g.L[d] / nc[d];
  }
  if (!zeroed) GDC_TRY(fill_zero(cell_count, cell_count_bytes(nc), s));
  hipLaunchKernelGGL(k_bin_blobs, dim3(nblk(b.M)), dim3(NT), 0, s, C, b.M, r, cell_count, cell_list, cap, overflow);
  GDC_TRY(check_launch("k_bin_blobs"));
  hipLaunchKernelGGL(k_steric, dim3(nblk((long long)b.M * STERIC_LANES)), dim3(NT), 0, s, C, b, r, cell_count,
                     cell_list, cap, k, cutoff, fblob);
  return check_launch("k_steric");
}

int body_forces(const BodyTables& b, const double* Y, const double* r, const double* fblob, const double* cforce,
                double* F, hipStream_t s) {
  hipLaunchKernelGGL(k_body_forces, dim3(nblk(b.N)), dim3(NT), 0, s, b, Y, r, fblob, cforce, F);
  return check_launch("k_body_forces");
}

int check_finite(const double* x, long long n, int* flag, hipStream_t s) {
  const long long want = (n + 255) / 256;
  hipLaunchKernelGGL(k_check_finite, dim3((unsigned)(want < 4096 ? (want > 0 ? want : 1) : 4096)), dim3(256), 0, s,
                     x, n, flag);
  return check_launch("k_check_finite");
}

}  // namespace gdc
