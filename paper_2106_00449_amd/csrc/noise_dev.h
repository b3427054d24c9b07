// Device side of the noise contract, shared by the kernels that draw random
// numbers (stress spectrum, random finite differences).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace gdc {

// ------------------------------------------------------------ noise contract
// Philox4x32-10 (Salmon et al., SC'11) and Box-Muller with series log, sin and
// cos evaluated without contraction in a fixed order, so that every normal is
// reproducible bit for bit by an independent implementation of the same
// definition.

__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint32_t lo0 = 0xD2511F53u * c[0], hi0 = __umulhi(0xD2511F53u, c[0]);
    const uint32_t lo1 = 0xCD9E8D57u * c[2], hi1 = __umulhi(0xCD9E8D57u, c[2]);
    const uint32_t n0 = hi1 ^ c[1] ^ k0;
    const uint32_t n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
  }
}

__device__ __forceinline__ double uniform_open(uint32_t x) {
  return ((double)x + 0.5) * (1.0 / 4294967296.0);
}

// ln u: u = m 2^e with m in [sqrt(1/2), sqrt(2)); ln m = 2 atanh(s),
// s = (m-1)/(m+1), series in s^2 to the 1/25 term.
__device__ inline double series_log(double u) {
#pragma clang fp contract(off)
  int e;
  double m = frexp(u, &e);
  if (m < 0.7071067811865475244) {
    m = m * 2.0;
    e -= 1;
  }
  const double s = (m - 1.0) / (m + 1.0);
  const double z = s * s;
  double p = 1.0 / 25.0;
  p = p * z + 1.0 / 23.0;
  p = p * z + 1.0 / 21.0;
  p = p * z + 1.0 / 19.0;
  p = p * z + 1.0 / 17.0;
  p = p * z + 1.0 / 15.0;
  p = p * z + 1.0 / 13.0;
  p = p * z + 1.0 / 11.0;
  p = p * z + 1.0 / 9.0;
  p = p * z + 1.0 / 7.0;
  p = p * z + 1.0 / 5.0;
  p = p * z + 1.0 / 3.0;
  p = p * z + 1.0 / 1.0;
  const double t = s * p;
  return (t + t) + (double)e * 0.6931471805599453094;
}

// sin and cos of 2 pi u: 4u = j + f, theta = f pi/2 in [-pi/4, pi/4], Taylor
// series to theta^17 and theta^18, quarter-turn identities for j mod 4.
__device__ inline void series_sincos_2pi(double u, double* sn_out, double* cs_out) {
#pragma clang fp contract(off)
  const double t = 4.0 * u;
  const double j = floor(t + 0.5);
  const double f = t - j;
  const double th = f * 1.5707963267948966192;
  const double z = th * th;
  double ps = 1.0 / 355687428096000.0;
  ps = ps * z + -1.0 / 1307674368000.0;
  ps = ps * z + 1.0 / 6227020800.0;
  ps = ps * z + -1.0 / 39916800.0;
  ps = ps * z + 1.0 / 362880.0;
  ps = ps * z + -1.0 / 5040.0;
  ps = ps * z + 1.0 / 120.0;
  ps = ps * z + -1.0 / 6.0;
  ps = ps * z + 1.0;
  const double sn = th * ps;
  double pc = -1.0 / 6402373705728000.0;
  pc = pc * z + 1.0 / 20922789888000.0;
  pc = pc * z + -1.0 / 87178291200.0;
  pc = pc * z + 1.0 / 479001600.0;
  pc = pc * z + -1.0 / 3628800.0;
  pc = pc * z + 1.0 / 40320.0;
  pc = pc * z + -1.0 / 720.0;
  pc = pc * z + 1.0 / 24.0;
  pc = pc * z + -1.0 / 2.0;
  pc = pc * z + 1.0;
  const double cs = pc;
  switch (((int)j) & 3) {
    case 0: *sn_out = sn; *cs_out = cs; break;
    case 1: *sn_out = cs; *cs_out = -sn; break;
    case 2: *sn_out = -sn; *cs_out = -cs; break;
    default: *sn_out = -cs; *cs_out = sn; break;
  }
}

// Four normals from one counter (c0, c1, step lo, step hi), key = seed.
__device__ inline void four_normals(uint64_t seed, uint32_t c0, uint32_t c1, uint64_t step, double z[4]) {
#pragma clang fp contract(off)
  uint32_t c[4] = {c0, c1, (uint32_t)(step & 0xFFFFFFFFu), (uint32_t)(step >> 32)};
  philox4x32_10(c, (uint32_t)(seed & 0xFFFFFFFFu), (uint32_t)(seed >> 32));
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const double u1 = uniform_open(c[2 * h]);
    const double u2 = uniform_open(c[2 * h + 1]);
    const double r = sqrt(-2.0 * series_log(u1));
    double s, co;
    series_sincos_2pi(u2, &s, &co);
    z[2 * h] = r * co;
    z[2 * h + 1] = r * s;
  }
}

}  // namespace gdc
