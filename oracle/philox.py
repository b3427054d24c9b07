"""Counter-based noise: Philox4x32-10 and a Box-Muller normal transform.

Philox4x32-10 follows its published definition (Salmon, Moraes, Dror & Shaw,
"Parallel random numbers: as easy as 1, 2, 3", SC'11): ten rounds of two
32x32->64-bit multiplications with constants 0xD2511F53 and 0xCD9E8D57, a
word permutation, and a Weyl key schedule with increments 0x9E3779B9 and
0xBB67AE85.  Pinned by the paper's published known-answer vectors.

Normal transform (the project's noise contract, written once here in NumPy
and independently once in HIP): each 32-bit word x gives u = (x + 1/2) 2^-32
in (0, 1); a pair (u1, u2) gives r cos(2 pi u2), r sin(2 pi u2) with
r = sqrt(-2 ln u1) (Box & Muller 1958).  ln, sin and cos are evaluated by the
series below, using only IEEE +, -, *, / and sqrt in a fixed order, so that a
GPU build without floating-point contraction reproduces every bit.

Oracle code: test infrastructure only.
"""

import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = np.uint32(0x9E3779B9)
W1 = np.uint32(0xBB67AE85)
MASK32 = np.uint64(0xFFFFFFFF)


def philox4x32_10(ctr, key):
    """ctr: (..., 4) uint32, key: (..., 2) uint32 -> (..., 4) uint32."""
    c = [np.asarray(ctr[..., i], dtype=np.uint64) for i in range(4)]
    k0 = np.asarray(key[..., 0], dtype=np.uint32).copy()
    k1 = np.asarray(key[..., 1], dtype=np.uint32).copy()
    with np.errstate(over="ignore"):
        for rnd in range(10):
            if rnd > 0:
                k0 = (k0 + W0).astype(np.uint32)
                k1 = (k1 + W1).astype(np.uint32)
            p0 = M0 * c[0]
            p1 = M1 * c[2]
            hi0, lo0 = p0 >> np.uint64(32), p0 & MASK32
            hi1, lo1 = p1 >> np.uint64(32), p1 & MASK32
            c = [hi1 ^ c[1] ^ k0.astype(np.uint64), lo1,
                 hi0 ^ c[3] ^ k1.astype(np.uint64), lo0]
    return np.stack([x.astype(np.uint32) for x in c], axis=-1)


def uniform_open(x):
    """uint32 -> (x + 1/2) 2^-32, exact in FP64, strictly inside (0, 1)."""
    return (np.asarray(x, dtype=np.float64) + 0.5) * (1.0 / 4294967296.0)


LN2 = 0.6931471805599453094
SQRT_HALF = 0.7071067811865475244
HALF_PI = 1.5707963267948966192


def series_log(u):
    """ln u for u > 0: u = m 2^e with m in [sqrt(1/2), sqrt(2)), then
    ln m = 2 atanh(s), s = (m-1)/(m+1), summed as s * sum_k s^(2k)/(2k+1)
    for k = 0..12 (|s| <= 0.172, truncation below 1e-18)."""
    m, e = np.frexp(np.asarray(u, dtype=np.float64))  # m in [0.5, 1)
    low = m < SQRT_HALF
    m = np.where(low, m * 2.0, m)
    e = np.where(low, e - 1, e).astype(np.float64)
    s = (m - 1.0) / (m + 1.0)
    z = s * s
    p = np.full_like(s, 1.0 / 25.0)
    for k in range(11, -1, -1):
        p = p * z + 1.0 / (2 * k + 1)
    t = s * p
    return (t + t) + e * LN2


# Taylor coefficients (-1)^k / (2k+1)! and (-1)^k / (2k)!, k <= 8 and 9; all
# factorials involved are exact in FP64.
_SIN_C = [(-1.0) ** k / float(np.prod(np.arange(1, 2 * k + 2, dtype=np.float64)))
          for k in range(9)]
_COS_C = [(-1.0) ** k / float(np.prod(np.arange(1, 2 * k + 1, dtype=np.float64)))
          for k in range(10)]


def series_sincos_2pi(u):
    """(sin(2 pi u), cos(2 pi u)) for u in (0, 1): t = 4u = j + f with j the
    nearest integer, theta = f pi/2 in [-pi/4, pi/4], Taylor series of sin
    and cos of theta, then the quarter-turn identities for j mod 4."""
    t = 4.0 * np.asarray(u, dtype=np.float64)
    j = np.floor(t + 0.5)
    f = t - j
    th = f * HALF_PI
    z = th * th
    ps = np.full_like(z, _SIN_C[8])
    for k in range(7, -1, -1):
        ps = ps * z + _SIN_C[k]
    sn = th * ps
    pc = np.full_like(z, _COS_C[9])
    for k in range(8, -1, -1):
        pc = pc * z + _COS_C[k]
    cs = pc
    q = j.astype(np.int64) & 3
    sin_out = np.choose(q, [sn, cs, -sn, -cs])
    cos_out = np.choose(q, [cs, -sn, -cs, sn])
    return sin_out, cos_out


def box_muller(x_a, x_b):
    """Two uint32 words -> two N(0,1) FP64 normals (r cos, r sin)."""
    u1 = uniform_open(x_a)
    u2 = uniform_open(x_b)
    r = np.sqrt(-2.0 * series_log(u1))
    s, c = series_sincos_2pi(u2)
    return r * c, r * s


def normals(key_seed, c0, c1, step):
    """Four normals per counter: Philox4x32-10 with key = (seed lo, seed hi),
    counter = (c0, c1, step lo, step hi); words (0,1) and (2,3) each feed one
    Box-Muller pair.  c0, c1: integer arrays of equal shape -> (..., 4)."""
    c0 = np.asarray(c0, dtype=np.uint64)
    c1 = np.broadcast_to(np.asarray(c1, dtype=np.uint64), c0.shape)
    step = int(step)
    ctr = np.stack([c0.astype(np.uint32), c1.astype(np.uint32),
                    np.full(c0.shape, step & 0xFFFFFFFF, dtype=np.uint32),
                    np.full(c0.shape, (step >> 32) & 0xFFFFFFFF, dtype=np.uint32)],
                   axis=-1)
    seed = int(key_seed)
    key = np.broadcast_to(np.array([seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF],
                                   dtype=np.uint32), c0.shape + (2,))
    w = philox4x32_10(ctr, key)
    z0, z1 = box_muller(w[..., 0], w[..., 1])
    z2, z3 = box_muller(w[..., 2], w[..., 3])
    return np.stack([z0, z1, z2, z3], axis=-1)
