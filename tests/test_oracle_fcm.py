"""Pins of oracle.fcm: brute-force DFTs, closed-form Stokes solutions, the
periodic single-blob lattice sum (and Hasimoto's finite-size law), the
adjointness J = dV S^T, symmetry and positive definiteness of M_FCM."""
import math

import numpy as np

from oracle import fcm

ETA = 1.0 / (6.0 * math.pi)
A = 1.0
SIG = A / math.sqrt(math.pi)


def _params(L, n, rc=3.0 * A, sigma=SIG):
    return fcm.FcmParams(fcm.Grid(L if np.ndim(L) else [L] * 3, n if np.ndim(n) else (n,) * 3),
                         ETA, sigma, rc)


def _pou_bound(sigma, dx, rc):
    # Poisson summation: the first aliases contribute 6 exp(-2 pi^2 sigma^2/dx^2)
    # (three axes, +/- one reciprocal-lattice vector); the truncation removes the
    # Gaussian mass beyond rc, erfc(x/sqrt2) + sqrt(2/pi) x exp(-x^2/2), x = rc/sigma.
    x = rc / sigma
    tail = math.erfc(x / math.sqrt(2)) + math.sqrt(2 / math.pi) * x * math.exp(-x * x / 2)
    return 1.1 * (6 * math.exp(-2 * math.pi ** 2 * sigma ** 2 / dx ** 2) + tail)


def test_partition_of_unity_within_aliasing_bound():
    # dV sum_g Delta_i(x_g) = 1 up to aliasing and truncation (bounds above):
    # ~1.2e-2 at dx = a, ~8e-6 at dx = 2a/3.
    rng = np.random.default_rng(0)
    for L, n in [(16.0, 16), (16.0, 24)]:
        p = _params(L, n)
        bound = _pou_bound(p.sigma, p.grid.dx[0], p.rc)
        r = rng.uniform(0, L, (20, 3))
        W = fcm.weight_matrix(r, p.grid, p.sigma, p.rc)
        s = p.grid.dV * np.asarray(W.sum(axis=1)).ravel()
        assert np.abs(s - 1).max() < bound


def test_stencil_is_minimum_image_sphere():
    p = _params(12.0, 12)
    r = np.array([[0.2, 11.9, 6.0]])
    bi, gi, w = fcm.blob_stencils(r, p.grid, p.sigma, p.rc)
    g = np.stack(np.unravel_index(gi, p.grid.n), axis=1) * p.grid.dx
    d = g - r
    d -= p.grid.L * np.round(d / p.grid.L)
    assert np.all((d * d).sum(1) <= 9.0 + 1e-12)
    # brute force over the whole grid
    allg = np.stack(np.meshgrid(*[np.arange(12)] * 3, indexing="ij"), -1).reshape(-1, 3) * 1.0
    dd = allg - r
    dd -= 12.0 * np.round(dd / 12.0)
    assert len(gi) == int(((dd * dd).sum(1) <= 9.0).sum())


def _brute_stokes(f, grid, eta):
    """Explicit-sum DFT, projection and inverse DFT on the full spectrum."""
    n0, n1, n2 = grid.n
    idx = np.stack(np.meshgrid(np.arange(n0), np.arange(n1), np.arange(n2), indexing="ij"), -1).reshape(-1, 3)
    x = idx * grid.dx
    m = idx.copy()
    for d, nd in enumerate(grid.n):
        m[:, d] = np.where(m[:, d] < nd // 2, m[:, d], m[:, d] - nd)
    k = 2 * np.pi * m / grid.L
    E = np.exp(-1j * (k @ x.T))                         # (modes, points)
    fh = E @ f.reshape(3, -1).T                          # (modes, 3)
    nyq = np.zeros(len(idx), bool)
    for d, nd in enumerate(grid.n):
        nyq |= idx[:, d] == nd // 2
    k2 = (k * k).sum(1)
    keep = (~nyq) & (k2 > 0)
    uh = np.zeros_like(fh)
    kk = k[keep]
    ff = fh[keep]
    uh[keep] = (ff - kk * ((kk * ff).sum(1) / k2[keep])[:, None]) / (eta * k2[keep])[:, None]
    u = (E.conj().T @ uh) / grid.G
    assert np.abs(u.imag).max() < 1e-10 * np.abs(u.real).max()
    return u.real.T.reshape(f.shape)


def test_stokes_solve_equals_brute_force_dft():
    rng = np.random.default_rng(1)
    for n in [(8, 8, 8), (6, 8, 4)]:
        p = _params([8.0, 9.0, 7.0], n)
        f = rng.standard_normal((3,) + p.grid.n)
        u = fcm.stokes_solve(f, p.grid, ETA)
        ub = _brute_stokes(f, p.grid, ETA)
        assert np.abs(u - ub).max() < 1e-12 * np.abs(ub).max()


def test_plane_wave_closed_form():
    # f = sin(k y) e_x is divergence-free: the Stokes solution is f/(eta k^2);
    # a longitudinal force grad(phi) is balanced by pressure: u = 0.
    p = _params([10.0, 12.0, 14.0], (10, 12, 14))
    g = p.grid
    y = np.arange(g.n[1]) * g.dx[1]
    k = 2 * np.pi * 2 / g.L[1]
    f = np.zeros((3,) + g.n)
    f[0] = np.sin(k * y)[None, :, None]
    u = fcm.stokes_solve(f, g, ETA)
    assert np.abs(u - f / (ETA * k * k)).max() < 1e-12
    f2 = np.zeros((3,) + g.n)
    f2[1] = np.cos(k * y)[None, :, None]
    assert np.abs(fcm.stokes_solve(f2, g, ETA)).max() < 1e-12


def test_spectral_velocity_is_divergence_free():
    rng = np.random.default_rng(2)
    p = _params(8.0, 8)
    u = fcm.stokes_solve(rng.standard_normal((3, 8, 8, 8)), p.grid, ETA)
    uh = np.fft.rfftn(u, axes=(1, 2, 3))
    K, _ = fcm.wavevectors(p.grid)
    div = K[0] * uh[0] + K[1] * uh[1] + K[2] * uh[2]
    assert np.abs(div).max() < 1e-12 * np.abs(uh).max()


def _lattice_sum(L, sigma, sep=np.zeros(3), a_idx=0, b_idx=0, mmax=60):
    m = np.arange(-mmax, mmax + 1)
    kk = 2 * np.pi * m / L
    K = np.meshgrid(kk, kk, kk, indexing="ij")
    k2 = K[0] ** 2 + K[1] ** 2 + K[2] ** 2
    k2[mmax, mmax, mmax] = 1.0
    s = np.exp(-sigma ** 2 * k2) * ((a_idx == b_idx) - K[a_idx] * K[b_idx] / k2) / k2
    s *= np.cos(K[0] * sep[0] + K[1] * sep[1] + K[2] * sep[2])
    s[mmax, mmax, mmax] = 0.0
    return s.sum() / (ETA * L ** 3)


def test_single_blob_periodic_mobility():
    # A fine grid (sigma/dx = 1.69) and a long cutoff remove aliasing, spectral
    # truncation and envelope truncation: the grid mobility equals the
    # continuum lattice sum
    # (1/(eta L^3)) sum_{k != 0} e^{-sigma^2 k^2} (1 - k_a^2/k^2)/k^2.
    L = 16.0
    p = _params(L, 48, rc=7.5)
    r = np.array([[3.3, 7.1, 1.9]])
    v = fcm.mobility_apply(r, np.array([[1.0, 0, 0]]), p)
    ref = _lattice_sum(L, SIG)
    assert abs(v[0, 0] - ref) < 1e-9
    assert np.abs(v[0, 1:]).max() < 1e-12
    # Hasimoto (1959): 6 pi eta a M = 1 - 2.837297 a/L + O((a/L)^3); at L = 32a
    # the O(a^3/L^3) remainder is ~1.3e-4.
    ref32 = _lattice_sum(32.0, SIG)
    assert abs(ref32 - (1 - 2.837297 / 32)) < 3e-4
    p32 = _params(32.0, 48)
    v32 = fcm.mobility_apply(r, np.array([[0, 0, 1.0]]), p32)
    assert abs(v32[0, 2] - (1 - 2.837297 / 32)) < 4e-4
    # at L = 64a the remainder is ~1.6e-5; the isolated-blob limit
    # 1/(6 pi eta a) = 1 is approached as 1 - 2.837297 a/L
    assert abs(_lattice_sum(64.0, SIG, mmax=110) - (1 - 2.837297 / 64)) < 3e-5


def test_two_blob_pair_mobility_lattice_sum():
    L = 16.0
    p = _params(L, 48, rc=7.5)
    r = np.array([[2.0, 3.0, 4.0], [5.1, 6.3, 2.2]])
    sep = r[0] - r[1]
    lam = np.zeros((2, 3))
    lam[1, 1] = 1.0
    v = fcm.mobility_apply(r, lam, p)
    for a in range(3):
        assert abs(v[0, a] - _lattice_sum(L, SIG, sep, a, 1)) < 1e-9


def test_adjointness_and_symmetry():
    rng = np.random.default_rng(3)
    p = _params(12.0, 16)
    r = rng.uniform(0, 12.0, (5, 3))
    W = fcm.weight_matrix(r, p.grid, p.sigma, p.rc)
    lam = rng.standard_normal((5, 3))
    u = rng.standard_normal((3,) + p.grid.n)
    lhs = p.grid.dV * np.sum(fcm.spread(W, lam, p.grid) * u)
    rhs = np.sum(lam * fcm.interp(W, u, p.grid))
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)
    Mm = fcm.dense_mobility(r, p)
    assert np.abs(Mm - Mm.T).max() < 1e-13 * np.abs(Mm).max()
    assert np.linalg.eigvalsh(0.5 * (Mm + Mm.T)).min() > 0


def test_grid_translation_and_rotation_invariance():
    rng = np.random.default_rng(4)
    p = _params(12.0, 12)
    r = rng.uniform(0, 12.0, (4, 3))
    Mm = fcm.dense_mobility(r, p)
    Mt = fcm.dense_mobility(r + np.array([3.0, -2.0, 7.0]), p)   # whole grid cells (dx = 1)
    assert np.abs(Mm - Mt).max() < 1e-13 * np.abs(Mm).max()
    # 90 degree rotation about z (x, y) -> (-y, x): M -> R M R^T blockwise
    Rz = np.array([[0, -1, 0], [1, 0, 0], [0, 0, 1.0]])
    Mr = fcm.dense_mobility(r @ Rz.T, p)
    B = np.kron(np.eye(4), Rz)
    assert np.abs(Mr - B @ Mm @ B.T).max() < 1e-13 * np.abs(Mm).max()
