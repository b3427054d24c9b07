"""Pins of the slip channel of Sec. 6.3 in the oracle: walls at y = 0 and
y = H = L_y/2 of a periodic box twice the channel's height, enforced by an
image system for the blob forces and for the fluctuating stress.

* The flow of any blob forces, and the random velocity field, are mirror
  symmetric, u(x, L_y - y, z) = R u(x, y, z), so u_y = 0 and
  d u_x/dy = d u_z/dy = 0 on both walls (the slip conditions), to
  round-off; without the images they are not (power).
* The channel mobility is symmetric and positive definite.
* One blob: M_aa = S_aa(0) + R_aa S_aa(r - sigma r), the continuum lattice
  sums of the periodic box without and with its image's separation (a fine
  grid and a long cut-off remove aliasing and truncation).
* Fluctuation-dissipation inside the channel: Cov(J u_brev) = (2 kT/dt) M
  of the channel (whitened statistic), and the periodic noise fails it.
* The blob-wall harmonic force against its closed form.
"""
import math

import numpy as np
import pytest

import workloads as wl
from oracle import fcm, gdc, noise, rigid

ETA = 1.0 / (6.0 * math.pi)
SIG = 1.0 / math.sqrt(math.pi)


def _p(L, n, rc=3.0, channel=True):
    return fcm.FcmParams(fcm.Grid(L, n), ETA, SIG, rc, channel=channel)


def _mirror_rows(u):
    """u at the mirror point of every grid point: row j1 <- (n1 - j1) mod n1."""
    return np.roll(u[:, :, ::-1, :], 1, axis=2)


def _dy(u, grid):
    n1 = grid.n[1]
    k = 2 * np.pi * np.fft.fftfreq(n1, grid.L[1] / n1)
    k[n1 // 2] = 0.0
    return np.real(np.fft.ifft(1j * k[None, None, :, None] * np.fft.fft(u, axis=2), axis=2))


def _slip_residuals(u, grid):
    """max |u_y| and max |d u_x/dy|, |d u_z/dy| on the walls j1 = 0 and n1/2,
    relative to max |u|, and the mirror asymmetry."""
    n1 = grid.n[1]
    walls = [0, n1 // 2]
    du = _dy(u, grid)
    scale = np.abs(u).max()
    uy = np.abs(u[1][:, walls, :]).max() / scale
    dxz = max(np.abs(du[0][:, walls, :]).max(), np.abs(du[2][:, walls, :]).max()) / (scale / grid.dx[1])
    sym = np.abs(_mirror_rows(u) * fcm.MIRROR[:, None, None, None] - u).max() / scale
    return uy, dxz, sym


def test_flow_of_forces_is_mirror_symmetric_with_slip_walls():
    rng = np.random.default_rng(1)
    L, n = (12.0, 16.0, 12.0), (12, 16, 12)
    H = L[1] / 2
    r = np.column_stack([rng.uniform(0, L[0], 5), rng.uniform(0.4, H - 0.4, 5), rng.uniform(0, L[2], 5)])
    lam = rng.standard_normal((5, 3))
    for channel, ok in [(True, True), (False, False)]:
        p = _p(L, n, channel=channel)
        u = fcm.stokes_solve(fcm.spread_forces(fcm.weights(r, p), lam, p), p.grid, ETA)
        uy, dxz, sym = _slip_residuals(u, p.grid)
        if ok:
            assert uy < 1e-14 and dxz < 1e-12 and sym < 1e-14, (uy, dxz, sym)
        else:
            assert uy > 1e-3 and sym > 1e-3, (uy, sym)


def test_channel_noise_is_mirror_symmetric_with_slip_walls():
    g = fcm.Grid((12.0, 16.0, 12.0), (12, 16, 12))
    u = noise.channel_field(g, 1.0, ETA, 0.01, seed=4, step=3)
    uy, dxz, sym = _slip_residuals(u, g)
    assert uy < 1e-14 and dxz < 1e-12 and sym < 1e-14, (uy, dxz, sym)
    up = noise.fourier_field(g, 1.0, ETA, 0.01, seed=4, step=3)
    assert _slip_residuals(up, g)[2] > 0.1


def test_channel_mobility_symmetric_positive_definite():
    p = _p((10.0, 12.0, 10.0), (10, 12, 10))
    r = np.array([[1.2, 0.7, 3.3], [4.4, 5.1, 6.2], [7.7, 2.9, 0.5]])   # near both walls and inside
    Mm = fcm.dense_mobility(r, p)
    assert np.abs(Mm - Mm.T).max() < 1e-13 * np.abs(Mm).max()
    assert np.linalg.eigvalsh(0.5 * (Mm + Mm.T)).min() > 0.0
    # and it differs from the periodic box's near the walls
    Mp = fcm.dense_mobility(r, _p((10.0, 12.0, 10.0), (10, 12, 10), channel=False))
    assert np.abs(Mm - Mp).max() > 1e-2 * np.abs(Mp).max()


def _lattice_sum(L, sigma, sep, a, b, mmax=40):
    m = np.arange(-mmax, mmax + 1)
    K = np.meshgrid(*(2 * np.pi * m / L[d] for d in range(3)), indexing="ij")
    k2 = K[0] ** 2 + K[1] ** 2 + K[2] ** 2
    k2[mmax, mmax, mmax] = 1.0
    s = np.exp(-sigma ** 2 * k2) * ((a == b) - K[a] * K[b] / k2) / k2
    s *= np.cos(K[0] * sep[0] + K[1] * sep[1] + K[2] * sep[2])
    s[mmax, mmax, mmax] = 0.0
    return s.sum() / (ETA * np.prod(L))


def test_one_blob_mobility_is_the_lattice_sum_with_its_image():
    L = (16.0, 16.0, 16.0)
    p = _p(L, (48, 48, 48), rc=7.5)
    for h in [1.7, 3.2, 6.1]:
        r = np.array([[3.3, h, 1.9]])
        sep = r[0] - fcm.mirror_positions(r, p.grid)[0]
        for a in range(3):
            lam = np.zeros((1, 3))
            lam[0, a] = 1.0
            v = fcm.mobility_apply(r, lam, p)
            ref = _lattice_sum(L, SIG, np.zeros(3), a, a) + fcm.MIRROR[a] * _lattice_sum(L, SIG, sep, a, a)
            assert abs(v[0, a] - ref) < 1e-9, (h, a, v[0, a], ref)
            assert np.abs(np.delete(v[0], a)).max() < 1e-12


def _fdt_check(sample_fn, n_samples, p, r, kT, dt):
    W = fcm.weight_matrix(r, p.grid, p.sigma, p.rc)
    V = np.array([fcm.interp(W, sample_fn(s), p.grid).ravel() for s in range(n_samples)])
    C = (2 * kT / dt) * fcm.dense_mobility(r, p)
    Z = np.linalg.solve(np.linalg.cholesky(C), V.T).T
    Cz = Z.T @ Z / n_samples
    dev = np.abs(Cz - np.eye(Cz.shape[0])).max()
    assert dev < 6 * math.sqrt(2.0 / n_samples), dev
    assert np.abs(Z.mean(0)).max() < 6 / math.sqrt(n_samples)


def test_fluctuation_dissipation_in_the_channel():
    g = fcm.Grid((8.0, 12.0, 8.0), (8, 12, 8))
    p = fcm.FcmParams(g, ETA, SIG, 3.0, channel=True)
    r = np.array([[1.3, 0.9, 3.9], [3.4, 5.2, 5.1]])    # 0.9 from one wall, 0.8 from the other
    kT, dt = 1.0, 0.01
    _fdt_check(lambda s: noise.channel_field(g, kT, ETA, dt, seed=31, step=s), 10000, p, r, kT, dt)
    # power: the periodic noise has the periodic covariance, not the channel's
    with pytest.raises(AssertionError):
        _fdt_check(lambda s: noise.fourier_field(g, kT, ETA, dt, seed=31, step=s), 10000, p, r, kT, dt)


def test_wall_forces_closed_form():
    k, b = 40.0 / 2.2, 2.2
    s = rigid.Suspension(_p((12.0, 16.0, 12.0), (12, 16, 12)),
                         rigid.Bodies([np.zeros((1, 3))], [0, 0, 0, 0]), 1.0)
    cfg = gdc.Config(s, 1.0, 0.01, 0, gdc.Forces(wall_k=k, wall_cutoff=b))
    r = np.array([[1.0, 0.5, 1.0], [2.0, 4.0, 2.0], [3.0, 7.2, 3.0], [4.0, -0.3, 4.0]])
    f = gdc.wall_blob_forces(cfg, r)
    assert np.allclose(f[:, 1], [k * (b - 0.5), 0.0, -k * (b - 0.8), k * (b + 0.3)], rtol=0, atol=1e-14)
    assert np.all(f[:, [0, 2]] == 0.0)
    # no walls in the periodic box
    cfg.susp.fcm.channel = False
    assert np.all(gdc.wall_blob_forces(cfg, r) == 0.0)


def test_channel_step_at_zero_temperature_is_forward_euler():
    # kT = 0: the gDC step is x + dt N F with the channel's body mobility
    shapes = [wl.rod(3), wl.tetrahedron()]
    s = rigid.Suspension(_p((12.0, 16.0, 12.0), (12, 16, 12)), rigid.Bodies(shapes, [0, 1]), 1.0)
    cfg = gdc.Config(s, 0.0, 0.01, 0, gdc.Forces(wall_k=40.0 / 2.2, wall_cutoff=2.2,
                                                  const_force=np.array([0.3, -1.0, 0.2, 0.0, 0.1, 0.0])))
    Y = np.array([[4.0, 1.9, 5.0], [8.1, 5.7, 3.3]])
    q = np.array([[0.9, 0.3, 0.2, 0.1], [0.6, -0.2, 0.7, 0.3]])
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    Y1, q1, info = gdc.gdc_step(cfg, Y, q, 0, dense=True)
    r = rigid.blob_positions(s.bodies, Y, q)
    N = rigid.body_mobility(s, Y, r)
    V = (N @ gdc.body_forces(cfg, Y, r).ravel()).reshape(-1, 6)
    assert np.abs(Y1 - (Y + cfg.dt * V[:, :3])).max() < 1e-9 * cfg.dt * np.abs(V).max()
    # the wall force on the rod near y = 0 pushes it up
    assert gdc.wall_blob_forces(cfg, r)[:3, 1].max() > 0
