"""Pins of oracle.noise: the Hermitian construction, the per-mode law of the
stress spectrum, and the fluctuation-dissipation theorem
Cov(v_brev) = (2 kT/dt) M_FCM (eq. fluctu_dissip) for both the canonical
Fourier-space generator and the real-space construction printed in Sec. 6.1."""
import math

import numpy as np
import pytest

from oracle import fcm, noise

ETA = 1.0 / (6.0 * math.pi)
SIG = 1.0 / math.sqrt(math.pi)


def test_hermitian_plane_and_zeroed_modes():
    g = fcm.Grid([8.0, 10.0, 12.0], (8, 10, 12))
    W = noise.fourier_stress(g, 1.0, ETA, 0.01, seed=3, step=5)
    n0, n1, _ = g.n
    for j0 in range(n0):
        for j1 in range(n1):
            assert np.allclose(W[:, j0, j1, 0], np.conj(W[:, (-j0) % n0, (-j1) % n1, 0]), rtol=0, atol=0)
    assert np.all(W[:, 0, 0, 0] == 0)
    assert np.all(W[:, n0 // 2] == 0) and np.all(W[:, :, n1 // 2] == 0) and np.all(W[:, :, :, -1] == 0)
    # the Hermitian completion of the half spectrum is a real field
    full = np.fft.irfftn(W, s=g.n, axes=(1, 2, 3))
    back = np.fft.rfftn(full, axes=(1, 2, 3))
    assert np.abs(back - W).max() < 1e-12 * np.abs(W).max()


def test_per_mode_variance():
    g = fcm.Grid([32.0] * 3, (32,) * 3)
    kT, dt = 1.3, 0.02
    W = noise.fourier_stress(g, kT, ETA, dt, seed=11, step=0)
    var = noise.stress_variances(g, kT, ETA, dt)
    _, keep = fcm.wavevectors(g)
    sel = keep.copy()
    sel[:, :, 0] = False           # independent modes only
    nmodes = sel.sum()
    for c in range(6):
        w = W[c][sel]
        ratio = np.mean(np.abs(w) ** 2) / (g.G * var[c])
        assert abs(ratio - 1) < 6 / math.sqrt(nmodes)
        assert abs(np.mean(w.real ** 2) / np.mean(w.imag ** 2) - 1) < 9 / math.sqrt(nmodes)
        assert abs(np.mean(w.real * w.imag)) < 6 * g.G * var[c] / 2 / math.sqrt(nmodes)


def test_velocity_spectrum_divergence_free():
    g = fcm.Grid([8.0] * 3, (8,) * 3)
    u = noise.fourier_field(g, 1.0, ETA, 0.01, seed=1, step=2)
    uh = np.fft.rfftn(u, axes=(1, 2, 3))
    K, _ = fcm.wavevectors(g)
    assert np.abs(K[0] * uh[0] + K[1] * uh[1] + K[2] * uh[2]).max() < 1e-12 * np.abs(uh).max()


def _fdt_check(sample_fn, n_samples, p, r, kT, dt):
    W = fcm.weight_matrix(r, p.grid, p.sigma, p.rc)
    V = np.array([fcm.interp(W, sample_fn(s), p.grid).ravel() for s in range(n_samples)])
    C = (2 * kT / dt) * fcm.dense_mobility(r, p)
    Lc = np.linalg.cholesky(C)
    Z = np.linalg.solve(Lc, V.T).T                 # whitened: Cov(Z) = I under the law
    Cz = Z.T @ Z / n_samples
    dev = np.abs(Cz - np.eye(Cz.shape[0])).max()
    assert dev < 6 * math.sqrt(2.0 / n_samples), dev
    assert np.abs(Z.mean(0)).max() < 6 / math.sqrt(n_samples)


@pytest.mark.parametrize("mode", ["fourier", "real_space"])
def test_fluctuation_dissipation(mode):
    g = fcm.Grid([8.0] * 3, (8,) * 3)
    p = fcm.FcmParams(g, ETA, SIG, 3.0)
    r = np.array([[1.3, 2.2, 3.9], [3.4, 3.0, 5.1]])
    kT, dt, ns = 1.0, 0.01, 10000
    if mode == "fourier":
        fn = lambda s: noise.fourier_field(g, kT, ETA, dt, seed=21, step=s)  # noqa: E731
    else:
        rng = np.random.default_rng(5)
        fn = lambda s: noise.real_space_field(g, kT, ETA, dt, rng)  # noqa: E731
    _fdt_check(fn, ns, p, r, kT, dt)


def test_fdt_check_has_power():
    # a planted mistake (off-diagonal stress variance doubled) must fail the
    # same check: the test can tell a wrong law from the right one
    g = fcm.Grid([8.0] * 3, (8,) * 3)
    p = fcm.FcmParams(g, ETA, SIG, 3.0)
    r = np.array([[1.3, 2.2, 3.9], [3.4, 3.0, 5.1]])

    def wrong(s):
        Wh = noise.fourier_stress(g, 1.0, ETA, 0.01, seed=21, step=s)
        Wh[3:] *= math.sqrt(2.0)
        return noise.fluct_velocity_from_spectrum(Wh, g, ETA)
    with pytest.raises(AssertionError):
        _fdt_check(wrong, 10000, p, r, 1.0, 0.01)
