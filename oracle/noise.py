"""Fluctuating stress and the random velocity field (paper Sec. 4.2, Sec. 6.1).

The stress W is symmetric, white in space and time, with
<W_ab(x,t) W_cd(y,t')> = 2 eta kT (d_ac d_bd + d_ad d_bc) d(x-y) d(t-t')
(Sec. 4.2).  On the grid (Sec. 6.1, C++ FCM implementation) each point carries
six independent N(0,1) numbers; the off-diagonal ones are scaled by
sqrt(2 kT eta / dx^3) dt^{-1/2}, the diagonal ones by 2 sqrt(kT eta / dx^3)
dt^{-1/2}.  The random velocity field is
u_brev = L^-1 D W: Fourier divergence g_hat_a = i k_b W_hat_ab, then the Stokes
projection, then the inverse DFT; and v_brev = J u_brev (Sec. 4.2, eq.
fluctu_dissip).

Two generators with the same law:
  * real_space_field: the paper's construction as printed (six normals per
    grid point, scaled, then a forward DFT);
  * fourier_field (canonical): the DFT of that real field has, on every mode
    the solver keeps, independent complex Gaussians W_hat(k) with
    E|W_hat_aa|^2 = G 4 kT eta/(dV dt), E|W_hat_ab|^2 = G 2 kT eta/(dV dt)
    (a != b), real and imaginary parts independent with half that variance
    each, and W_hat(-k) = conj(W_hat(k)).  The generator draws these directly
    from Philox counters keyed by mode, which removes six forward FFTs per
    step.  On the k_2 = 0 plane only the canonical member of each +/-k pair
    is drawn and the other is its conjugate.

Philox counter of a mode: c0 = (j0 n1 + j1) (n2/2) + j2 (j2 < n2/2, the
stored half spectrum), c1 = 16*stage + call (call 0..2 gives 12 normals per
mode), (c2, c3) = step; key = seed.  Normals 2c and 2c+1 are Re and Im of
component c in the order xx, yy, zz, xy, xz, yz.

Slip channel (Sec. 6.3): the stress is given its image in the mirror half
of the box, W'(x) = (W(x) + R W(sigma x) R) / sqrt(2) (R W R flips the
xy and yz components), which keeps the random velocity mirror-symmetric
and gives Cov(J u_brev) = (2 kT/dt) M of the channel.  The oracle applies the
reflection in real space to the canonical stress field (channel_field).

Oracle code: test infrastructure only.
"""

import numpy as np
import scipy.fft

from . import philox
from . import fcm
from .fcm import Grid, wavevectors, project_spectrum

STAGE_STRESS = 0
STAGE_RFD = 1

# component c -> (a, b) of the symmetric stress
PAIRS = [(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)]


def stress_variances(grid: Grid, kT, eta, dt):
    """Real-space variances of the six stored components per grid point."""
    base = kT * eta / (grid.dV * dt)
    return np.array([4.0 * base] * 3 + [2.0 * base] * 3)


def mode_normals(grid: Grid, seed, step, stage=STAGE_STRESS):
    """12 normals per stored half-spectrum mode (j0, j1, j2 < n2/2):
    array (n0, n1, n2/2, 12)."""
    n0, n1, n2 = grid.n
    h = n2 // 2
    idx = np.arange(n0 * n1 * h, dtype=np.uint64)
    out = np.empty((n0 * n1 * h, 12))
    for call in range(3):
        out[:, 4 * call:4 * call + 4] = philox.normals(
            seed, idx, 16 * stage + call, step)
    return out.reshape(n0, n1, h, 12)


def fourier_stress(grid: Grid, kT, eta, dt, seed, step):
    """Canonical W_hat on the rfftn half spectrum (6, n0, n1, n2/2+1),
    zero on modes the solver discards (k = 0, any Nyquist index)."""
    n0, n1, n2 = grid.n
    h = n2 // 2
    z = mode_normals(grid, seed, step)
    var = stress_variances(grid, kT, eta, dt)
    scale = np.sqrt(grid.G * var / 2.0)
    W = np.zeros((6, n0, n1, h + 1), dtype=np.complex128)
    for c in range(6):
        W[c, :, :, :h] = scale[c] * (z[..., 2 * c] + 1j * z[..., 2 * c + 1])
    # Hermitian symmetry on the k2 = 0 plane: canonical member of +/-k is the
    # one with m1 > 0, or m1 == 0 and m0 > 0 (signed indices).
    m0 = np.fft.fftfreq(n0, 1.0 / n0).astype(np.int64)
    m1 = np.fft.fftfreq(n1, 1.0 / n1).astype(np.int64)
    M0, M1 = np.meshgrid(m0, m1, indexing="ij")
    canon = (M1 > 0) | ((M1 == 0) & (M0 > 0))
    J0, J1 = np.meshgrid(np.arange(n0), np.arange(n1), indexing="ij")
    P0, P1 = (-J0) % n0, (-J1) % n1
    for c in range(6):
        plane = W[c, :, :, 0].copy()
        W[c, :, :, 0] = np.where(canon, plane, np.conj(plane[P0, P1]))
    _, keep = wavevectors(grid)
    return W * keep[None]


def real_space_stress(grid: Grid, kT, eta, dt, rng):
    """The construction as printed in Sec. 6.1: six N(0,1) per grid point,
    scaled; returns the symmetric components (6, n0, n1, n2)."""
    var = stress_variances(grid, kT, eta, dt)
    z = rng.standard_normal((6,) + grid.n)
    return np.sqrt(var)[:, None, None, None] * z


def divergence_spectrum(Wh, grid: Grid):
    """g_hat_a = i sum_b k_b W_hat_ab (the Fourier divergence D W)."""
    K, _ = wavevectors(grid)
    g = np.zeros((3,) + Wh.shape[1:], dtype=np.complex128)
    for c, (a, b) in enumerate(PAIRS):
        g[a] += 1j * K[b] * Wh[c]
        if a != b:
            g[b] += 1j * K[a] * Wh[c]
    return g


def fluct_velocity_from_spectrum(Wh, grid: Grid, eta):
    """u_brev = L^-1 D W from a stress spectrum: divergence, Stokes
    projection, inverse DFT."""
    g = divergence_spectrum(Wh, grid)
    uh = project_spectrum(g, grid, eta)
    return scipy.fft.irfftn(uh, s=grid.n, axes=(1, 2, 3), workers=fcm.DEFAULT_WORKERS)


def fourier_field(grid: Grid, kT, eta, dt, seed, step):
    """Canonical random velocity field for one step, (3, n0, n1, n2)."""
    Wh = fourier_stress(grid, kT, eta, dt, seed, step)
    return fluct_velocity_from_spectrum(Wh, grid, eta)


def real_space_field(grid: Grid, kT, eta, dt, rng):
    """Random velocity field from the printed real-space construction."""
    Wr = real_space_stress(grid, kT, eta, dt, rng)
    Wh = scipy.fft.rfftn(Wr, axes=(1, 2, 3))
    return fluct_velocity_from_spectrum(Wh, grid, eta)


def mirror_stress(Wr):
    """(W + R W(sigma x) R) / sqrt(2) of a real-space stress field (6, n0, n1,
    n2): sigma maps grid row j1 to (n1 - j1) mod n1 (y -> L_y - y), and
    R W R flips the sign of the xy and yz components."""
    Wm = np.roll(Wr[:, :, ::-1, :], 1, axis=2)    # row j1 <- row (n1 - j1) mod n1
    sign = np.array([1.0, 1.0, 1.0, -1.0, 1.0, -1.0])[:, None, None, None]
    return (Wr + sign * Wm) / np.sqrt(2.0)


def channel_field(grid: Grid, kT, eta, dt, seed, step):
    """Random velocity field of the slip channel: the canonical stress
    spectrum taken to real space, reflected there (mirror_stress), and
    transformed back before the divergence and projection."""
    Wh = fourier_stress(grid, kT, eta, dt, seed, step)
    Wr = scipy.fft.irfftn(Wh, s=grid.n, axes=(1, 2, 3), workers=fcm.DEFAULT_WORKERS)
    Wh2 = scipy.fft.rfftn(mirror_stress(Wr), axes=(1, 2, 3), workers=fcm.DEFAULT_WORKERS)
    _, keep = wavevectors(grid)
    return fluct_velocity_from_spectrum(Wh2 * keep[None], grid, eta)
