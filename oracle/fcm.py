"""Fluctuating force-coupling method, deterministic part (paper Sec. 4.2).

Grid conventions: x_g = dx * g, g in {0..n_d-1} per axis d, dx_d = L_d/n_d,
dV = dx_0 dx_1 dx_2, G = n_0 n_1 n_2.  Fields are stored (3, n0, n1, n2); axis
d of the array is coordinate d of the position.  Forward DFTs are
unnormalised (e^{-i k.x}), inverse ones carry 1/G: numpy's rfftn/irfftn.
Wavenumbers k_d = 2 pi m_d / L_d with signed m_d.

What is computed (all FP64):
  * envelope  Delta_i(x) = (2 pi sigma^2)^{-3/2} exp(-|x - r_i|^2 / 2 sigma^2)
    (eq. spreading ff.), truncated to 0 beyond the cutoff radius (3a in the
    paper's implementation, Sec. 6.1), minimum-image distance, no
    renormalisation;
  * spreading f = S lambda (eq. spreading) on the grid;
  * the Fourier-spectral Stokes solve u = L^-1 f (Sec. 4.2, last paragraph):
    u_hat = (I - k k^T/|k|^2) f_hat / (eta |k|^2) with the k = 0 mode and
    every mode with an index at n_d/2 set to zero;
  * averaging v_i = J[u]_i = dV sum_g u(x_g) Delta_i(x_g) (eq. averaging, the
    trapezoidal rule), so that J = dV S^T exactly;
  * M_FCM lambda = J L^-1 S lambda (Sec. 4.2);
  * the slip channel of Sec. 6.3: walls at y = 0 and y = L_y/2 of a box of
    height L_y (the computational domain twice the channel), the flow kept
    mirror-symmetric about them by an image system: every blob force
    lambda_i at r_i has an image R lambda_i at sigma(r_i), sigma(x, y, z) =
    (x, L_y - y, z), R = diag(1, -1, 1).  A mirror-symmetric field has
    u_y = 0 and d u_x/dy = d u_z/dy = 0 on both mirror planes, the slip
    conditions; averaging reads the real blobs only.

Oracle code: test infrastructure only.
"""

from dataclasses import dataclass

import numpy as np
import scipy.fft
import scipy.sparse


# Threads for scipy.fft (None: scipy's default of one); callers that time the
# oracle may set the host's core count here.
DEFAULT_WORKERS = None


@dataclass
class Grid:
    L: np.ndarray  # (3,) box lengths
    n: tuple       # (n0, n1, n2) grid points per axis

    def __post_init__(self):
        self.L = np.asarray(self.L, dtype=np.float64).reshape(3)
        self.n = tuple(int(x) for x in self.n)
        self.dx = self.L / np.asarray(self.n, dtype=np.float64)
        self.dV = float(np.prod(self.dx))
        self.G = int(np.prod(self.n))


def envelope_norm(sigma):
    """(2 pi sigma^2)^{-3/2}, the Gaussian normalisation of eq. (spreading)."""
    return (2.0 * np.pi * sigma * sigma) ** -1.5


def blob_stencils(r, grid, sigma, rc):
    """All (blob, grid point, weight) triples with minimum-image distance
    |x_g - r_i| <= rc.  Returns (blob index, flat grid index, weight) arrays.

    Each blob's candidates are the integer points g_d in
    [ceil((r_d - rc)/dx_d), floor((r_d + rc)/dx_d)] (this set contains every
    periodic image within rc because rc < L_d/2); the distance used is the
    minimum-image one of the wrapped point."""
    r = np.asarray(r, dtype=np.float64).reshape(-1, 3)
    L, n, dx = grid.L, np.asarray(grid.n), grid.dx
    if np.any(2.0 * rc >= L):
        raise ValueError("cutoff radius must be below L/2")
    rw = r - L * np.floor(r / L)
    lo = np.ceil((rw - rc) / dx).astype(np.int64)
    hi = np.floor((rw + rc) / dx).astype(np.int64)
    span = (hi - lo + 1).max(axis=0)
    offs = np.stack(np.meshgrid(*[np.arange(s) for s in span], indexing="ij"),
                    axis=-1).reshape(-1, 3)
    M = r.shape[0]
    g = lo[:, None, :] + offs[None, :, :]                  # (M, P, 3) unwrapped
    gw = np.mod(g, n)                                      # wrapped indices
    d = gw * dx - rw[:, None, :]
    d = d - L * np.round(d / L)                            # minimum image
    d2 = np.sum(d * d, axis=-1)
    keep = (g <= hi[:, None, :]).all(axis=-1) & (d2 <= rc * rc)
    w = envelope_norm(sigma) * np.exp(-d2 / (2.0 * sigma * sigma))
    flat = (gw[..., 0] * n[1] + gw[..., 1]) * n[2] + gw[..., 2]
    bi = np.broadcast_to(np.arange(M)[:, None], flat.shape)
    return bi[keep], flat[keep], w[keep]


def weight_matrix(r, grid, sigma, rc):
    """Sparse (M x G) matrix W with W[i, g] = Delta_i(x_g) (truncated)."""
    bi, gi, w = blob_stencils(r, grid, sigma, rc)
    M = np.asarray(r).reshape(-1, 3).shape[0]
    return scipy.sparse.csr_matrix((w, (bi, gi)), shape=(M, grid.G))


def spread(W, lam, grid):
    """f = S lambda on the grid, eq. (spreading): f(x_g) = sum_i lambda_i
    Delta_i(x_g).  lam: (M, 3) -> (3, n0, n1, n2)."""
    lam = np.asarray(lam, dtype=np.float64).reshape(-1, 3)
    f = W.T @ lam                                          # (G, 3)
    return np.ascontiguousarray(f.T).reshape((3,) + grid.n)


def interp(W, u, grid):
    """v = J[u], eq. (averaging) by the trapezoidal rule:
    v_i = dV sum_g u(x_g) Delta_i(x_g).  u: (3, n0, n1, n2) -> (M, 3)."""
    uf = np.asarray(u, dtype=np.float64).reshape(3, -1)
    return grid.dV * (W @ uf.T)


def wavevectors(grid):
    """k_d = 2 pi m_d / L_d on the rfftn half spectrum, with the mask of the
    modes the solver keeps (k != 0, no index at n_d/2)."""
    n0, n1, n2 = grid.n
    m0 = np.fft.fftfreq(n0, 1.0 / n0)
    m1 = np.fft.fftfreq(n1, 1.0 / n1)
    m2 = np.arange(n2 // 2 + 1, dtype=np.float64)
    k0 = (2.0 * np.pi / grid.L[0]) * m0[:, None, None]
    k1 = (2.0 * np.pi / grid.L[1]) * m1[None, :, None]
    k2 = (2.0 * np.pi / grid.L[2]) * m2[None, None, :]
    j0 = np.arange(n0)[:, None, None]
    j1 = np.arange(n1)[None, :, None]
    j2 = np.arange(n2 // 2 + 1)[None, None, :]
    keep = (j0 != n0 // 2) & (j1 != n1 // 2) & (j2 != n2 // 2)
    keep = keep & ~((j0 == 0) & (j1 == 0) & (j2 == 0))
    K = np.broadcast_arrays(k0, k1, k2)
    return [np.asarray(x) for x in K], keep


def project_spectrum(fh, grid, eta):
    """u_hat = (I - k k^T/|k|^2) f_hat / (eta |k|^2) on kept modes, 0 elsewhere
    (Fourier form of eq. fluc_stokes1/2 with the pressure eliminated)."""
    K, keep = wavevectors(grid)
    k2 = K[0] ** 2 + K[1] ** 2 + K[2] ** 2
    k2s = np.where(keep, k2, 1.0)
    kdotf = K[0] * fh[0] + K[1] * fh[1] + K[2] * fh[2]
    uh = np.empty_like(fh)
    for a in range(3):
        uh[a] = np.where(keep, (fh[a] - K[a] * kdotf / k2s) / (eta * k2s), 0.0)
    return uh


def stokes_solve(f, grid, eta, workers=None):
    """u = L^-1 f on the periodic grid (Sec. 4.2): rfftn, projection, irfftn."""
    workers = DEFAULT_WORKERS if workers is None else workers
    fh = scipy.fft.rfftn(f, axes=(1, 2, 3), workers=workers)
    uh = project_spectrum(fh, grid, eta)
    return scipy.fft.irfftn(uh, s=grid.n, axes=(1, 2, 3), workers=workers)


@dataclass
class FcmParams:
    grid: Grid
    eta: float
    sigma: float
    rc: float
    channel: bool = False   # slip walls at y = 0 and y = L_y/2 by images (Sec. 6.3)


# R: the mirror image of a force about a plane y = const flips its y component
MIRROR = np.array([1.0, -1.0, 1.0])


def mirror_positions(r, grid):
    """sigma(r) = (x, L_y - y, z): the image of each blob about the wall
    y = L_y/2 (equivalently about y = 0, the box being periodic in y)."""
    m = np.array(r, dtype=np.float64).reshape(-1, 3)
    m[:, 1] = grid.L[1] - m[:, 1]
    return m


def weights(r, p: FcmParams):
    """(W, W_image): weight matrices of the blobs and, in the slip channel,
    of their images (None in a periodic box)."""
    W = weight_matrix(r, p.grid, p.sigma, p.rc)
    Wm = weight_matrix(mirror_positions(r, p.grid), p.grid, p.sigma, p.rc) if p.channel else None
    return W, Wm


def spread_forces(Ws, lam, p: FcmParams):
    """f = S lambda, plus the image forces R lambda_i at sigma(r_i) in the
    slip channel."""
    W, Wm = Ws
    f = spread(W, lam, p.grid)
    if Wm is not None:
        f = f + spread(Wm, np.asarray(lam, dtype=np.float64).reshape(-1, 3) * MIRROR, p.grid)
    return f


def mobility_apply(r, lam, p: FcmParams, workers=None):
    """M_FCM lambda = J L^-1 S lambda (Sec. 4.2), with the images of the slip
    channel when p.channel.  r, lam: (M, 3) -> (M, 3)."""
    Ws = weights(r, p)
    u = stokes_solve(spread_forces(Ws, lam, p), p.grid, p.eta, workers)
    return interp(Ws[0], u, p.grid)


def dense_mobility(r, p: FcmParams):
    """The 3M x 3M matrix M_FCM, assembled column by column (small M only)."""
    r = np.asarray(r, dtype=np.float64).reshape(-1, 3)
    M = r.shape[0]
    Ws = weights(r, p)
    out = np.empty((3 * M, 3 * M))
    for j in range(3 * M):
        lam = np.zeros(3 * M)
        lam[j] = 1.0
        f = spread_forces(Ws, lam.reshape(M, 3), p)
        out[:, j] = interp(Ws[0], stokes_solve(f, p.grid, p.eta), p.grid).reshape(-1)
    return out
