"""The gDC time step (paper Sec. 3), the Euler-Maruyama step (Appendix D) and
the force models of the synthetic workloads.

One gDC step from x^n = (Y^n, q^n) (Lie-algebra elements reset to 0):
  1. draw the stress noise; u_brev = L^-1 D W for this step (Sec. 4.2/5:
     only J depends on the configuration, so the field is reused);
  2. v_brev^n = J(x^n) u_brev, calV^n = (K^T K)^+ K^T v_brev^n (eq. unconst,
     eq. sol_unconst);
  3. nu = 1 + dt/2 (d_x . calV)^n, the divergence by forward differences
     (eq. FD) with translations scaled by L_p (footnote of step 3), or by
     random finite differences (eq. rfd_div);
  4. x^m = x^n + dt/2 calV^n, q^m = exp(u^m) . q^n;
  5. solve the full saddle problem at x^m with the same W (eq. step5);
  6. x^{n+1} = x^n + nu dt V^m, q^{n+1} = exp(u^{n+1}) . q^n.

Readings where the paper is silent: nu is one scalar for the whole
suspension (the sum over p and i in eq. FD); the update uses
u^{n+1} = nu dt Omega^m literally (no dexpinv factor); forces act only at
the midpoint; L_p = max blob-blob distance in body p, or the blob radius for
a single blob.

Oracle code: test infrastructure only.
"""

from dataclasses import dataclass, field

import numpy as np
from scipy.spatial import cKDTree

from . import fcm, noise, philox, rigid
from .quaternion import qexp, qmul


@dataclass
class Forces:
    """Force model of the synthetic workloads.
    steric_k, steric_cutoff: harmonic blob-pair repulsion V = (k/2)(r - b)^2
      for r < b between blobs of different bodies (the harmonic potential of
      Sec. 6.3 used between blob pairs; k = 40 kT/(a b), b = 2.2 a there);
    const_force: (6,) force and torque applied to every body;
    shear_rate: imposed background flow u_inf = rate (y - L_y/2) e_x, with y
      measured from the body's wrapped centre so the flow is continuous
      across each body (not Lees-Edwards);
    sine_force: f0 of the periodic force density f0 sin(k y) e_x on the
      fluid, k = 2 pi / L_y (Sec. 6.4, rheology);
    wall_k, wall_cutoff: in the slip channel, the harmonic blob-wall
      repulsion V(h) = (k/2)(h - b)^2 for h < b, h the blob's distance from
      the wall y = 0 or y = L_y/2 (Sec. 6.3: b = 2.2a, k = 40 kT/(a b))."""
    steric_k: float = 0.0
    steric_cutoff: float = 0.0
    const_force: np.ndarray = field(default_factory=lambda: np.zeros(6))
    shear_rate: float = 0.0
    sine_force: float = 0.0
    wall_k: float = 0.0
    wall_cutoff: float = 0.0


@dataclass
class Config:
    susp: rigid.Suspension
    kT: float
    dt: float
    seed: int
    forces: Forces
    fd_delta: float = 1e-6
    divergence: str = "fd"      # "fd" or "rfd"


def body_length(shape, a):
    """L_p: the maximum distance between two blobs of the body (footnote to
    step 3); the blob radius a for a one-blob body."""
    b = np.asarray(shape)
    if b.shape[0] < 2:
        return a
    d = b[:, None, :] - b[None, :, :]
    return float(np.sqrt((d * d).sum(-1)).max())


def steric_blob_forces(cfg: Config, r):
    """Blob forces of the harmonic pair repulsion, minimum image, pairs of
    blobs in different bodies only.  -> (M, 3)."""
    f = np.zeros_like(r)
    F = cfg.forces
    if F.steric_k == 0.0 or F.steric_cutoff <= 0.0:
        return f
    grid = cfg.susp.fcm.grid
    rw = r - grid.L * np.floor(r / grid.L)
    tree = cKDTree(rw, boxsize=grid.L)
    pairs = tree.query_pairs(F.steric_cutoff, output_type="ndarray")
    if pairs.size == 0:
        return f
    body = cfg.susp.bodies.body_of_blob()
    pairs = pairs[body[pairs[:, 0]] != body[pairs[:, 1]]]
    d = rw[pairs[:, 0]] - rw[pairs[:, 1]]
    d = d - grid.L * np.round(d / grid.L)
    dist = np.sqrt((d * d).sum(-1))
    inside = dist < F.steric_cutoff
    pairs, d, dist = pairs[inside], d[inside], dist[inside]
    mag = F.steric_k * (F.steric_cutoff - dist)        # -dV/dr > 0: repulsive
    fij = (mag / dist)[:, None] * d
    np.add.at(f, pairs[:, 0], fij)
    np.add.at(f, pairs[:, 1], -fij)
    return f


def wall_blob_forces(cfg: Config, r):
    """Blob forces of the harmonic wall repulsion of the slip channel (Sec.
    6.3): along +y, k (b - y) when y < b (wall y = 0); along -y,
    k (b - (H - y)) when H - y < b (wall y = H, H = L_y/2 the channel
    height).  y is the blob's coordinate as stepped (not wrapped), so a blob
    pushed through a wall feels a force that grows with the depth.  -> (M, 3)."""
    f = np.zeros_like(r)
    F = cfg.forces
    if not cfg.susp.fcm.channel or F.wall_k == 0.0 or F.wall_cutoff <= 0.0:
        return f
    H = 0.5 * cfg.susp.fcm.grid.L[1]
    y = r[:, 1]
    lo = y < F.wall_cutoff
    hi = H - y < F.wall_cutoff
    f[lo, 1] += F.wall_k * (F.wall_cutoff - y[lo])
    f[hi, 1] -= F.wall_k * (F.wall_cutoff - (H - y[hi]))
    return f


def body_forces(cfg: Config, Y, r):
    """F^m: (N, 6) force and torque on each body = K^T f_blob + constant."""
    b = cfg.susp.bodies
    F = rigid.KT_apply(b, Y, r, steric_blob_forces(cfg, r) + wall_blob_forces(cfg, r))
    return F + np.asarray(cfg.forces.const_force, dtype=np.float64)[None, :]


def sine_average(cfg: Config, r):
    """s_i = J[sin(k y)](r_i): the averaged sine profile at each blob (the
    trapezoidal average of eq. averaging), k = 2 pi / L_y."""
    p = cfg.susp.fcm
    grid = p.grid
    k = 2.0 * np.pi / grid.L[1]
    field = np.zeros((3,) + grid.n)
    field[0] = np.sin(k * grid.dx[1] * np.arange(grid.n[1]))[None, :, None]
    W = fcm.weight_matrix(r, grid, p.sigma, p.rc)
    return fcm.interp(W, field, grid)[:, 0]


def sine_flow_scale(cfg: Config):
    """f0 / (eta k^2): the fluid velocity amplitude the forcing f0 sin(k y) e_x
    drives alone.  The single Fourier mode is unchanged by the projection, so
    on the grid L^-1 f = f0/(eta k^2) sin(k y_g) e_x exactly."""
    k = 2.0 * np.pi / cfg.susp.fcm.grid.L[1]
    return cfg.forces.sine_force / (cfg.susp.fcm.eta * k * k)


def sine_amplitude(cfg: Config, r, lam):
    """v_x, the sin(k y) amplitude of the x-velocity of the fluid at a solved
    configuration: the sine mode of L^-1 (S lambda + f0 sin(k y) e_x), i.e.
    (f0 + (2/V) sum_i lambda_ix s_i) / (eta k^2) with s_i = J[sin(k y)](r_i)
    (the blob forces seen by the grid's sine mode; V the box volume).  The
    effective viscosity is eta_eff = f0 / (k^2 v_x)."""
    grid = cfg.susp.fcm.grid
    k = 2.0 * np.pi / grid.L[1]
    V = float(np.prod(grid.L))
    s_i = sine_average(cfg, r)
    return (cfg.forces.sine_force + (2.0 / V) * float(lam[:, 0] @ s_i)) / (cfg.susp.fcm.eta * k * k)


def background_flow(cfg: Config, Y, r):
    """u_inf at every blob: the shear profile and the averaged flow of the
    sine forcing (zero when neither is set)."""
    out = np.zeros_like(r)
    if cfg.forces.sine_force != 0.0:
        out[:, 0] += sine_flow_scale(cfg) * sine_average(cfg, r)
    g = cfg.forces.shear_rate
    if g == 0.0:
        return out
    Ly = cfg.susp.fcm.grid.L[1]
    b = cfg.susp.bodies
    Yb = np.asarray(Y).reshape(-1, 3)[b.body_of_blob()]
    ywrap = (Yb[:, 1] - Ly * np.floor(Yb[:, 1] / Ly)) + (r[:, 1] - Yb[:, 1])
    out[:, 0] += g * (ywrap - 0.5 * Ly)
    return out


def fluct_field(cfg: Config, step):
    """u_brev of the step: the canonical field, or the mirror-symmetric one of
    the slip channel."""
    p = cfg.susp.fcm
    if p.channel:
        return noise.channel_field(p.grid, cfg.kT, p.eta, cfg.dt, cfg.seed, step)
    return noise.fourier_field(p.grid, cfg.kT, p.eta, cfg.dt, cfg.seed, step)


def averaged(cfg: Config, r, u):
    p = cfg.susp.fcm
    W = fcm.weight_matrix(r, p.grid, p.sigma, p.rc)
    return fcm.interp(W, u, p.grid)


def predictor(cfg: Config, Y, q, ufl):
    """Steps 2-3: calV^n (N, 6) and the per-body forward-difference
    divergences d_p, so that nu = 1 + dt/2 sum_p d_p.

    Perturbing body p alone changes only calV^(p) (calV is per body and the
    field is fixed), so the six perturbations are applied to all bodies at
    once and differenced body by body."""
    b = cfg.susp.bodies
    Y = np.asarray(Y, dtype=np.float64).reshape(-1, 3)
    q = np.asarray(q, dtype=np.float64).reshape(-1, 4)
    r = rigid.blob_positions(b, Y, q)
    calV = rigid.lsq_velocity(b, Y, r, averaged(cfg, r, ufl))
    delta = cfg.fd_delta
    Lp = np.array([body_length(b.shapes[s], cfg.susp.a) for s in b.body_shape])
    d = np.zeros(b.N)
    for al in range(3):
        Yp = Y.copy()
        Yp[:, al] += delta * Lp
        rp = rigid.blob_positions(b, Yp, q)
        Vp = rigid.lsq_velocity(b, Yp, rp, averaged(cfg, rp, ufl))
        d += (Vp[:, al] - calV[:, al]) / (delta * Lp)
    for al in range(3):
        e = np.zeros((b.N, 3))
        e[:, al] = delta
        qp = qmul(qexp(e), q)
        rp = rigid.blob_positions(b, Y, qp)
        Vp = rigid.lsq_velocity(b, Y, rp, averaged(cfg, rp, ufl))
        d += (Vp[:, 3 + al] - calV[:, 3 + al]) / delta
    return calV, d


def rfd_divergence(cfg: Config, Y, q, ufl, calV, step):
    """Random finite difference (eq. rfd_div): W~ ~ N(0,1)^{6N} from Philox
    (stage 1, counter c0 = body, two calls of which the first six normals are
    used), translations scaled by L_p; returns per-body terms d_p whose sum
    has the divergence as its expectation (pinned by that law against the
    forward-difference divergence)."""
    b = cfg.susp.bodies
    Y = np.asarray(Y, dtype=np.float64).reshape(-1, 3)
    q = np.asarray(q, dtype=np.float64).reshape(-1, 4)
    idx = np.arange(b.N, dtype=np.uint64)
    z = np.concatenate([philox.normals(cfg.seed, idx, 16 * noise.STAGE_RFD + c, step)
                        for c in range(2)], axis=-1)[:, :6]
    delta = cfg.fd_delta
    Lp = np.array([body_length(b.shapes[s], cfg.susp.a) for s in b.body_shape])
    Yp = Y + delta * Lp[:, None] * z[:, :3]
    qp = qmul(qexp(delta * z[:, 3:]), q)
    rp = rigid.blob_positions(b, Yp, qp)
    Vp = rigid.lsq_velocity(b, Yp, rp, averaged(cfg, rp, ufl))
    dV = Vp - calV
    return (z[:, :3] * dV[:, :3]).sum(-1) / (delta * Lp) + (z[:, 3:] * dV[:, 3:]).sum(-1) / delta


def midpoint(cfg: Config, Y, q, calV):
    """Step 4: Y^m = Y^n + dt/2 calV_U, q^m = exp(dt/2 calV_Omega) . q^n."""
    h = 0.5 * cfg.dt
    return Y + h * calV[:, :3], qmul(qexp(h * calV[:, 3:]), q)


def corrector_solve(cfg: Config, Ym, qm, ufl, tol=1e-12, dense=None):
    """Step 5 at x^m: V^m from the saddle problem with slip v_brev^m + u_inf
    and body forces F^m."""
    b = cfg.susp.bodies
    rm = rigid.blob_positions(b, Ym, qm)
    slip = averaged(cfg, rm, ufl) + background_flow(cfg, Ym, rm)
    F = body_forces(cfg, Ym, rm)
    lam, V, info = rigid.solve_saddle(cfg.susp, Ym, rm, slip, F, tol=tol, dense=dense)
    if cfg.forces.sine_force != 0.0:
        info["sine_vx"] = sine_amplitude(cfg, rm, lam)
    return V, info


def gdc_step(cfg: Config, Y, q, step, tol=1e-12, dense=None):
    """One gDC step (Sec. 3).  Returns (Y^{n+1}, q^{n+1}, diagnostics)."""
    Y = np.asarray(Y, dtype=np.float64).reshape(-1, 3)
    q = np.asarray(q, dtype=np.float64).reshape(-1, 4)
    ufl = fluct_field(cfg, step)
    calV, d = predictor(cfg, Y, q, ufl)
    if cfg.divergence == "rfd":
        d = rfd_divergence(cfg, Y, q, ufl, calV, step)
    nu = 1.0 + 0.5 * cfg.dt * d.sum()
    Ym, qm = midpoint(cfg, Y, q, calV)
    V, info = corrector_solve(cfg, Ym, qm, ufl, tol=tol, dense=dense)
    Y1 = Y + nu * cfg.dt * V[:, :3]
    q1 = qmul(qexp(nu * cfg.dt * V[:, 3:]), q)
    return Y1, q1, {"nu": nu, "calV": calV, "d": d, "V": V, **info}


def em_step(cfg: Config, Y, q, step, tol=1e-12, dense=None):
    """Euler-Maruyama (Appendix D): the full saddle problem at x^n with the
    same random slip, x^{n+1} = x^n + dt V^n.  No drift correction."""
    Y = np.asarray(Y, dtype=np.float64).reshape(-1, 3)
    q = np.asarray(q, dtype=np.float64).reshape(-1, 4)
    ufl = fluct_field(cfg, step)
    V, info = corrector_solve(cfg, Y, q, ufl, tol=tol, dense=dense)
    return Y + cfg.dt * V[:, :3], qmul(qexp(cfg.dt * V[:, 3:]), q), {"V": V, **info}


def mobility_divergence(cfg: Config, Y, q, h=1e-4):
    """kT-free drift of the overdamped dynamics: (d_x . N)_i = sum_j dN_ij/dx_j
    over the 6N generalised coordinates (Sec. 3: the term the drift
    correction captures, so that E[x^{n+1} - x^n] = dt (N F + kT d_x . N)
    + O(dt^2)).  Translations perturb Y_p; rotations perturb q_p <-
    exp(h e) q_p, the Lie-algebra coordinates reset to 0 at x^n.  Central
    differences of the dense body mobility (small systems only)."""
    b = cfg.susp.bodies
    Y = np.asarray(Y, dtype=np.float64).reshape(-1, 3)
    q = np.asarray(q, dtype=np.float64).reshape(-1, 4)

    def N_at(Yx, qx):
        return rigid.body_mobility(cfg.susp, Yx, rigid.blob_positions(b, Yx, qx))

    div = np.zeros(6 * b.N)
    for j in range(6 * b.N):
        p, c = divmod(j, 6)
        Yp, Ym, qp, qm = Y.copy(), Y.copy(), q.copy(), q.copy()
        if c < 3:
            Yp[p, c] += h
            Ym[p, c] -= h
        else:
            e = np.zeros((1, 3))
            e[0, c - 3] = h
            qp[p] = qmul(qexp(e), q[p:p + 1])[0]
            qm[p] = qmul(qexp(-e), q[p:p + 1])[0]
        div += (N_at(Yp, qp)[:, j] - N_at(Ym, qm)[:, j]) / (2.0 * h)
    return div
