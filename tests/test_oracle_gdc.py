"""Pins of oracle.gdc: the noiseless limit (gDC = Euler-Maruyama = forward
Euler, Sec. 3 and Appendix D), norm preservation of the quaternion update,
the forward-difference divergence against an analytic derivative, and the
pair-force model."""
import math

import numpy as np

import workloads as wl
from oracle import fcm, gdc, rigid
from oracle.quaternion import qexp, qmul

ETA = 1.0 / (6.0 * math.pi)


def _cfg(shapes, body_shape, kT=1.0, L=12.0, n=12, dt=0.01, seed=3, **fk):
    p = fcm.FcmParams(fcm.Grid([L] * 3, (n,) * 3), ETA, 1.0 / math.sqrt(math.pi), 3.0)
    s = rigid.Suspension(p, rigid.Bodies(shapes, body_shape), 1.0)
    return gdc.Config(s, kT, dt, seed, gdc.Forces(**fk))


def _state(cfg, seed=0):
    rng = np.random.default_rng(seed)
    N = cfg.susp.bodies.N
    q = rng.standard_normal((N, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    Y = np.array([[2.0, 3.0, 4.0], [7.5, 8.0, 6.5], [4.0, 9.0, 10.0]])[:N]
    return Y, q


def test_zero_temperature_is_forward_euler():
    cfg = _cfg([wl.boomerang(), wl.rod(3)], [0, 1], kT=0.0,
               const_force=np.array([0.0, 0.3, 1.0, 0.1, 0.0, -0.2]))
    Y, q = _state(cfg)
    Y1, q1, d = gdc.gdc_step(cfg, Y, q, step=0, dense=True)
    assert d["nu"] == 1.0 and np.all(d["calV"] == 0)
    Ye, qe, de = gdc.em_step(cfg, Y, q, step=0, dense=True)
    assert np.abs(Y1 - Ye).max() < 1e-15 and np.abs(q1 - qe).max() < 1e-15
    # forward Euler with V = N F
    r = rigid.blob_positions(cfg.susp.bodies, Y, q)
    N = rigid.body_mobility(cfg.susp, Y, r)
    F = gdc.body_forces(cfg, Y, r)
    V = (N @ F.ravel()).reshape(-1, 6)
    assert np.abs(Y1 - (Y + cfg.dt * V[:, :3])).max() < 1e-8 * cfg.dt
    assert np.abs(q1 - qmul(qexp(cfg.dt * V[:, 3:]), q)).max() < 1e-8 * cfg.dt


def test_step_preserves_quaternion_norm_and_is_deterministic():
    cfg = _cfg([wl.tetrahedron()], [0, 0])
    Y, q = _state(cfg, 1)
    Y1, q1, d = gdc.gdc_step(cfg, Y, q, step=4, dense=True)
    assert np.abs(np.linalg.norm(q1, axis=1) - 1).max() < 2e-15
    Y2, q2, _ = gdc.gdc_step(cfg, Y, q, step=4, dense=True)
    assert np.array_equal(Y1, Y2) and np.array_equal(q1, q2)
    Y3, _, _ = gdc.gdc_step(cfg, Y, q, step=5, dense=True)
    assert not np.array_equal(Y1, Y3)


def test_fd_divergence_matches_analytic_derivative():
    # translational part: d/dY_a calV_a = [(K^T K)^+ K^T dv/dY_a]_a with
    # dv_i/dY_a = dV sum_g u_g Delta_i(x_g) (x_g - r_i)_a / sigma^2 (exact
    # derivative of the Gaussian, no truncation crossing for this state)
    cfg = _cfg([wl.boomerang()], [0])
    Y, q = _state(cfg, 2)
    ufl = gdc.fluct_field(cfg, 0)
    b = cfg.susp.bodies
    p = cfg.susp.fcm
    r = rigid.blob_positions(b, Y, q)
    bi, gi, w = fcm.blob_stencils(r, p.grid, p.sigma, p.rc)
    gidx = np.stack(np.unravel_index(gi, p.grid.n), 1) * p.grid.dx
    dvec = gidx - (r[bi] - p.grid.L * np.floor(r[bi] / p.grid.L))
    dvec -= p.grid.L * np.round(dvec / p.grid.L)
    uflat = ufl.reshape(3, -1)[:, gi].T
    Lp = gdc.body_length(b.shapes[0], 1.0)
    K = rigid.body_K(r - Y[0])
    Pinv = np.linalg.pinv(K.T @ K)
    ana = 0.0
    for a in range(3):
        dv = np.zeros((b.M, 3))
        np.add.at(dv, bi, p.grid.dV * uflat * (w * dvec[:, a] / p.sigma ** 2)[:, None])
        ana += (Pinv @ K.T @ dv.ravel())[a]
    fd = 0.0
    calV = rigid.lsq_velocity(b, Y, r, gdc.averaged(cfg, r, ufl))
    for a in range(3):
        Yp = Y.copy()
        Yp[0, a] += 1e-6 * Lp
        rp = rigid.blob_positions(b, Yp, q)
        fd += (rigid.lsq_velocity(b, Yp, rp, gdc.averaged(cfg, rp, ufl))[0, a] - calV[0, a]) / (1e-6 * Lp)
    assert abs(fd - ana) < 1e-4 * abs(ana) + 1e-6
    # and the predictor's d_p includes exactly this translational sum
    cfg_rot_only = gdc.predictor(cfg, Y, q, ufl)[1]
    assert np.isfinite(cfg_rot_only).all()


def test_fd_first_order_in_delta():
    cfg = _cfg([wl.tetrahedron(), wl.rod(3)], [0, 1])
    Y, q = _state(cfg, 3)
    ufl = gdc.fluct_field(cfg, 1)
    # (larger deltas can move a grid point across the truncation sphere of
    # radius 3a, a jump of relative size ~1e-6/delta; below 1e-5 it is rare)
    ds = []
    for delta in [1e-5, 1e-6, 1e-7]:
        cfg.fd_delta = delta
        ds.append(gdc.predictor(cfg, Y, q, ufl)[1])
    e1 = np.abs(ds[0] - ds[2]).max()
    e2 = np.abs(ds[1] - ds[2]).max()
    assert e2 < 0.2 * e1                       # error shrinks ~10x per decade of delta


def test_steric_pair_forces():
    k, b = 40.0 / 2.2, 2.2
    cfg = _cfg([np.zeros((1, 3)), wl.rod(2)], [0, 0, 1], steric_k=k, steric_cutoff=b)
    Y = np.array([[1.0, 1.0, 1.0], [1.0, 1.0, 3.0], [6.0, 6.0, 6.0]])   # blobs 0-1 at distance 2
    q = np.tile([1.0, 0, 0, 0], (3, 1))
    r = rigid.blob_positions(cfg.susp.bodies, Y, q)
    f = gdc.steric_blob_forces(cfg, r)
    assert np.allclose(f[0], [0, 0, -k * (b - 2.0)]) and np.allclose(f[1], [0, 0, k * (b - 2.0)])
    assert np.abs(f[2:]).max() == 0.0           # rod blobs at distance 2 but same body
    assert np.abs(f.sum(0)).max() < 1e-15
    # minimum image across the periodic boundary
    Y2 = np.array([[0.5, 5.0, 5.0], [11.5 - 0.1, 5.0, 5.0], [6.0, 6.0, 0.0]])
    r2 = rigid.blob_positions(cfg.susp.bodies, Y2, q)
    f2 = gdc.steric_blob_forces(cfg, r2)
    assert f2[0, 0] > 0 and abs(f2[0, 0] - k * (b - 1.1)) < 1e-12


def test_background_shear_profile():
    cfg = _cfg([wl.rod(2)], [0], shear_rate=0.1)
    Y = np.array([[3.0, 12.0 + 9.0, 4.0]])           # unwrapped centre
    q = np.array([[math.cos(0.4), math.sin(0.4), 0, 0]])
    r = rigid.blob_positions(cfg.susp.bodies, Y, q)
    u = gdc.background_flow(cfg, Y, r)
    assert np.allclose(u[:, 0], 0.1 * (9.0 + (r[:, 1] - Y[0, 1]) - 6.0))
    assert np.all(u[:, 1:] == 0)


def test_rfd_mean_is_the_fd_divergence():
    # eq. rfd_div: with W~ ~ N(0, I) the random difference quotient of each
    # body has that body's divergence as its mean.  W~ is keyed by the step
    # counter while the field is passed in, so averaging over counters with
    # the field held fixed samples W~ alone; the mean must match the
    # forward-difference divergence (pinned above) within its standard error.
    cfg = _cfg([wl.boomerang(), wl.rod(3)], [0, 1])
    Y, q = _state(cfg, 4)
    ufl = gdc.fluct_field(cfg, 0)
    calV, d_fd = gdc.predictor(cfg, Y, q, ufl)
    K = 3000
    smp = np.array([gdc.rfd_divergence(cfg, Y, q, ufl, calV, s) for s in range(K)])
    mean = smp.mean(0)
    se = smp.std(0, ddof=1) / math.sqrt(K)
    assert np.all(np.abs(mean - d_fd) < 5.0 * se), (mean, d_fd, se)
    # the test resolves the divergence: it is many standard errors from 0
    assert np.all(np.abs(d_fd) > 5.0 * se), (d_fd, se)


def _pair_cfg(shape, L=16.0, n=16):
    return _cfg([shape], [0, 0], L=L, n=n)


def test_mobility_divergence_pins():
    # (a) one body in a periodic box on a fine grid (sigma/dx = 2.3, aliasing
    # ~1e-40): N does not depend on the body's position, so the derivatives
    # along translations vanish and the divergence is its rotational part
    # alone (on the dx = a grids of the workloads the sampled envelope makes
    # N vary with the sub-grid position at the 1e-3 level, so there they do
    # not vanish); (b) second-order convergence in h; (c) swapping two
    # bodies of the same shape swaps the blocks of the divergence.
    one = _cfg([wl.tetrahedron()], [0], L=8.0, n=32)
    Y1 = np.array([[4.13, 3.76, 4.21]])
    q1 = np.array([[0.8, 0.2, -0.4, 0.4]]) / np.linalg.norm([0.8, 0.2, -0.4, 0.4])
    d1 = gdc.mobility_divergence(one, Y1, q1)
    N1 = rigid.body_mobility(one.susp, Y1, rigid.blob_positions(one.susp.bodies, Y1, q1))
    rot = np.zeros(6)
    for j in range(3, 6):
        e = np.zeros((1, 3))
        e[0, j - 3] = 1e-4
        Np = rigid.body_mobility(one.susp, Y1, rigid.blob_positions(one.susp.bodies, Y1, qmul(qexp(e), q1)))
        Nm = rigid.body_mobility(one.susp, Y1, rigid.blob_positions(one.susp.bodies, Y1, qmul(qexp(-e), q1)))
        rot += (Np[:, j] - Nm[:, j]) / 2e-4
    # (cut-off sphere crossings and round-off leave ~1e-6; the rotational
    # terms are ~1e-2)
    assert np.abs(d1 - rot).max() < 1e-5 * np.abs(N1).max()
    assert np.abs(rot).max() > 1e-3 * np.abs(N1).max()
    cfg = _pair_cfg(wl.rod(3))
    Y = np.array([[6.5, 8.0, 8.3], [9.5, 8.4, 8.0]])
    q = np.array([[0.9, 0.3, 0.2, 0.1], [0.7, -0.2, 0.5, 0.3]])
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    d_a = gdc.mobility_divergence(cfg, Y, q, h=1e-3)
    d_b = gdc.mobility_divergence(cfg, Y, q, h=1e-4)
    assert np.abs(d_a - d_b).max() < 1e-4 * np.abs(d_b).max()
    assert np.abs(d_b).max() > 1e-2            # the pair has a drift to see
    d_s = gdc.mobility_divergence(cfg, Y[::-1].copy(), q[::-1].copy(), h=1e-4)
    assert np.abs(d_s - np.concatenate([d_b[6:], d_b[:6]])).max() < 1e-9 * np.abs(d_b).max()


def test_sine_average_closed_form():
    # J[sin(k y)](r) is the Gaussian average of sin(k y): exp(-k^2 sigma^2 / 2)
    # sin(k r_y) in the continuum; on a grid with sigma/dx = 1.13 the
    # trapezoidal average matches it to the cut-off and aliasing errors (<1e-5)
    cfg = _cfg([np.zeros((1, 3))], [0, 0, 0], L=16.0, n=32)
    r = np.array([[1.3, 2.2, 3.9], [7.4, 11.05, 5.1], [14.9, 15.7, 0.4]])
    k = 2.0 * math.pi / 16.0
    s = gdc.sine_average(cfg, r)
    ref = math.exp(-0.5 * (k / math.sqrt(math.pi)) ** 2) * np.sin(k * r[:, 1])
    assert np.abs(s - ref).max() < 1e-5


def test_sine_forcing_force_free_blobs_follow_the_flow():
    # single-blob bodies without forces carry no constraint force (K^T lambda
    # = 0 gives lambda = 0): they move with the averaged forcing flow, and the
    # measured amplitude is the unhindered f0 / (eta k^2), so eta_eff = eta
    cfg = _cfg([np.zeros((1, 3))], [0, 0, 0], kT=0.0, L=12.0, n=12, sine_force=0.7)
    Y = np.array([[1.3, 2.2, 3.9], [7.4, 8.05, 5.1], [10.9, 5.7, 0.4]])
    q = np.tile([1.0, 0.0, 0.0, 0.0], (3, 1))
    Y1, _, info = gdc.gdc_step(cfg, Y, q, step=0, dense=True)
    k = 2.0 * math.pi / 12.0
    scale = 0.7 / (ETA * k * k)
    r = rigid.blob_positions(cfg.susp.bodies, Y, q)
    u = scale * gdc.sine_average(cfg, r)
    assert np.abs((Y1 - Y)[:, 0] - cfg.dt * u).max() < 1e-12 * abs(scale) * cfg.dt
    assert np.abs((Y1 - Y)[:, 1:]).max() < 1e-15
    assert abs(info["sine_vx"] - scale) < 1e-12 * scale


def test_sine_forcing_rigid_bodies_raise_the_viscosity():
    # rigid bodies resist the imposed flow: the response to the same force
    # density is weaker, so eta_eff = f0 / (k^2 v_x) > eta, and the amplitude
    # is linear in f0
    cfg = _cfg([wl.rod(4), wl.boomerang()], [0, 1, 0], kT=0.0, L=12.0, n=12, sine_force=1.0)
    Y = np.array([[2.0, 3.0, 4.0], [7.5, 8.0, 6.5], [4.0, 9.0, 10.0]])
    q = np.array([[0.9, 0.3, 0.2, 0.1], [0.7, -0.2, 0.5, 0.3], [0.5, 0.5, 0.5, 0.5]])
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    _, _, info = gdc.gdc_step(cfg, Y, q, step=0, dense=True)
    k = 2.0 * math.pi / 12.0
    eta_eff = 1.0 / (k * k * info["sine_vx"])
    assert eta_eff > ETA * (1.0 + 1e-3), eta_eff / ETA
    cfg.forces.sine_force = 2.0
    _, _, info2 = gdc.gdc_step(cfg, Y, q, step=0, dense=True)
    assert abs(info2["sine_vx"] - 2.0 * info["sine_vx"]) < 1e-10 * abs(info["sine_vx"])
