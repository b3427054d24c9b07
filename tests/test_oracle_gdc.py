"""Pins of oracle.gdc: the noiseless limit (gDC = Euler-Maruyama = forward
Euler, Sec. 3 and Appendix D), norm preservation of the quaternion update,
the forward-difference divergence against an analytic derivative, and the
pair-force model."""
import math

import numpy as np

import workloads as wl
from oracle import fcm, gdc, rigid
from oracle.quaternion import cross_matrix, qexp, qmul, rotation_matrix

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


# ---------------------------------------------------------------- exact derivatives
# The divergence of eq. FD perturbs body p by a translation Y_p += theta e_a
# or a rotation q_p <- exp(theta e_a) q_p (the Lie-algebra coordinate of the
# midpoint and update moves, reset to 0 at x^n).  Below, the exact theta-
# derivatives at theta = 0, written from the chain rule on their own:
#   blob motion  dr_i = e_a (translation) or e_a x (r_i - Y_p) (rotation);
#   averaging    dv_i = dV sum_g u_g Delta_i(x_g) (x_g - r_i) . dr_i / sigma^2;
#   rigid map    dK rows [0, -[d(r_i - Y_p) x]];
#   pseudo-inverse of A = K^T K at constant rank (Golub and Pereyra 1973):
#     dA^+ = -A^+ dA A^+ + A^+ A^+ dA (I - A A^+) + (I - A A^+) dA A^+ A^+.
# They pin the oracle's finite differences, including the choice of axis
# (lab-frame e_a, left multiplication) that nothing else fixes.


def _pinv_derivative(A, dA):
    Ap = np.linalg.pinv(A, rcond=rigid.PINV_RCOND)
    PN = np.eye(A.shape[0]) - A @ Ap
    return -Ap @ dA @ Ap + Ap @ Ap @ dA @ PN + PN @ dA @ Ap @ Ap


def _stencil_offsets(p, r):
    """(blob, grid point, weight, x_g - r_i minimum image) over all stencils."""
    bi, gi, w = fcm.blob_stencils(r, p.grid, p.sigma, p.rc)
    xg = np.stack(np.unravel_index(gi, p.grid.n), 1) * p.grid.dx
    d = xg - (r[bi] - p.grid.L * np.floor(r[bi] / p.grid.L))
    return bi, gi, w, d - p.grid.L * np.round(d / p.grid.L)


def _blob_motion(rel, kind, a, axis_frame=None):
    """dr_i of the body's blobs (rel_i = r_i - Y_p) for a unit translation
    or rotation along e_a; axis_frame rotates the axis (R(q) e_a is the
    body-frame reading, used only to show that the pins tell them apart)."""
    e = np.zeros(3)
    e[a] = 1.0
    if kind == "t":
        return np.tile(e, (rel.shape[0], 1))
    if axis_frame is not None:
        e = axis_frame @ e
    return np.cross(e, rel)


def _dcalV(cfg, Y, q, ufl, p, kind, a, axis_frame=None):
    """Exact d calV_p / d theta for body p's perturbation (kind, a)."""
    b, P = cfg.susp.bodies, cfg.susp.fcm
    r = rigid.blob_positions(b, Y, q)
    o, c = b.offsets[p], b.counts[p]
    rel = r[o:o + c] - Y[p]
    dr_b = _blob_motion(rel, kind, a, axis_frame)
    drel = np.zeros_like(rel) if kind == "t" else dr_b
    bi, gi, w, d = _stencil_offsets(P, r)
    on = (bi >= o) & (bi < o + c)
    uf = ufl.reshape(3, -1)[:, gi[on]].T
    coef = P.grid.dV * w[on] * (d[on] * dr_b[bi[on] - o]).sum(1) / P.sigma ** 2
    dv = np.zeros((c, 3))
    np.add.at(dv, bi[on] - o, uf * coef[:, None])
    v = gdc.averaged(cfg, r, ufl)[o:o + c].reshape(-1)
    K = rigid.body_K(rel)
    dK = np.zeros_like(K)
    for i in range(c):
        dK[3 * i:3 * i + 3, 3:] = -cross_matrix(drel[i])
    A = K.T @ K
    Ap = np.linalg.pinv(A, rcond=rigid.PINV_RCOND)
    return _pinv_derivative(A, dK.T @ K + K.T @ dK) @ (K.T @ v) + Ap @ (dK.T @ v + K.T @ dv.reshape(-1))


def _cutoff_crossings(P, r0, r1):
    """Grid points whose distance to a blob crosses the cut-off radius between
    positions r0 and r1 (each crossing is a jump of the truncated envelope)."""
    bi, gi, _ = fcm.blob_stencils(r0, P.grid, P.sigma, P.rc + 0.05)
    xg = np.stack(np.unravel_index(gi, P.grid.n), 1) * P.grid.dx

    def dist(r):
        d = xg - (r[bi] - P.grid.L * np.floor(r[bi] / P.grid.L))
        d -= P.grid.L * np.round(d / P.grid.L)
        return np.sqrt((d * d).sum(1))
    return int(np.count_nonzero((dist(r0) <= P.rc) != (dist(r1) <= P.rc)))


def test_fd_divergence_matches_exact_derivative():
    # eq. FD term by term: a boomerang and a tetrahedron (full rank) and a
    # straight rod (K^T K of rank 5: the pseudo-inverse derivative), at
    # generic positions (a blob on a grid point has lattice points exactly
    # at the cut-off, where the quotient grows like 1/delta)
    cfg = _cfg([wl.boomerang(), wl.tetrahedron(), wl.rod(3)], [0, 1, 2], L=16.0, n=16)
    rng = np.random.default_rng(7)
    Y = np.array([[3.13, 4.27, 5.31], [10.52, 9.07, 7.71], [5.09, 12.03, 11.41]])
    q = rng.standard_normal((3, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    ufl = gdc.fluct_field(cfg, 0)
    b, P = cfg.susp.bodies, cfg.susp.fcm
    r0 = rigid.blob_positions(b, Y, q)
    delta = cfg.fd_delta
    for p in range(b.N):
        Lp = gdc.body_length(b.shapes[b.body_shape[p]], 1.0)
        for a in range(3):
            Yp = Y.copy()
            Yp[p, a] += delta * Lp
            e = np.zeros((b.N, 3))
            e[p, a] = delta
            assert _cutoff_crossings(P, r0, rigid.blob_positions(b, Yp, q)) == 0
            assert _cutoff_crossings(P, r0, rigid.blob_positions(b, Y, qmul(qexp(e), q))) == 0
    _, d = gdc.predictor(cfg, Y, q, ufl)
    for p in range(b.N):
        trans = sum(_dcalV(cfg, Y, q, ufl, p, "t", a)[a] for a in range(3))
        rot = sum(_dcalV(cfg, Y, q, ufl, p, "r", a)[3 + a] for a in range(3))
        # the forward difference is first order in delta = 1e-6
        assert abs(d[p] - (trans + rot)) < 1e-4 * abs(trans + rot), (p, d[p], trans, rot)
        # both halves matter, and the body-frame axis (q exp(delta e)) would
        # be caught: its rotational sum differs by far more than the bound
        assert abs(rot) > 0.2 * abs(trans + rot) or abs(trans) > 0.2 * abs(trans + rot)
        R = rotation_matrix(q[p])
        rot_body = sum(_dcalV(cfg, Y, q, ufl, p, "r", a, axis_frame=R)[3 + a] for a in range(3))
        assert abs(rot_body - rot) > 100 * 1e-4 * abs(trans + rot), (p, rot, rot_body)


def test_mobility_divergence_matches_exact_derivative():
    # d_x . N by the chain rule on N = (K^T M^-1 K)^-1 with M = J L^-1 S:
    # dM = dJ L^-1 S + (dJ L^-1 S)^T (J = dV S^T, L^-1 symmetric),
    # dN = -N (dK^T M^-1 K + K^T M^-1 dK - K^T M^-1 dM M^-1 K) N; column
    # (p, a) of dN under body p's perturbation a, summed over all (p, a).
    cfg = _cfg([wl.tetrahedron(), wl.boomerang()], [0, 1], L=16.0, n=16)
    b, P = cfg.susp.bodies, cfg.susp.fcm
    g = P.grid
    Y = np.array([[5.13, 7.27, 6.31], [9.52, 8.07, 9.71]])
    q = np.array([[0.9, 0.3, 0.2, 0.1], [0.7, -0.2, 0.5, 0.3]])
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    r = rigid.blob_positions(b, Y, q)
    M = b.M
    W = fcm.weight_matrix(r, g, P.sigma, P.rc)
    U = np.empty((3 * M, 3, g.G))
    for j in range(3 * M):
        lam = np.zeros(3 * M)
        lam[j] = 1.0
        U[j] = fcm.stokes_solve(fcm.spread(W, lam.reshape(M, 3), g), g, P.eta).reshape(3, -1)
    Mm = g.dV * np.einsum("ig,jcg->icj", W.toarray(), U).reshape(3 * M, 3 * M)
    bi, gi, w, d = _stencil_offsets(P, r)
    K = np.zeros((3 * M, 6 * b.N))
    for p, sl, rel in rigid.per_body(b, Y, r):
        K[3 * sl.start:3 * sl.stop, 6 * p:6 * p + 6] = rigid.body_K(rel)
    Minv = np.linalg.inv(Mm)
    N = np.linalg.inv(K.T @ Minv @ K)

    def divergence(axis_frames=None):
        div = np.zeros(6 * b.N)
        for p, sl, rel in rigid.per_body(b, Y, r):
            for a in range(6):
                fr = None if axis_frames is None else axis_frames[p]
                drb = _blob_motion(rel, "t" if a < 3 else "r", a % 3, fr)
                dr = np.zeros((M, 3))
                dr[sl] = drb
                dJ = np.zeros((M, g.G))
                np.add.at(dJ, (bi, gi), g.dV * w * (d * dr[bi]).sum(1) / P.sigma ** 2)
                D = np.einsum("ig,jcg->icj", dJ, U).reshape(3 * M, 3 * M)
                dK = np.zeros_like(K)
                if a >= 3:
                    for k, i in enumerate(range(sl.start, sl.stop)):
                        dK[3 * i:3 * i + 3, 6 * p + 3:6 * p + 6] = -cross_matrix(drb[k])
                dB = dK.T @ Minv @ K + K.T @ Minv @ dK - K.T @ Minv @ (D + D.T) @ Minv @ K
                div += (-N @ dB @ N)[:, 6 * p + a]
        return div

    exact = divergence()
    fd = gdc.mobility_divergence(cfg, Y, q, h=1e-4)
    # central differences: O(h^2) plus cut-off crossings (none at this state)
    assert np.abs(fd - exact).max() < 1e-5 * np.abs(exact).max(), np.abs(fd - exact).max()
    # rotational columns carry a resolvable share, and the body-frame axis
    # reading gives a different divergence
    rot_idx = np.array([6 * p + a for p in range(b.N) for a in range(3, 6)])
    assert np.abs(exact[rot_idx]).max() > 0.1 * np.abs(exact).max()
    body = divergence(axis_frames=rotation_matrix(q))
    assert np.abs(body - exact).max() > 100 * 1e-5 * np.abs(exact).max()


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
