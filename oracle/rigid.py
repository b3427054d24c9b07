"""Rigid multiblob bodies and the constrained mobility problem (paper Sec. 2.2).

Body p has blobs B_p at r_i = Y_p + R(q_p) b_i (Sec. 2).  The rigid-body map
K (eq. rigid_body_cond, K block) sends V_p = (U_p, Omega_p) to blob
velocities U_p + Omega_p x (r_i - Y_p); K^T sums blob forces to (F_p, T_p)
(eq. force_torque_balance_compact).

Degenerate bodies.  For a body whose blobs are collinear (straight rods) or a
single blob, K_p has a null space (spin about the axis moves no blob), so
K^T K and the saddle system are singular.  The reading taken here: those
degrees of freedom are frozen.  The least-squares velocity uses the
Moore-Penrose pseudo-inverse of K^T K (relative cutoff 1e-10); the saddle
system gets -Pi_p in its (V, V) block, Pi_p the orthogonal projector onto
null(K_p), and the applied force is projected onto range(K_p^T).  The
solution then satisfies Pi_p V_p = 0 and is unchanged for full-rank bodies.

Oracle code: test infrastructure only.
"""

from dataclasses import dataclass, field

import numpy as np

from . import fcm
from .quaternion import rotation_matrix, cross_matrix

PINV_RCOND = 1e-10


@dataclass
class Bodies:
    """A suspension's bodies: shapes[s] is an (n_b, 3) array of body-frame
    blob offsets; body_shape[p] names the shape of body p.  Blobs are
    numbered body by body in body order."""
    shapes: list
    body_shape: np.ndarray
    offsets: np.ndarray = field(init=False)   # first blob of each body
    counts: np.ndarray = field(init=False)

    def __post_init__(self):
        self.shapes = [np.asarray(s, dtype=np.float64).reshape(-1, 3) for s in self.shapes]
        self.body_shape = np.asarray(self.body_shape, dtype=np.int64)
        self.counts = np.array([self.shapes[s].shape[0] for s in self.body_shape], dtype=np.int64)
        self.offsets = np.concatenate([[0], np.cumsum(self.counts)[:-1]]).astype(np.int64)

    @property
    def N(self):
        return int(self.body_shape.size)

    @property
    def M(self):
        return int(self.counts.sum())

    def body_of_blob(self):
        return np.repeat(np.arange(self.N), self.counts)


def blob_positions(bodies: Bodies, Y, q):
    """r_i = Y_p + R(q_p) b_i (Sec. 2), unwrapped.  -> (M, 3)."""
    Y = np.asarray(Y, dtype=np.float64).reshape(-1, 3)
    R = rotation_matrix(np.asarray(q, dtype=np.float64).reshape(-1, 4))
    out = np.empty((bodies.M, 3))
    for p in range(bodies.N):
        b = bodies.shapes[bodies.body_shape[p]]
        o = bodies.offsets[p]
        out[o:o + b.shape[0]] = Y[p] + b @ R[p].T
    return out


def body_K(rel):
    """K_p (3 n_b x 6) from blob offsets rel_i = r_i - Y_p: block row i is
    [I, [x rel_i]] with [x v] = -[v x] (eq. rigid_body_cond)."""
    n = rel.shape[0]
    K = np.zeros((3 * n, 6))
    for i in range(n):
        K[3 * i:3 * i + 3, :3] = np.eye(3)
        K[3 * i:3 * i + 3, 3:] = -cross_matrix(rel[i])
    return K


def KtK_closed_form(rel):
    """The 6x6 block of K^T K printed in Sec. 5 (cost of step 2):
    [[n_b I, sum [x rel]], [sum [rel x], -sum [rel x]^2]]."""
    n = rel.shape[0]
    A = np.zeros((6, 6))
    A[:3, :3] = n * np.eye(3)
    S = np.zeros((3, 3))
    Q = np.zeros((3, 3))
    for i in range(n):
        C = cross_matrix(rel[i])
        S += C
        Q += C @ C
    A[:3, 3:] = -S
    A[3:, :3] = S
    A[3:, 3:] = -Q
    return A


def per_body(bodies: Bodies, Y, r):
    """Yields (p, blob slice, rel = r_i - Y_p) for every body."""
    Y = np.asarray(Y, dtype=np.float64).reshape(-1, 3)
    for p in range(bodies.N):
        o, c = bodies.offsets[p], bodies.counts[p]
        yield p, slice(o, o + c), r[o:o + c] - Y[p]


def K_apply(bodies, Y, r, V):
    """Blob velocities K V.  V: (N, 6) -> (M, 3)."""
    out = np.empty((bodies.M, 3))
    for p, sl, rel in per_body(bodies, Y, r):
        out[sl] = (body_K(rel) @ V[p]).reshape(-1, 3)
    return out


def KT_apply(bodies, Y, r, lam):
    """(F_p, T_p) = K^T lambda.  lam: (M, 3) -> (N, 6)."""
    out = np.empty((bodies.N, 6))
    for p, sl, rel in per_body(bodies, Y, r):
        out[p] = body_K(rel).T @ lam[sl].reshape(-1)
    return out


def null_projector(rel):
    """Pi_p: orthogonal projector onto null(K_p), from the pseudo-inverse:
    Pi = I - (K^T K)^+ (K^T K)."""
    A = body_K(rel).T @ body_K(rel)
    return np.eye(6) - np.linalg.pinv(A, rcond=PINV_RCOND) @ A


def lsq_velocity(bodies, Y, r, v):
    """Step 2 of the gDC (eq. sol_unconst): calV_p = (K_p^T K_p)^+ K_p^T v_p,
    the least-squares rigid-body velocity.  v: (M, 3) -> (N, 6)."""
    out = np.empty((bodies.N, 6))
    for p, sl, rel in per_body(bodies, Y, r):
        K = body_K(rel)
        out[p] = np.linalg.pinv(K.T @ K, rcond=PINV_RCOND) @ (K.T @ v[sl].reshape(-1))
    return out


# --------------------------------------------------------------- RPY blocks

def rpy_tensor(d, a, eta):
    """Unbounded Rotne-Prager-Yamakawa tensor for equal radii a at separation
    d (Sec. 4.1; standard closed form): 1/(6 pi eta a) I at d = 0,
    (1/(8 pi eta r))[(1 + 2a^2/3r^2) I + (1 - 2a^2/r^2) rr] for r >= 2a,
    (1/(6 pi eta a))[(1 - 9r/32a) I + (3r/32a) rr] for r < 2a."""
    r = np.linalg.norm(d)
    if r == 0.0:
        return np.eye(3) / (6.0 * np.pi * eta * a)
    e = np.outer(d, d) / (r * r)
    if r >= 2.0 * a:
        return ((1.0 + 2.0 * a * a / (3.0 * r * r)) * np.eye(3)
                + (1.0 - 2.0 * a * a / (r * r)) * e) / (8.0 * np.pi * eta * r)
    return ((1.0 - 9.0 * r / (32.0 * a)) * np.eye(3)
            + (3.0 * r / (32.0 * a)) * e) / (6.0 * np.pi * eta * a)


def body_saddle_block(rel, a, eta):
    """Block-diagonal preconditioner block of Sec. 2.2 (M with inter-body
    entries removed): [[M_pp, -K_p], [-K_p^T, -Pi_p]], with M_pp taken from
    the unbounded RPY tensor (FCM's own self block has no closed form; RPY
    matches its diagonal at sigma = a/sqrt(pi))."""
    n = rel.shape[0]
    Mpp = np.zeros((3 * n, 3 * n))
    for i in range(n):
        for j in range(n):
            Mpp[3 * i:3 * i + 3, 3 * j:3 * j + 3] = rpy_tensor(rel[i] - rel[j], a, eta)
    K = body_K(rel)
    A = np.zeros((3 * n + 6, 3 * n + 6))
    A[:3 * n, :3 * n] = Mpp
    A[:3 * n, 3 * n:] = -K
    A[3 * n:, :3 * n] = -K.T
    A[3 * n:, 3 * n:] = -null_projector(rel)
    return A


# ------------------------------------------------------------ saddle problem

@dataclass
class Suspension:
    fcm: fcm.FcmParams
    bodies: Bodies
    a: float


def unknowns(bodies):
    return 3 * bodies.M + 6 * bodies.N


def saddle_apply(s: Suspension, Y, r, x, Ws=None):
    """[[M, -K], [-K^T, -Pi]] [lambda; V] (eq. lin_sys_RMB with the frozen
    null space).  x: flat (3M + 6N,).  Ws: fcm.weights(r) if precomputed."""
    b = s.bodies
    lam = x[:3 * b.M].reshape(-1, 3)
    V = x[3 * b.M:].reshape(-1, 6)
    if Ws is None:
        Ws = fcm.weights(r, s.fcm)
    f = fcm.spread_forces(Ws, lam, s.fcm)
    Mlam = fcm.interp(Ws[0], fcm.stokes_solve(f, s.fcm.grid, s.fcm.eta), s.fcm.grid)
    top = Mlam - K_apply(b, Y, r, V)
    bot = -KT_apply(b, Y, r, lam)
    for p, sl, rel in per_body(b, Y, r):
        bot[p] -= null_projector(rel) @ V[p]
    return np.concatenate([top.reshape(-1), bot.reshape(-1)])


def saddle_rhs(s: Suspension, Y, r, v_slip, F):
    """Right-hand side [-v_slip; -(I - Pi) F] (eq. lin_sys_RMB / step5)."""
    b = s.bodies
    Fp = np.array(F, dtype=np.float64).reshape(-1, 6).copy()
    for p, sl, rel in per_body(b, Y, r):
        Fp[p] = Fp[p] - null_projector(rel) @ Fp[p]
    return np.concatenate([-np.asarray(v_slip).reshape(-1), -Fp.reshape(-1)])


def block_preconditioner(s: Suspension, Y, r):
    """Returns a function applying P^-1 (Sec. 2.2): per-body dense inverses of
    body_saddle_block, on the (lambda_p, V_p) pieces of a vector."""
    b = s.bodies
    invs = []
    for p, sl, rel in per_body(b, Y, r):
        invs.append(np.linalg.inv(body_saddle_block(rel, s.a, s.fcm.eta)))

    def apply(x):
        lam = x[:3 * b.M].reshape(-1, 3)
        V = x[3 * b.M:].reshape(-1, 6)
        ol = np.empty_like(lam)
        oV = np.empty_like(V)
        for p in range(b.N):
            o, c = b.offsets[p], b.counts[p]
            y = invs[p] @ np.concatenate([lam[o:o + c].reshape(-1), V[p]])
            ol[o:o + c] = y[:3 * c].reshape(-1, 3)
            oV[p] = y[3 * c:]
        return np.concatenate([ol.reshape(-1), oV.reshape(-1)])
    return apply


def gmres(apply_A, rhs, apply_Pinv=None, tol=1e-12, restart=100, maxiter=2000):
    """Right-preconditioned restarted GMRES (Saad & Schultz 1986) with
    modified Gram-Schmidt and Givens rotations, zero initial guess; stops when
    the true residual |b - A x| <= tol |b|.  Returns (x, iterations, relres)."""
    if apply_Pinv is None:
        def apply_Pinv(v):
            return v
    b = np.asarray(rhs, dtype=np.float64)
    nb = np.linalg.norm(b)
    x = np.zeros_like(b)
    if nb == 0.0:
        return x, 0, 0.0
    its = 0
    while True:
        r = b - apply_A(apply_Pinv(x)) if its else b.copy()
        beta = np.linalg.norm(r)
        if beta <= tol * nb or its >= maxiter:
            return apply_Pinv(x), its, beta / nb
        m = restart
        V = np.zeros((m + 1, b.size))
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        V[0] = r / beta
        k_done = 0
        for k in range(m):
            w = apply_A(apply_Pinv(V[k]))
            for j in range(k + 1):
                H[j, k] = V[j] @ w
                w = w - H[j, k] * V[j]
            H[k + 1, k] = np.linalg.norm(w)
            if H[k + 1, k] > 0:
                V[k + 1] = w / H[k + 1, k]
            for j in range(k):
                t = cs[j] * H[j, k] + sn[j] * H[j + 1, k]
                H[j + 1, k] = -sn[j] * H[j, k] + cs[j] * H[j + 1, k]
                H[j, k] = t
            den = np.hypot(H[k, k], H[k + 1, k])
            cs[k], sn[k] = H[k, k] / den, H[k + 1, k] / den
            H[k, k] = den
            H[k + 1, k] = 0.0
            g[k + 1] = -sn[k] * g[k]
            g[k] = cs[k] * g[k]
            its += 1
            k_done = k + 1
            if abs(g[k + 1]) <= 0.5 * tol * nb or its >= maxiter:
                break
        yk = np.linalg.solve(np.triu(H[:k_done, :k_done]), g[:k_done])
        x = x + V[:k_done].T @ yk


def solve_saddle(s: Suspension, Y, r, v_slip, F, tol=1e-12, dense=None):
    """Solve [[M, -K], [-K^T, -Pi]] [lambda; V] = [-v_slip; -(I-Pi)F]
    (eq. lin_sys_RMB, eq. step5).  dense=True assembles the matrix (small
    systems); otherwise GMRES with the block preconditioner.
    Returns (lambda (M,3), V (N,6), info)."""
    b = s.bodies
    rhs = saddle_rhs(s, Y, r, v_slip, F)
    n = unknowns(b)
    if dense is None:
        dense = n <= 1500
    Ws = fcm.weights(r, s.fcm)

    def A(x):
        return saddle_apply(s, Y, r, x, Ws)
    if dense:
        Amat = np.empty((n, n))
        for j in range(n):
            e = np.zeros(n)
            e[j] = 1.0
            Amat[:, j] = A(e)
        x = np.linalg.solve(Amat, rhs)
        info = {"iterations": 0, "relres": float(np.linalg.norm(Amat @ x - rhs) / max(np.linalg.norm(rhs), 1e-300))}
    else:
        P = block_preconditioner(s, Y, r)
        x, its, rr = gmres(A, rhs, P, tol=tol)
        info = {"iterations": its, "relres": rr}
    return x[:3 * b.M].reshape(-1, 3), x[3 * b.M:].reshape(-1, 6), info


def body_mobility(s: Suspension, Y, r):
    """N = (K^T M^-1 K)^+ (eq. body_mob), dense, from M assembled directly
    (small systems only).  The pseudo-inverse freezes null(K) as above."""
    Mm = fcm.dense_mobility(r, s.fcm)
    b = s.bodies
    K = np.zeros((3 * b.M, 6 * b.N))
    for p, sl, rel in per_body(b, Y, r):
        K[3 * sl.start:3 * sl.stop, 6 * p:6 * p + 6] = body_K(rel)
    return np.linalg.pinv(K.T @ np.linalg.solve(Mm, K), rcond=1e-9)
