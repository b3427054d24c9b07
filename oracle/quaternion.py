"""Unit quaternions and the Lie-algebra update (paper Sec. 2 and Appendix A).

Convention: scalar-first q = (q0, q1, q2, q3) with the Hamilton product of
Appendix A.  All functions accept a leading batch axis.  Oracle code: test
infrastructure only.
"""

import numpy as np


def rotation_matrix(q):
    """R(q) of eq. (quaternion_rotation_matrix), Sec. 2: a body-frame vector b
    appears in the lab frame as R(q) b.  q: (..., 4) -> (..., 3, 3)."""
    q = np.asarray(q, dtype=np.float64)
    q0, q1, q2, q3 = q[..., 0], q[..., 1], q[..., 2], q[..., 3]
    R = np.empty(q.shape[:-1] + (3, 3))
    R[..., 0, 0] = 1.0 - 2.0 * q2 * q2 - 2.0 * q3 * q3
    R[..., 0, 1] = 2.0 * (q1 * q2 - q3 * q0)
    R[..., 0, 2] = 2.0 * (q1 * q3 + q2 * q0)
    R[..., 1, 0] = 2.0 * (q1 * q2 + q3 * q0)
    R[..., 1, 1] = 1.0 - 2.0 * q1 * q1 - 2.0 * q3 * q3
    R[..., 1, 2] = 2.0 * (q3 * q2 - q1 * q0)
    R[..., 2, 0] = 2.0 * (q1 * q3 - q2 * q0)
    R[..., 2, 1] = 2.0 * (q3 * q2 + q1 * q0)
    R[..., 2, 2] = 1.0 - 2.0 * q2 * q2 - 2.0 * q1 * q1
    return R


def qmul(p, q):
    """Hamilton product p . q (Appendix A): scalar p0 q0 - p.q, vector
    p0 q + q0 p + p x q.  Rotating by p.q means rotating by q first."""
    p = np.asarray(p, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    p0, pv = p[..., :1], p[..., 1:]
    q0, qv = q[..., :1], q[..., 1:]
    s = p0 * q0 - np.sum(pv * qv, axis=-1, keepdims=True)
    v = p0 * qv + q0 * pv + np.cross(pv, qv)
    return np.concatenate([s, v], axis=-1)


def qinv(q):
    """Inverse of a unit quaternion, (q0, -q) (Appendix A)."""
    q = np.asarray(q, dtype=np.float64)
    return np.concatenate([q[..., :1], -q[..., 1:]], axis=-1)


def rotate_by_product(q, x):
    """Image of x under q via (0, x') = q . (0, x) . q^-1 (Appendix A); an
    independent route to R(q) x used to pin rotation_matrix."""
    x = np.asarray(x, dtype=np.float64)
    x4 = np.concatenate([np.zeros(x.shape[:-1] + (1,)), x], axis=-1)
    return qmul(qmul(q, x4), qinv(q))[..., 1:]


def qexp(u):
    """Lie-algebra exponential exp(u) = (cos(|u|/2), sin(|u|/2) u/|u|)
    (Sec. 2, Appendix A).  The printed form is 0/0 at u = 0; below |u| = 1e-4
    sin(t/2)/t is replaced by its series 1/2 - t^2/48 + t^4/3840 (the exact
    Taylor expansion, accurate to ~1e-20 there)."""
    u = np.asarray(u, dtype=np.float64)
    t = np.sqrt(np.sum(u * u, axis=-1, keepdims=True))
    small = t < 1e-4
    safe_t = np.where(small, 1.0, t)
    sinc_half = np.where(small, 0.5 - t * t / 48.0 + t ** 4 / 3840.0,
                         np.sin(0.5 * safe_t) / safe_t)
    return np.concatenate([np.cos(0.5 * t), sinc_half * u], axis=-1)


def cross_matrix(v):
    """[v x], the matrix with [v x] w = v x w (Sec. 2: [v x]_ij = eps_ikj v_k)."""
    v = np.asarray(v, dtype=np.float64)
    C = np.zeros(v.shape[:-1] + (3, 3))
    C[..., 0, 1] = -v[..., 2]
    C[..., 0, 2] = v[..., 1]
    C[..., 1, 0] = v[..., 2]
    C[..., 1, 2] = -v[..., 0]
    C[..., 2, 0] = -v[..., 1]
    C[..., 2, 1] = v[..., 0]
    return C


def dexpinv(u):
    """dexpinv matrix D^-1_u of eq. (dexpinv), extended by D^-1_0 = I
    (Appendix A).  Used only by the identity tests of Appendices C and E."""
    u = np.asarray(u, dtype=np.float64)
    t = np.linalg.norm(u)
    C = cross_matrix(u)
    if t < 1e-6:
        # (t cot(t/2) - 2)/(2 t^2) -> -1/12 as t -> 0
        g = -1.0 / 12.0 - t * t / 720.0
    else:
        g = (t / np.tan(0.5 * t) - 2.0) / (2.0 * t * t)
    return np.eye(3) - 0.5 * C - g * (C @ C)


def psi_matrix(q):
    """Psi_q of eq. (psi_mat_def): dq/dt = Psi_q Omega (Appendix A)."""
    q = np.asarray(q, dtype=np.float64)
    P = np.zeros((4, 3))
    P[0, :] = -q[1:]
    P[1:, :] = q[0] * np.eye(3) - cross_matrix(q[1:])
    return 0.5 * P
