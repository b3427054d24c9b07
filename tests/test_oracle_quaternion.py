"""Pins of oracle.quaternion against closed forms and invariants of Appendix A."""
import math

import numpy as np

from oracle import quaternion as Q


def _rand_q(rng, n):
    q = rng.standard_normal((n, 4))
    return q / np.linalg.norm(q, axis=1, keepdims=True)


def test_rotation_matrix_orthonormal_det1():
    R = Q.rotation_matrix(_rand_q(np.random.default_rng(0), 50))
    I = np.einsum("nij,nkj->nik", R, R)
    assert np.abs(I - np.eye(3)).max() < 1e-14
    assert np.abs(np.linalg.det(R) - 1.0).max() < 1e-14


def test_rotation_matrix_equals_product_rotation():
    # R(q) x == vector part of q . (0, x) . q^-1 (Appendix A)
    rng = np.random.default_rng(1)
    q = _rand_q(rng, 40)
    x = rng.standard_normal((40, 3))
    a = np.einsum("nij,nj->ni", Q.rotation_matrix(q), x)
    b = Q.rotate_by_product(q, x)
    assert np.abs(a - b).max() < 1e-14


def test_polar_form_is_anticlockwise_rotation():
    # q = (cos(t/2), sin(t/2) e_z) rotates anticlockwise by t about z (textbook)
    t = 0.7
    R = Q.rotation_matrix(Q.qexp(np.array([0.0, 0.0, t])))
    ref = np.array([[math.cos(t), -math.sin(t), 0], [math.sin(t), math.cos(t), 0], [0, 0, 1]])
    assert np.abs(R - ref).max() < 1e-15


def test_exp_inverse_and_norm():
    rng = np.random.default_rng(2)
    u = rng.standard_normal((30, 3)) * np.logspace(-9, 0.5, 30)[:, None]
    p = Q.qmul(Q.qexp(u), Q.qexp(-u))
    assert np.abs(p - np.array([1, 0, 0, 0])).max() < 1e-15
    q = _rand_q(rng, 30)
    n = np.linalg.norm(Q.qmul(Q.qexp(u), q), axis=1)
    assert np.abs(n - 1).max() < 2e-15


def test_exp_small_series_continuity():
    # the series branch and the closed form agree across the switch at 1e-4
    for t in [0.99e-4, 1.01e-4]:
        u = np.array([t, 0.0, 0.0])
        q = Q.qexp(u)
        assert abs(q[1] - math.sin(t / 2)) < 1e-20 + 1e-16 * t
        assert abs(q[0] - math.cos(t / 2)) < 1e-16


def test_hamilton_product_composes_rotations():
    rng = np.random.default_rng(3)
    p, q = _rand_q(rng, 10), _rand_q(rng, 10)
    lhs = Q.rotation_matrix(Q.qmul(p, q))
    rhs = np.einsum("nij,njk->nik", Q.rotation_matrix(p), Q.rotation_matrix(q))
    assert np.abs(lhs - rhs).max() < 1e-14


def _div_dexpinv(u0, h=1e-5):
    div = np.zeros(3)
    for j in range(3):
        e = np.zeros(3)
        e[j] = h
        dD = (Q.dexpinv(u0 + e) - Q.dexpinv(u0 - e)) / (2 * h)
        div += dD[j, :]
    return div


def test_dexpinv_identities():
    # D^-1_0 = I; d_j D^-1_jb = 0 at u = 0 (the point where Appendix E uses it);
    # d_j D^-1_ia |_0 = -eps_ija / 2 (Appendix E)
    assert np.abs(Q.dexpinv(np.zeros(3)) - np.eye(3)).max() < 1e-15
    assert np.abs(_div_dexpinv(np.zeros(3))).max() < 1e-9
    # Away from 0, differentiating the printed form gives d_j D^-1_jb = -2 g(|u|) u_b
    # with g = (|u| cot(|u|/2) - 2)/(2|u|^2): the [u x]^2 term is not divergence-free.
    u0 = np.array([0.3, -0.2, 0.5])
    t = np.linalg.norm(u0)
    g = (t / np.tan(t / 2) - 2) / (2 * t * t)
    assert np.abs(_div_dexpinv(u0) + 2 * g * u0).max() < 1e-8
    h = 1e-5
    eps = np.zeros((3, 3, 3))
    eps[0, 1, 2] = eps[1, 2, 0] = eps[2, 0, 1] = 1
    eps[0, 2, 1] = eps[2, 1, 0] = eps[1, 0, 2] = -1
    for j in range(3):
        e = np.zeros(3)
        e[j] = h
        dD = (Q.dexpinv(e) - Q.dexpinv(-e)) / (2 * h)
        assert np.abs(dD + 0.5 * eps[:, j, :]).max() < 1e-8


def test_psi_matches_half_product():
    rng = np.random.default_rng(4)
    q = _rand_q(rng, 1)[0]
    w = rng.standard_normal(3)
    lhs = Q.psi_matrix(q) @ w
    rhs = 0.5 * Q.qmul(np.concatenate([[0.0], w]), q)
    assert np.abs(lhs - rhs).max() < 1e-15


def test_dexpinv_maps_angular_velocity():
    # q(t) = exp(u(t)) . q0 with du/dt = D^-1_u Omega satisfies dq/dt = Psi_q Omega
    rng = np.random.default_rng(5)
    q0 = _rand_q(rng, 1)[0]
    u = np.array([0.4, -0.3, 0.2])
    Om = rng.standard_normal(3)
    h = 1e-6
    du = Q.dexpinv(u) @ Om
    qp = Q.qmul(Q.qexp(u + h * du), q0)
    qm = Q.qmul(Q.qexp(u - h * du), q0)
    q = Q.qmul(Q.qexp(u), q0)
    assert np.abs((qp - qm) / (2 * h) - Q.psi_matrix(q) @ Om).max() < 1e-8
