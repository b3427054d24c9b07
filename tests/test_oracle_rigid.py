"""Pins of oracle.rigid: the printed K^T K block, least-squares exactness,
the frozen null space of collinear and one-blob bodies, GMRES against the
dense direct solve, independence from the preconditioner, force balance,
and symmetry / positive definiteness of the body mobility N."""
import math

import numpy as np

import workloads as wl
from oracle import fcm, rigid
from oracle.quaternion import rotation_matrix

ETA = 1.0 / (6.0 * math.pi)


def _susp(shapes, body_shape, L=12.0, n=12):
    p = fcm.FcmParams(fcm.Grid([L] * 3, (n,) * 3), ETA, 1.0 / math.sqrt(math.pi), 3.0)
    return rigid.Suspension(p, rigid.Bodies(shapes, body_shape), 1.0)


def _state(s, seed):
    rng = np.random.default_rng(seed)
    N = s.bodies.N
    q = rng.standard_normal((N, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    Y = rng.uniform(0, s.fcm.grid.L[0], (N, 3))
    return Y, q, rigid.blob_positions(s.bodies, Y, q)


def test_KtK_matches_printed_block():
    rng = np.random.default_rng(0)
    rel = rng.standard_normal((7, 3))
    K = rigid.body_K(rel)
    assert np.abs(K.T @ K - rigid.KtK_closed_form(rel)).max() < 1e-13


def test_K_is_rigid_motion():
    rng = np.random.default_rng(1)
    rel = rng.standard_normal((5, 3))
    U, Om = rng.standard_normal(3), rng.standard_normal(3)
    v = (rigid.body_K(rel) @ np.concatenate([U, Om])).reshape(-1, 3)
    assert np.abs(v - (U + np.cross(Om, rel))).max() < 1e-14


def test_lsq_exact_for_rigid_input():
    s = _susp([wl.boomerang(), wl.tetrahedron()], [0, 1, 0])
    Y, q, r = _state(s, 2)
    V0 = np.random.default_rng(3).standard_normal((3, 6))
    v = rigid.K_apply(s.bodies, Y, r, V0)
    assert np.abs(rigid.lsq_velocity(s.bodies, Y, r, v) - V0).max() < 1e-12


def test_lsq_collinear_and_single_blob_null_space():
    s = _susp([wl.rod(4), np.zeros((1, 3))], [0, 1])
    Y, q, r = _state(s, 4)
    rng = np.random.default_rng(5)
    v = rng.standard_normal((s.bodies.M, 3))
    calV = rigid.lsq_velocity(s.bodies, Y, r, v)
    axis = rotation_matrix(q[0]) @ np.array([0, 0, 1.0])
    assert abs(calV[0, 3:] @ axis) < 1e-12             # no spin about the rod axis
    assert np.abs(calV[1, 3:]).max() < 1e-14           # a point blob has no rotation
    assert np.abs(calV[1, :3] - v[-1]).max() < 1e-14   # one blob: calV = v exactly
    # the residual is orthogonal to range(K) (normal equations)
    res = v[:4] - rigid.K_apply(rigid.Bodies([wl.rod(4)], [0]), Y[:1], r[:4], calV[:1])
    assert np.abs(rigid.body_K(r[:4] - Y[0]).T @ res.ravel()).max() < 1e-12


def test_gmres_equals_dense_and_preconditioner_free():
    s = _susp([wl.rod(3), wl.tetrahedron()], [0, 1, 1, 0])
    Y, q, r = _state(s, 6)
    rng = np.random.default_rng(7)
    slip = rng.standard_normal((s.bodies.M, 3))
    F = rng.standard_normal((s.bodies.N, 6))
    lam_d, V_d, _ = rigid.solve_saddle(s, Y, r, slip, F, dense=True)
    lam_g, V_g, info = rigid.solve_saddle(s, Y, r, slip, F, dense=False, tol=1e-13)
    assert np.abs(V_g - V_d).max() < 1e-10 * np.abs(V_d).max()
    # plain (unpreconditioned) GMRES converges to the same answer
    W = fcm.weights(r, s.fcm)
    rhs = rigid.saddle_rhs(s, Y, r, slip, F)
    x, its, rr = rigid.gmres(lambda x: rigid.saddle_apply(s, Y, r, x, W), rhs, None, tol=1e-13, restart=200)
    assert np.abs(x[3 * s.bodies.M:].reshape(-1, 6) - V_d).max() < 1e-9 * np.abs(V_d).max()
    assert info["iterations"] < its                       # the preconditioner helps
    # force balance K^T lambda = F on the non-null part; rigid-body slip
    Kt = rigid.KT_apply(s.bodies, Y, r, lam_d)
    for p, sl, rel in rigid.per_body(s.bodies, Y, r):
        Pi = rigid.null_projector(rel)
        assert np.abs(Kt[p] - (F[p] - Pi @ F[p])).max() < 1e-10
        assert np.abs(Pi @ V_d[p]).max() < 1e-12


def test_body_mobility_symmetric_positive_and_matches_solve():
    s = _susp([wl.boomerang()], [0, 0])
    Y, q, r = _state(s, 8)
    N = rigid.body_mobility(s, Y, r)
    assert np.abs(N - N.T).max() < 1e-9 * np.abs(N).max()
    assert np.linalg.eigvalsh(0.5 * (N + N.T)).min() > 0
    F = np.random.default_rng(9).standard_normal((2, 6))
    _, V, _ = rigid.solve_saddle(s, Y, r, np.zeros((s.bodies.M, 3)), F, dense=True)
    assert np.abs(V.ravel() - N @ F.ravel()).max() < 1e-8 * np.abs(V).max()


def test_single_blob_body_is_blob_mobility():
    # a one-blob body under a force moves with the blob self-mobility M_ii
    s = _susp([np.zeros((1, 3))], [0])
    Y = np.array([[2.5, 3.5, 4.5]])
    q = np.array([[1.0, 0, 0, 0]])
    r = rigid.blob_positions(s.bodies, Y, q)
    F = np.array([[0.0, 0.0, 1.0, 0.3, 0.2, 0.1]])
    _, V, _ = rigid.solve_saddle(s, Y, r, np.zeros((1, 3)), F, dense=True)
    Mm = fcm.dense_mobility(r, s.fcm)
    assert np.abs(V[0, :3] - Mm @ F[0, :3]).max() < 1e-12
    assert np.abs(V[0, 3:]).max() < 1e-14


def test_rpy_tensor_continuous_and_self():
    a = 1.0
    assert np.allclose(rigid.rpy_tensor(np.zeros(3), a, ETA), np.eye(3))   # 1/(6 pi eta a) = 1
    d = np.array([0.0, 0.0, 2.0])
    lo = rigid.rpy_tensor(d * (1 - 1e-12), a, ETA)
    hi = rigid.rpy_tensor(d, a, ETA)
    assert np.abs(lo - hi).max() < 1e-10
