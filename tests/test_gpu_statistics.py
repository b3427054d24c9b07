"""Statistical laws of the whole stochastic step on the GPU, through the C ABI.

Fluctuation-dissipation at the body level.  From a fixed state with no
forces, the one-step increment of a rigid body is, to leading order in dt,
Gaussian with covariance 2 kT dt N: N is the body mobility (the inverse of
K^T M^-1 K, Sec. 2.2), with the drift contributing only O(dt) to the mean
(Sec. 3, weak accuracy).  Many one-step increments are drawn with different
Philox counters; translation and rotation vector (the logarithm of
q1 q0^-1) are stacked, whitened with the oracle's dense N, and their sample
covariance must be the identity within its sampling error.  The same samples
must fail the check against a mobility 25% too large, so the test can tell a
wrong amplitude from the right one.
"""
import math
import sys

import numpy as np
import pytest

import workloads as wl
from oracle import rigid
from oracle.quaternion import qmul
from tests._common import oracle_config

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def lib():
    import paper_2106_00449_amd as g
    return g


def _rotation_vector(q1, q0):
    """theta with q1 q0^-1 = exp(theta) (scalar-first unit quaternions)."""
    q0i = q0 * np.array([1.0, -1.0, -1.0, -1.0])
    d = qmul(q1[None, :], q0i[None, :])[0]
    if d[0] < 0:
        d = -d
    v = d[1:]
    s = np.linalg.norm(v)
    return np.zeros(3) if s == 0 else 2.0 * math.atan2(s, d[0]) * v / s


def _whitened_deviation(X, N):
    Xc = X - X.mean(0)
    Lc = np.linalg.cholesky(N)
    Z = np.linalg.solve(Lc, Xc.T).T
    C = Z.T @ Z / (len(Z) - 1)
    return np.abs(C - np.eye(len(N))).max()


@pytest.mark.parametrize("prec,scheme", [("fp64", "gdc"), ("fp32", "gdc"), ("fp32", "em")])
def test_one_step_covariance_is_2kT_dt_N(lib, prec, scheme):
    w = wl.small_case("fdt_boomerang", n_bodies=1, n=16, L=16.0, shapes=[wl.boomerang()],
                      precision=prec, seed=31, dt=0.01)
    Y0 = np.array([[8.3, 7.6, 8.1]])
    q0 = np.array([0.8, 0.2, -0.4, 0.4])
    q0 = (q0 / np.linalg.norm(q0))[None, :]
    o = oracle_config(w)
    N = rigid.body_mobility(o.susp, Y0, rigid.blob_positions(o.susp.bodies, Y0, q0))
    n_s = 8000
    _say("fdt", prec, scheme, n_s)
    s = lib.Suspension(**wl.library_kwargs(w, scheme=scheme, gmres_tol=1e-9 if prec == "fp64" else 1e-6,
                                           gmres_maxit=300))
    X = np.empty((n_s, 6))
    for k in range(n_s):
        Y, q = Y0.copy(), q0.copy()
        s.step_counter = 7919 * k
        s.step(Y, q, 1)
        X[k, :3] = (Y - Y0)[0]
        X[k, 3:] = _rotation_vector(q[0], q0[0])
    s.close()
    X /= math.sqrt(2.0 * w.kT * w.dt)
    bound = 6.0 * math.sqrt(2.0 / n_s)
    dev = _whitened_deviation(X, N)
    _say("deviation", dev, "bound", bound)
    assert dev < bound, dev
    assert _whitened_deviation(X, 1.25 * N) > bound


def _drift_samples(lib, w, Y0, q0, scheme, rounds, K=16):
    """One-step increments (per body: translation, rotation vector) from the
    same state, K suspensions stepped together per round."""
    from paper_2106_00449_amd import batch_step
    ss = [lib.Suspension(**wl.library_kwargs(w, scheme=scheme, seed=1000 + k, gmres_tol=1e-9, gmres_maxit=300))
          for k in range(K)]
    X = np.empty((rounds * K, 6 * w.N))
    for r in range(rounds):
        for s in ss:
            s.set_state(Y0, q0)
            s.step_counter = r
        left, _, rc = batch_step(ss, [1] * K)
        assert rc == 0 and not any(left)
        for k, s in enumerate(ss):
            Y, q = s.get_state()
            row = X[r * K + k]
            for p in range(w.N):
                row[6 * p:6 * p + 3] = Y[p] - Y0[p]
                row[6 * p + 3:6 * p + 6] = _rotation_vector(q[p], q0[p])
        if r % 250 == 0:
            _say("drift", scheme, "round", r, "of", rounds)
    for s in ss:
        s.close()
    return X


def test_mean_increment_is_the_drift_gdc_has_it_em_does_not(lib):
    # Two tetrahedra at centre distance 3a, no forces: from a fixed state the
    # mean one-step increment is kT dt (d_x . N) + O(dt^2) for gDC (Sec. 3,
    # weak first order) and 0 for Euler-Maruyama (Appendix D), which has no
    # drift correction.  The divergence comes from the oracle's central
    # differences of its dense N.  chi^2 of the sample mean against kT dt d.N
    # with the covariance 2 kT dt N / n (12 degrees of freedom): gDC must stay
    # below the 1e-4 tail quantile (37.7) and EM must exceed it (expected
    # ~73 at this sample size).
    from oracle import gdc as ogdc
    w = wl.small_case("drift_pair", n_bodies=2, n=16, L=16.0, shapes=[wl.tetrahedron()], precision="fp64",
                      seed=41, dt=0.02)
    Y0 = np.array([[6.5, 8.0, 8.3], [9.5, 8.4, 8.0]])
    q0 = np.array([[0.9, 0.3, 0.2, 0.1], [0.7, -0.2, 0.5, 0.3]])
    q0 /= np.linalg.norm(q0, axis=1, keepdims=True)
    o = oracle_config(w)
    N = rigid.body_mobility(o.susp, Y0, rigid.blob_positions(o.susp.bodies, Y0, q0))
    drift = w.kT * w.dt * ogdc.mobility_divergence(o, Y0, q0)
    rounds = 1000
    Cinv = np.linalg.inv(2.0 * w.kT * w.dt * N)
    chi2 = {}
    for scheme in ["gdc", "em"]:
        X = _drift_samples(lib, w, Y0, q0, scheme, rounds)
        dm = X.mean(0) - drift
        chi2[scheme] = float(len(X) * dm @ Cinv @ dm)
    _say("chi2", chi2)
    assert chi2["gdc"] < 37.7, chi2
    assert chi2["em"] > 37.7, chi2
