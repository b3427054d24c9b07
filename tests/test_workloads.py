"""The synthetic initial states: unit quaternions and no two blobs of
different bodies closer than 2a (minimum image), checked by brute force with
the oracle's rotation matrix, for both placement modes."""
import numpy as np
import pytest

import workloads as wl
from oracle.quaternion import rotation_matrix


def _min_interbody_distance(w, Y, q):
    r = np.concatenate([Y[p] + (rotation_matrix(q[p]) @ np.asarray(w.shapes[w.body_shape[p]]).T).T
                        for p in range(w.N)])
    body = np.repeat(np.arange(w.N), [len(w.shapes[s]) for s in w.body_shape])
    L = np.asarray(w.L)
    best = np.inf
    for i in range(0, len(r), 400):
        d = r[i:i + 400, None, :] - r[None, :, :]
        d -= L * np.round(d / L)
        d2 = (d * d).sum(-1)
        d2[body[i:i + 400, None] == body[None, :]] = np.inf
        best = min(best, d2.min())
    return np.sqrt(best)


CASES = [
    lambda: wl.serving_requests(12)[3],
    lambda: wl.serving_requests(12)[7],
    lambda: wl.small_case("batch_mixed", n_bodies=60, n=32, L=30.0,
                          shapes=[wl.rod(10), wl.boomerang(), wl.tetrahedron()], placement="batch"),
    lambda: wl.small_case("seq_mixed", n_bodies=60, n=32, L=30.0,
                          shapes=[wl.rod(10), wl.boomerang(), wl.tetrahedron()]),
]


@pytest.mark.parametrize("make", CASES)
def test_initial_state_has_no_overlaps(make):
    w = make()
    Y, q = wl.initial_state(w)
    assert Y.shape == (w.N, 3) and q.shape == (w.N, 4)
    assert np.abs(np.linalg.norm(q, axis=1) - 1.0).max() < 1e-14
    assert np.all((Y >= 0) & (Y < np.asarray(w.L)))
    assert _min_interbody_distance(w, Y, q) >= 2.0


def test_nematic_cap():
    w = wl.small_case("cap", n_bodies=50, n=32, L=40.0, shapes=[wl.rod(10)], placement="batch",
                      nematic_cap_deg=15.0)
    Y, q = wl.initial_state(w)
    axes = np.array([rotation_matrix(qq)[:, 2] for qq in q])
    assert np.all(axes[:, 2] >= np.cos(np.radians(15.0)) - 1e-12)
    assert _min_interbody_distance(w, Y, q) >= 2.0


def test_pooled_placement_equals_serial():
    ws = wl.serving_requests(6)[:3]
    a = wl.initial_states(ws, processes=3)
    b = [wl.initial_state(w) for w in ws]
    for (Ya, qa), (Yb, qb) in zip(a, b):
        assert np.array_equal(Ya, Yb) and np.array_equal(qa, qb)
