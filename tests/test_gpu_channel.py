"""Slip channel (Sec. 6.3) on the GPU against the oracle, through the C ABI:
walls at y = 0 and y = H = L_y/2 of a box twice the channel's height, kept by
an image system (image forces in the library's spreading, the stress noise
mirrored per Fourier mode in its projection pass; the oracle places
explicit mirror blobs and reflects the stress in real space).

* u_brev: FP64 <= 1e-12, FP32 <= 1e-5, on a five-pass and a three-pass grid;
* blob mobility FP64 <= 1e-12, FP32 <= 1e-5; body mobility likewise;
* one gDC step with the blob-wall potential and pair repulsion, bodies
  within the wall potential's reach: FP64 <= 1e-10 (with the library's nu),
  FP32 <= 1e-5.
Element-wise bounds beside each relative L2 (check_close).
"""
import sys

import numpy as np
import pytest

import workloads as wl
from oracle import fcm, gdc, noise, rigid
from oracle.quaternion import qexp, qmul
from tests._common import check_close, fd_roundoff, oracle_config

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def lib():
    import paper_2106_00449_amd as g
    return g


def _channel_case(name, L, n, shapes, nb, prec, seed, **kw):
    w = wl.small_case(name, n_bodies=nb, n=n, L=L, shapes=shapes, precision=prec, seed=seed, **kw)
    w.channel = True
    return w


def _channel_state(w, seed, margin=1.2):
    """Centres uniform in x, z and in margin < y < H - margin; orientations
    uniform (overlaps allowed: no pair potential needs them apart here)."""
    rng = np.random.default_rng(seed)
    H = w.L[1] / 2
    Y = np.column_stack([rng.uniform(0, w.L[0], w.N), rng.uniform(margin, H - margin, w.N),
                         rng.uniform(0, w.L[2], w.N)])
    q = rng.standard_normal((w.N, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    return Y, q


@pytest.mark.parametrize("prec,n,L", [("fp64", (16, 24, 16), (16.0, 24.0, 16.0)),
                                      ("fp32", (16, 24, 16), (16.0, 24.0, 16.0)),
                                      ("fp32", (32, 32, 32), (24.0, 32.0, 24.0))])
def test_channel_fluct_velocity(lib, prec, n, L):
    w = _channel_case("chfl", L, n, [wl.rod(3)], 2, prec, 41)
    _say("channel fluct", prec, n)
    s = lib.Suspension(**wl.library_kwargs(w))
    for step in [0, 3]:
        u = s.fluct_velocity(step)
        ref = noise.channel_field(fcm.Grid(w.L, w.n), w.kT, w.eta, w.dt, w.noise_seed, step)
        check_close(f"channel u_brev {prec} {n} #{step}", u, ref, 1e-12 if prec == "fp64" else 1e-5)
    s.close()


CASES = [("ch24", (24, 32, 24), (20.0, 28.0, 20.0), [wl.rod(4), wl.boomerang(), wl.tetrahedron()]),
         ("ch32", 32, 32.0, [wl.rod(5), wl.tetrahedron()])]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_channel_blob_and_body_mobility(lib, prec, case):
    name, n, L, shapes = case
    w = _channel_case(name, L, n, shapes, 10, prec, 43)
    Y, q = _channel_state(w, 7)
    rng = np.random.default_rng(8)
    lam = rng.standard_normal((w.M, 3))
    F = rng.standard_normal((w.N, 6))
    _say("channel mobility", name, prec, w.M)
    o = oracle_config(w)
    r = rigid.blob_positions(o.susp.bodies, Y, q)
    s = lib.Suspension(**wl.library_kwargs(w))
    v = s.mobility_apply("blob", Y, q, lam)
    s.close()
    check_close(f"channel blob {name} {prec}", v, fcm.mobility_apply(r, lam, o.susp.fcm),
                1e-12 if prec == "fp64" else 1e-5)
    s = lib.Suspension(**wl.library_kwargs(w, gmres_tol=1e-13 if prec == "fp64" else 1e-7, gmres_maxit=500))
    V = s.mobility_apply("body", Y, q, F, allow_notconv=(prec == "fp32"))
    s.close()
    _, Vref, _ = rigid.solve_saddle(o.susp, Y, r, np.zeros((w.M, 3)), F, tol=1e-14)
    check_close(f"channel body {name} {prec}", V, Vref, 1e-12 if prec == "fp64" else 1e-5)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_channel_step_with_wall_and_pair_forces(lib, prec):
    w = _channel_case("chstep", (20.0, 28.0, 20.0), (24, 32, 24), [wl.rod(4), wl.boomerang(), wl.tetrahedron()],
                      9, prec, 45, dt=0.005, steric_k=40.0 / 2.2, steric_cutoff=2.2,
                      const_force=(0.2, -0.5, 0.3, 0.0, 0.05, 0.0))
    w.wall_k, w.wall_cutoff = 40.0 / 2.2, 2.2
    Y0, q0 = _channel_state(w, 9, margin=0.8)
    o = oracle_config(w)
    r0 = rigid.blob_positions(o.susp.bodies, Y0, q0)
    assert np.abs(gdc.wall_blob_forces(o, r0)).max() > 0     # the walls act in this state
    _say("channel step", prec)
    s = lib.Suspension(**wl.library_kwargs(w, gmres_tol=1e-13 if prec == "fp64" else 1e-7, gmres_maxit=500))
    for step in [0, 1]:
        Y, q = Y0.copy(), q0.copy()
        s.step_counter = step
        st = s.step(Y, q, 1)
        Yr, qr, info = gdc.gdc_step(o, Y0, q0, step, tol=1e-13)
        dx = np.concatenate([(Y - Y0).ravel(), (q - q0).ravel()])
        dr = np.concatenate([(Yr - Y0).ravel(), (qr - q0).ravel()])
        if prec == "fp32":
            assert abs(st["nu"] - info["nu"]) < 1e-5 * max(1.0, abs(info["nu"]))
            check_close(f"channel step fp32 #{step}", dx, dr, 1e-5 + abs(st["nu"] - info["nu"]) / abs(info["nu"]))
        else:
            _, nu_bound = fd_roundoff(o, Y0, q0, gdc.fluct_field(o, step))
            assert abs(st["nu"] - info["nu"]) <= nu_bound, (st["nu"], info["nu"], nu_bound)
            V = info["V"]
            Ya = Y0 + st["nu"] * w.dt * V[:, :3]
            qa = qmul(qexp(st["nu"] * w.dt * V[:, 3:]), q0)
            dxa = np.concatenate([(Ya - Y0).ravel(), (qa - q0).ravel()])
            check_close(f"channel step fp64 #{step} (library nu)", dx, dxa, 1e-10)
    s.close()


def test_channel_rejects_shear_and_periodic_walls(lib):
    w = _channel_case("chbad", 16, 16.0, [wl.rod(3)], 2, "fp64", 47)
    with pytest.raises(lib.GdcError):
        lib.Suspension(**wl.library_kwargs(w, shear_rate=0.1))
    w.channel = False
    with pytest.raises(lib.GdcError):
        lib.Suspension(**wl.library_kwargs(w, wall_k=1.0, wall_cutoff=2.2))
