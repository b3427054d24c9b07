"""Parity with the FP64 oracle at the full workload sizes, through the C ABI.

* 1,000 rods x 10 blobs, L = 128a, grid 128^3 (the benchmarked suspension,
  in the launch configuration the benchmark times): blob mobility in FP32
  and FP64, body mobility (saddle solve) in FP32, and one whole gDC step in
  FP32 from the benchmark's initial state.
* 4,096 mixed rods / boomerangs / tetrahedra, grid 256^3, and 32,768 rods,
  grid 384^3: blob mobility in FP32 (the oracle computes the whole field),
  and the first gDC step against the oracle's step stored in
  tests/golden/step0_*.json by tests/golden/make_golden.py (the oracle takes
  minutes to an hour per step there): nu, and for a fixed sample of bodies
  the least-squares velocity calV, the divergence terms d_p and the
  increment, element by element.
* 120 rods on a 192^3 grid (five-pass transforms at a radix-3 size): blob
  mobility in FP32 and FP64.
Tolerances: 1e-5 relative L2 in FP32, 1e-12 in FP64, with every element
within 4x that of the largest magnitude; the step increment 1e-5 with the
GPU solve at 1e-7 and the oracle's at 1e-10.
"""
import json
import os
import sys
import time

import numpy as np
import pytest

import workloads as wl
from oracle import fcm, gdc, rigid
from tests._common import check_close, oracle_config

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def lib():
    import paper_2106_00449_amd as g
    return g


@pytest.fixture(scope="module")
def rods1000():
    w = wl.rods1000("fp32")
    Y, q = wl.initial_state(w)
    return w, Y, q


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_rods1000_blob_mobility(lib, rods1000, prec):
    w, Y, q = rods1000
    lam = np.random.default_rng(31).standard_normal((w.M, 3))
    _say("full blob rods1000", prec)
    s = lib.Suspension(**wl.library_kwargs(w, precision=prec))
    v = s.mobility_apply("blob", Y, q, lam)
    s.close()
    o = oracle_config(w)
    ref = fcm.mobility_apply(rigid.blob_positions(o.susp.bodies, Y, q), lam, o.susp.fcm)
    check_close(f"full blob rods1000 {prec}", v, ref, 1e-5 if prec == "fp32" else 1e-12)


def test_rods1000_body_mobility(lib, rods1000):
    w, Y, q = rods1000
    F = np.random.default_rng(32).standard_normal((w.N, 6))
    _say("full body rods1000 fp32")
    s = lib.Suspension(**wl.library_kwargs(w, gmres_tol=1e-7, gmres_maxit=500))
    V = s.mobility_apply("body", Y, q, F, allow_notconv=True)
    s.close()
    o = oracle_config(w)
    r = rigid.blob_positions(o.susp.bodies, Y, q)
    t0 = time.time()
    _, Vref, _ = rigid.solve_saddle(o.susp, Y, r, np.zeros((w.M, 3)), F, tol=1e-9)
    _say("oracle solve", f"{time.time() - t0:.1f} s")
    check_close("full body rods1000 fp32", V, Vref, 1e-5)


def test_rods1000_one_step(lib, rods1000):
    w, Y0, q0 = rods1000
    _say("full step rods1000 fp32")
    s = lib.Suspension(**wl.library_kwargs(w, gmres_tol=1e-7, gmres_maxit=500))
    Y, q = Y0.copy(), q0.copy()
    st = s.step(Y, q, 1)
    s.close()
    o = oracle_config(w)
    t0 = time.time()
    Yr, qr, info = gdc.gdc_step(o, Y0, q0, 0, tol=1e-10)
    _say("oracle step", f"{time.time() - t0:.1f} s", "nu", info["nu"], st["nu"])
    dx = np.concatenate([(Y - Y0).ravel(), (q - q0).ravel()])
    dr = np.concatenate([(Yr - Y0).ravel(), (qr - q0).ravel()])
    assert abs(st["nu"] - info["nu"]) < 1e-5 * max(1.0, abs(info["nu"]))
    check_close("full step rods1000 fp32", dx, dr, 1e-5 + abs(st["nu"] - info["nu"]) / abs(info["nu"]))


@pytest.mark.parametrize("make", [wl.mixed4096, wl.rods32768], ids=["mixed4096", "rods32768"])
def test_large_blob_mobility(lib, make):
    w = make()
    t0 = time.time()
    Y, q = wl.initial_state(w)
    _say("full blob", w.name, w.M, w.n, f"placement {time.time() - t0:.1f} s")
    lam = np.random.default_rng(33).standard_normal((w.M, 3))
    s = lib.Suspension(**wl.library_kwargs(w, precision="fp32"))
    v = s.mobility_apply("blob", Y, q, lam)
    s.close()
    o = oracle_config(w)
    ref = fcm.mobility_apply(rigid.blob_positions(o.susp.bodies, Y, q), lam, o.susp.fcm)
    check_close(f"full blob {w.name} fp32", v, ref, 1e-5)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_grid192_blob_mobility(lib, prec):
    w = wl.small_case("rods192", n_bodies=120, n=192, L=192.0, shapes=[wl.rod(10)], precision=prec, seed=21)
    Y, q = wl.initial_state(w)
    lam = np.random.default_rng(34).standard_normal((w.M, 3))
    _say("blob rods192", prec, w.M)
    s = lib.Suspension(**wl.library_kwargs(w))
    v = s.mobility_apply("blob", Y, q, lam)
    s.close()
    o = oracle_config(w)
    ref = fcm.mobility_apply(rigid.blob_positions(o.susp.bodies, Y, q), lam, o.susp.fcm)
    check_close(f"blob rods192 {prec}", v, ref, 1e-5 if prec == "fp32" else 1e-12)


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.mark.parametrize("make", [wl.mixed4096, wl.rods32768], ids=["mixed4096", "rods32768"])
def test_large_first_step_against_stored_oracle(lib, make):
    # the oracle's step 0 (FP64, GMRES 1e-10) from the workload's seeded
    # state, written by tests/golden/make_golden.py; the library steps the
    # same state in FP32 with the same Philox noise
    import hashlib
    w = make()
    path = os.path.join(GOLDEN, f"step0_{w.name}.json")
    if not os.path.exists(path):
        pytest.skip(f"{path} not generated")
    ref = json.load(open(path))
    Y0, q0 = wl.initial_state(w)
    digest = hashlib.sha256(np.ascontiguousarray(Y0).tobytes() + np.ascontiguousarray(q0).tobytes()).hexdigest()
    assert digest == ref["state_sha256"], "initial state differs from the one the fixture was made from"
    idx = np.asarray(ref["bodies"])
    _say("golden step", w.name, w.M, w.n)
    s = lib.Suspension(**wl.library_kwargs(w, precision="fp32", gmres_tol=1e-7, gmres_maxit=500))
    calV, d = s.predictor(Y0, q0, 0)
    Y, q = Y0.copy(), q0.copy()
    s.step_counter = 0
    st = s.step(Y, q, 1)
    s.close()
    print(f"[err] golden {w.name}: nu gpu {st['nu']:.8f} oracle {ref['nu']:.8f}", flush=True)
    assert abs(st["nu"] - ref["nu"]) < 1e-5 * max(1.0, abs(ref["nu"]))
    # the increment is nu dt V: its relative error is V's plus nu's
    nu_rel = abs(st["nu"] - ref["nu"]) / abs(ref["nu"])
    check_close(f"golden {w.name} calV translational", calV[idx, :3], np.asarray(ref["calV"])[:, :3], 1e-5,
                elem_tol=4e-5 * ref["max_calV_t"] / np.abs(np.asarray(ref["calV"])[:, :3]).max())
    check_close(f"golden {w.name} calV rotational", calV[idx, 3:], np.asarray(ref["calV"])[:, 3:], 1e-5,
                elem_tol=4e-5 * ref["max_calV_r"] / np.abs(np.asarray(ref["calV"])[:, 3:]).max())
    check_close(f"golden {w.name} d", d[idx], np.asarray(ref["d"]), 1e-5)
    check_close(f"golden {w.name} dY", (Y - Y0)[idx], np.asarray(ref["dY"]), 1e-5 + nu_rel)
    check_close(f"golden {w.name} dq", (q - q0)[idx], np.asarray(ref["dq"]), 1e-5 + nu_rel)
    # whole-vector scales the fixture recorded
    assert abs(np.linalg.norm(Y - Y0) - ref["norm_dY"]) < (1e-5 + nu_rel) * ref["norm_dY"]
    assert abs(np.linalg.norm(q - q0) - ref["norm_dq"]) < (1e-5 + nu_rel) * ref["norm_dq"]
