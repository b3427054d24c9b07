"""Parity with the FP64 oracle at the full workload sizes, through the C ABI.

* 1,000 rods x 10 blobs, L = 128a, grid 128^3 (the benchmarked suspension,
  in the launch configuration the benchmark times): blob mobility in FP32
  and FP64, body mobility (saddle solve) in FP32, and one whole gDC step in
  FP32 from the benchmark's initial state.
* 4,096 mixed rods / boomerangs / tetrahedra, grid 256^3, and 32,768 rods,
  grid 384^3: blob mobility in FP32 (the oracle computes the whole field).
Tolerances: 1e-5 relative L2 in FP32, 1e-12 in FP64; the step increment
1e-5 with the GPU solve at 1e-7 and the oracle's at 1e-10.
"""
import sys
import time

import numpy as np
import pytest

import workloads as wl
from oracle import fcm, gdc, rigid
from tests._common import oracle_config, rel_l2

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
    assert rel_l2(v, ref) < (1e-5 if prec == "fp32" else 1e-12)


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
    assert rel_l2(V, Vref) < 1e-5


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
    assert rel_l2(dx, dr) < 1e-5
    assert abs(st["nu"] - info["nu"]) < 1e-5 * abs(info["nu"])


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
    assert rel_l2(v, ref) < 1e-5
