"""Parity of the HIP library (through the C ABI) with the FP64 oracle.

Tolerances: relative L2 over the whole output, and every element within
4x that of the output's largest magnitude (check_close).  Deterministic
mobility <= 1e-12 in FP64 (GMRES to 1e-13 for the body mode) and <= 1e-5 in
FP32; the least-squares velocity calV <= 1e-12 (FP64) and 1e-5 (FP32);
one-step increments <= 1e-10 (FP64) and <= 1e-5 (FP32); the FP64 divergence
terms d_p and nu within 8x the oracle's own rounding of its forward
differences (fd_roundoff); noise normals bit-identical.
"""
import math
import sys

import numpy as np
import pytest

import workloads as wl
from oracle import fcm, gdc, noise, philox, rigid
from oracle.quaternion import qexp, qmul
from tests._common import check_close, fd_roundoff, oracle_config, rel_l2

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def lib():
    import paper_2106_00449_amd as g
    return g


def _susp(lib, w, **over):
    return lib.Suspension(**wl.library_kwargs(w, **over))


def _rand_blobs(w, seed):
    rng = np.random.default_rng(seed)
    Y, q = wl.initial_state(w)
    lam = rng.standard_normal((w.M, 3))
    F = rng.standard_normal((w.N, 6))
    return Y, q, lam, F


# ------------------------------------------------------------------ noise

def test_philox_normals_bit_identical(lib):
    w = wl.small_case(n=8, L=8.0)
    s = _susp(lib, w)
    for (seed, c1, step) in [(0, 0, 0), (12345, 2, 7), (2**40 + 3, 17, 2**33 + 5)]:
        _say("philox", seed, c1, step)
        g = s.philox_normals(seed, c1, step, 1000, 200000)
        o = philox.normals(seed, np.arange(1000, 201000), c1, step)
        assert np.array_equal(g, o), np.abs(g - o).max()


# FP32 grids with n1 = n2 <= 128 (and n0 <= 128) take the three-pass plane
# transforms, other grids the five-pass ones: both are covered.
@pytest.mark.parametrize("prec,n,L", [("fp64", (16, 12, 24), (16.0, 12.0, 24.0)),
                                      ("fp32", (16, 12, 24), (16.0, 12.0, 24.0)),
                                      ("fp32", (24, 32, 32), (20.0, 26.0, 26.0)),
                                      ("fp32", (48, 48, 48), (32.0, 32.0, 32.0)),
                                      ("fp64", (48, 48, 48), (32.0, 32.0, 32.0)),
                                      ("fp32", (128, 12, 24), (96.0, 12.0, 19.0)),
                                      ("fp32", (24, 128, 256), (18.0, 96.0, 192.0)),
                                      ("fp32", (12, 12, 128), (9.0, 9.0, 96.0))])
def test_fluct_velocity_field(lib, prec, n, L):
    w = wl.small_case(n=n, L=L, precision=prec, seed=11)
    _say("fluct", prec, n)
    s = _susp(lib, w)
    for step in [0, 5]:
        u = s.fluct_velocity(step)
        ref = noise.fourier_field(fcm.Grid(w.L, w.n), w.kT, w.eta, w.dt, w.noise_seed, step)
        tol = 1e-12 if prec == "fp64" else 1e-5
        check_close(f"u_brev {prec} {n} step {step}", u, ref, tol)


# ------------------------------------------------------------------ mobility

CASES = [
    # name, grid, box, shapes
    ("small8", 8, 8.0, [wl.rod(2), np.zeros((1, 3))]),
    ("ragged24", (24, 16, 12), (20.0, 15.0, 13.0), [wl.tetrahedron(), wl.rod(3)]),
    ("rods48", 48, 32.0, [wl.rod(5)]),
    ("slab16x32", (16, 32, 32), (13.0, 24.0, 24.0), [wl.rod(4), wl.boomerang()]),
    ("mixed64", 64, 48.0, [wl.rod(10), wl.boomerang(), wl.tetrahedron()]),
    # a 20-blob shape: preconditioner block of 66, above the matrix-core
    # kernel's limit, so the per-body kernel runs
    ("rod20", 48, 48.0, [wl.rod(20), wl.tetrahedron()]),
    # one 8x8x8 tile holding 80 blobs: the spreading hit loop takes two
    # rounds of 64 and the tile sort ranks more records than a wave
    ("dense8", 8, 12.0, [wl.rod(5)]),
    # 96^3: the three-pass plane transforms at their largest radix-3 size
    # (FP32) and the five-pass transforms (FP64)
    ("rods96", 96, 96.0, [wl.rod(10)]),
    # grid spacing 0.375a: a 10-blob rod is longer than the 24 spacings an
    # averaging cluster may span, so its blobs are averaged in two clusters
    ("fine64", 64, 24.0, [wl.rod(10), wl.boomerang()]),
    # five-pass FP32 transforms with axis-0 lines of 128 (moved and projected
    # in whole-wave runs) and n1 = 12: the last workgroup of lines along
    # axis 1 holds 4 of its 8
    ("long128", (128, 12, 24), (96.0, 12.0, 19.0), [wl.rod(4), wl.tetrahedron()]),
    # five-pass FP32 transforms with axis-1 lines of 128 and axis-2 lines of
    # 256 (whole-wave runs) and n0 = 24: the last workgroup of axis-1 lines
    # holds 8 of its 16
    ("wide128", (24, 128, 256), (18.0, 96.0, 192.0), [wl.rod(4), wl.boomerang()]),
    # axis-2 lines of 128 in the untiled field layout (8 does not divide
    # n0 = n1 = 12), six of a workgroup's eight line pairs present
    ("slab12", (12, 12, 128), (9.0, 9.0, 96.0), [wl.rod(3), wl.tetrahedron()]),
]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_blob_mobility(lib, prec, case):
    name, n, L, shapes = case
    nb = {"small8": 3, "dense8": 16, "rods96": 60, "fine64": 8}.get(name, 12)
    w = wl.small_case(name, n_bodies=nb, n=n, L=L, shapes=shapes, precision=prec, seed=3)
    Y, q, lam, _ = _rand_blobs(w, 1)
    _say("blob", name, prec, w.M)
    s = _susp(lib, w)
    v = s.mobility_apply("blob", Y, q, lam)
    o = oracle_config(w)
    r = rigid.blob_positions(o.susp.bodies, Y, q)
    ref = fcm.mobility_apply(r, lam, o.susp.fcm)
    tol = 1e-12 if prec == "fp64" else 1e-5
    check_close(f"blob {name} {prec}", v, ref, tol)


# the saddle solve of every case but the smallest (and wide128, whose
# oracle solve takes half a minute for nothing the blob mode leaves untested)
BODY_CASES = [c for c in CASES[1:] if c[0] != "wide128"]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("case", BODY_CASES, ids=[c[0] for c in BODY_CASES])
def test_body_mobility(lib, prec, case):
    name, n, L, shapes = case
    w = wl.small_case(name, n_bodies=8, n=n, L=L, shapes=shapes, precision=prec, seed=5)
    Y, q, _, F = _rand_blobs(w, 2)
    _say("body", name, prec, w.M)
    s = _susp(lib, w, gmres_tol=1e-13 if prec == "fp64" else 1e-7, gmres_maxit=500)
    V = s.mobility_apply("body", Y, q, F, allow_notconv=(prec == "fp32"))
    o = oracle_config(w)
    r = rigid.blob_positions(o.susp.bodies, Y, q)
    _, Vref, _ = rigid.solve_saddle(o.susp, Y, r, np.zeros((w.M, 3)), F, tol=1e-14)
    tol = 1e-12 if prec == "fp64" else 1e-5
    check_close(f"body {name} {prec}", V, Vref, tol)


# ------------------------------------------------------------------ gDC pieces

@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_predictor(lib, prec):
    w = wl.small_case("pred", n_bodies=10, n=(24, 24, 32), L=(20.0, 20.0, 26.0),
                      shapes=[wl.rod(4), wl.boomerang(), wl.tetrahedron(), np.zeros((1, 3))],
                      precision=prec, seed=9)
    Y, q, _, _ = _rand_blobs(w, 3)
    _say("predictor", prec)
    s = _susp(lib, w)
    calV, d = s.predictor(Y, q, 4)
    o = oracle_config(w)
    ufl = gdc.fluct_field(o, 4)
    cref, dref = gdc.predictor(o, Y, q, ufl)
    if prec == "fp64":
        check_close("predictor calV fp64", calV, cref, 1e-12)
        # d_p: the oracle's forward differences carry their own rounding
        # (fd_roundoff); the library forms the differences from weight
        # differences, far more accurately
        bound, _ = fd_roundoff(o, Y, q, ufl)
        gap = np.abs(d - dref)
        print(f"[err] predictor d fp64: max |gap| / bound {np.max(gap / bound):.3f}", flush=True)
        assert np.all(gap <= bound), (gap, bound)
    else:
        check_close("predictor calV fp32", calV, cref, 1e-5)
        check_close("predictor d fp32", d, dref, 1e-5)


STEP_CASES = [
    ("rods8", lambda p: wl.rods8() if p == "fp64" else _with_prec(wl.rods8(), p), {}),
    ("mixed_forces", lambda p: wl.small_case("mixed_forces", n_bodies=9, n=(32, 32, 48), L=(24.0, 24.0, 36.0),
                                             shapes=[wl.rod(4), wl.boomerang(), wl.tetrahedron()],
                                             precision=p, seed=13, dt=0.005,
                                             steric_k=40.0 / 2.2, steric_cutoff=2.2,
                                             const_force=(0.0, 0.0, 1.0, 0.1, 0.0, 0.0),
                                             shear_rate=0.1), {}),
]


def _with_prec(w, p):
    w.precision = p
    return w


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("case", STEP_CASES, ids=[c[0] for c in STEP_CASES])
@pytest.mark.parametrize("scheme,div", [("gdc", "fd"), ("gdc", "rfd"), ("em", "fd")])
def test_one_step_increment(lib, prec, case, scheme, div):
    name, make, _ = case
    w = make(prec)
    Y0, q0 = wl.initial_state(w)
    _say("step", name, prec, scheme, div)
    s = _susp(lib, w, scheme=scheme, divergence=div,
              gmres_tol=1e-13 if prec == "fp64" else 1e-7, gmres_maxit=500)
    o = oracle_config(w, divergence=div)
    for step in [0, 1]:
        Y, q = Y0.copy(), q0.copy()
        s.step_counter = step
        st = s.step(Y, q, 1)
        if scheme == "gdc":
            Yr, qr, info = gdc.gdc_step(o, Y0, q0, step, tol=1e-13)
        else:
            Yr, qr, info = gdc.em_step(o, Y0, q0, step, tol=1e-13)
        dx_gpu = np.concatenate([(Y - Y0).ravel(), (q - q0).ravel()])
        dx_ref = np.concatenate([(Yr - Y0).ravel(), (qr - q0).ravel()])
        if prec == "fp32":
            check_close(f"step {name} {scheme}-{div} fp32 #{step}", dx_gpu, dx_ref, 1e-5)
            if scheme == "gdc":
                assert abs(st["nu"] - info["nu"]) < 1e-5 * max(1.0, abs(info["nu"]))
        else:
            # nu: the oracle's forward differences at delta = 1e-6 carry FP64
            # rounding, measured by fd_roundoff.  The rest of the step is
            # checked with the library's nu substituted into the oracle's
            # update, to 1e-10, and the whole increment to 1e-10 plus the
            # relative nu gap.
            nu_g = st["nu"] if scheme == "gdc" else 1.0
            if scheme == "gdc":
                _, nu_bound = fd_roundoff(o, Y0, q0, gdc.fluct_field(o, step), div, step)
                print(f"[err] nu fp64 {name} {div} #{step}: gap {abs(nu_g - info['nu']):.3e} "
                      f"bound {nu_bound:.3e}", flush=True)
                assert abs(nu_g - info["nu"]) <= nu_bound, (nu_g, info["nu"], nu_bound)
            V = info["V"]
            Ya = Y0 + nu_g * w.dt * V[:, :3]
            qa = qmul(qexp(nu_g * w.dt * V[:, 3:]), q0)
            dx_alt = np.concatenate([(Ya - Y0).ravel(), (qa - q0).ravel()])
            check_close(f"step {name} {scheme}-{div} fp64 #{step} (library nu)", dx_gpu, dx_alt, 1e-10)
            nu_rel = abs(nu_g - info.get("nu", 1.0)) / abs(info.get("nu", 1.0))
            check_close(f"step {name} {scheme}-{div} fp64 #{step}", dx_gpu, dx_ref, 1e-10 + nu_rel)
        assert s.step_counter == step + 1


def test_zero_temperature_step_is_deterministic(lib):
    w = wl.small_case("kT0", n_bodies=6, n=24, L=20.0, shapes=[wl.boomerang(), wl.rod(3)], precision="fp64",
                      kT=0.0, const_force=(0.0, 0.2, 1.0, 0.0, 0.1, 0.0))
    Y0, q0 = wl.initial_state(w)
    _say("kT0")
    s = _susp(lib, w, gmres_tol=1e-13)
    Y, q = Y0.copy(), q0.copy()
    st = s.step(Y, q, 1)
    assert st["nu"] == 1.0
    o = oracle_config(w)
    Yr, qr, _ = gdc.gdc_step(o, Y0, q0, 0, tol=1e-13)
    check_close("kT0 step fp64", Y - Y0, Yr - Y0, 1e-10)
    assert np.abs(np.linalg.norm(q, axis=1) - 1).max() < 1e-14


def test_error_paths(lib):
    w = wl.small_case(n=8, L=8.0)
    Y, q = wl.initial_state(w)
    s = _susp(lib, w)
    bad = q.copy()
    bad[0] *= 1.1
    with pytest.raises(lib.GdcError) as e:
        s.mobility_apply("blob", Y, bad, np.zeros((w.M, 3)))
    assert e.value.code == -1
    with pytest.raises(lib.GdcError):
        lib.Suspension(**wl.library_kwargs(w, n=(10, 8, 8)))
    with pytest.raises(lib.GdcError):
        lib.Suspension(**wl.library_kwargs(w, trunc=4.5))
    # a NaN position is rejected before anything is launched
    Yn = Y.copy()
    Yn[0, 0] = np.nan
    qn = q.copy()
    with pytest.raises(lib.GdcError) as e:
        s.step(Yn, qn, 1)
    assert e.value.code == -1


@pytest.mark.parametrize("prec,kT", [("fp64", 0.0), ("fp32", 0.0), ("fp32", 1.0)])
def test_sine_forcing_step(lib, prec, kT):
    # the rheology forcing f0 sin(k y) e_x: one step's increment and the
    # measured amplitude v_x against the oracle (kT = 0 isolates the
    # deterministic forcing response, nu = 1)
    w = wl.small_case("sine", n_bodies=9, n=(32, 32, 48), L=(24.0, 24.0, 36.0),
                      shapes=[wl.rod(4), wl.boomerang(), wl.tetrahedron()], precision=prec, seed=19,
                      dt=0.005, kT=kT, sine_force=2.0)
    Y0, q0 = wl.initial_state(w)
    _say("sine", prec, kT)
    s = lib.Suspension(**wl.library_kwargs(w, gmres_tol=1e-13 if prec == "fp64" else 1e-7, gmres_maxit=500))
    Y, q = Y0.copy(), q0.copy()
    st = s.step(Y, q, 1)
    s.close()
    o = oracle_config(w)
    Yr, qr, info = gdc.gdc_step(o, Y0, q0, 0, tol=1e-13)
    dx = np.concatenate([(Y - Y0).ravel(), (q - q0).ravel()])
    dr = np.concatenate([(Yr - Y0).ravel(), (qr - q0).ravel()])
    tol = 1e-10 if prec == "fp64" else 1e-5
    check_close(f"sine step {prec} kT {kT}", dx, dr, tol)
    assert abs(st["sine_vx"] - info["sine_vx"]) < tol * abs(info["sine_vx"])
