"""Shared test helpers: a workload as an oracle configuration or a library
handle, relative errors, and the GPU-availability gate."""
import numpy as np

import workloads as wl
from oracle import fcm, gdc, rigid


def oracle_config(w: wl.Workload, kT=None, dt=None, divergence="fd", fd_delta=1e-6):
    p = fcm.FcmParams(fcm.Grid(w.L, w.n), w.eta, w.sigma, w.rc, channel=w.channel)
    s = rigid.Suspension(p, rigid.Bodies(w.shapes, w.body_shape), w.a)
    F = gdc.Forces(w.steric_k, w.steric_cutoff, np.asarray(w.const_force, dtype=np.float64), w.shear_rate,
                   w.sine_force, w.wall_k, w.wall_cutoff)
    return gdc.Config(s, w.kT if kT is None else kT, w.dt if dt is None else dt, w.noise_seed, F,
                      fd_delta=fd_delta, divergence=divergence)


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def gpu_available():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def fd_roundoff(o, Y, q, ufl, divergence="fd", step=0, safety=8.0):
    """Rounding of the oracle's FP64 divergence terms d_p and of nu.

    The oracle forms each forward difference calV(x + delta e) - calV(x) from
    two separately rounded averages, so with delta = 1e-6 each quotient
    carries rounding of order eps |v| sqrt(S) / delta (S stencil points).
    Its size is measured rather than modelled: translating every body by a
    whole grid cell and rolling the field with it leaves d_p unchanged in
    exact arithmetic but changes every rounded operand, so the spread of d_p
    over three such translations is the oracle's own rounding.  Returns
    (per-body bound on |d_gpu - d_oracle|, bound on |nu_gpu - nu_oracle|),
    each `safety` times the largest change seen."""
    from oracle import gdc
    Y = np.asarray(Y, dtype=np.float64).reshape(-1, 3)
    calV, d = gdc.predictor(o, Y, q, ufl)
    if divergence == "rfd":
        d = gdc.rfd_divergence(o, Y, q, ufl, calV, step)
    dx = o.susp.fcm.grid.dx
    dd, dnu = np.zeros_like(d), 0.0
    for sh in [(1, 0, 0), (0, 1, 0), (0, 0, 1)]:
        Y1 = Y + np.asarray(sh) * dx
        u1 = np.roll(ufl, sh, axis=(1, 2, 3))
        c1, d1 = gdc.predictor(o, Y1, q, u1)
        if divergence == "rfd":
            d1 = gdc.rfd_divergence(o, Y1, q, u1, c1, step)
        dd = np.maximum(dd, np.abs(d1 - d))
        dnu = max(dnu, 0.5 * o.dt * abs(float(np.sum(d1 - d))))
    floor = 1e-14 * max(1.0, float(np.abs(d).max()))
    return safety * np.maximum(dd, floor), safety * max(dnu, 0.5 * o.dt * floor)


def max_rel(a, b):
    """Element-wise error relative to the reference's scale: max |a - b| / max |b|."""
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    m = np.abs(b).max() if b.size else 0.0
    return float(np.abs(a - b).max() / (m if m > 0 else 1.0)) if b.size else 0.0


def check_close(what, got, ref, tol, elem_tol=None):
    """Relative L2 over the whole vector within tol, and every element within
    elem_tol (default 4 tol) of the reference's largest magnitude, so that a
    few bad entries cannot hide in a long vector.  Prints both figures."""
    e2, em = rel_l2(got, ref), max_rel(got, ref)
    et = 4.0 * tol if elem_tol is None else elem_tol
    print(f"[err] {what}: rel L2 {e2:.3e} (tol {tol:.1e}), element max {em:.3e} (tol {et:.1e})", flush=True)
    assert e2 < tol, (what, e2, tol)
    assert em < et, (what, em, et)
    return e2, em
