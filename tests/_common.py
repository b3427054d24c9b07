"""Shared test helpers: a workload as an oracle configuration or a library
handle, relative errors, and the GPU-availability gate."""
import numpy as np

import workloads as wl
from oracle import fcm, gdc, rigid


def oracle_config(w: wl.Workload, kT=None, dt=None, divergence="fd", fd_delta=1e-6):
    p = fcm.FcmParams(fcm.Grid(w.L, w.n), w.eta, w.sigma, w.rc)
    s = rigid.Suspension(p, rigid.Bodies(w.shapes, w.body_shape), w.a)
    F = gdc.Forces(w.steric_k, w.steric_cutoff, np.asarray(w.const_force, dtype=np.float64), w.shear_rate,
                   w.sine_force)
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


def fd_nu_roundoff_bound(o, info, divergence="fd", safety=16.0):
    """Bound on the rounding error of the oracle's drift factor nu.

    The oracle forms each forward difference calV(x + delta e) - calV(x) in FP64
    with delta = 1e-6, so every quotient carries about
    2 eps sqrt(n) |calV| / delta_k of rounding (n = stencil points summed per
    blob average, delta_k = delta L_p for translations and delta for
    rotations); nu sums 6 such quotients per body, times dt/2.  RFD weights
    each quotient by |W~| (<~ 3)."""
    calV = np.asarray(info["calV"])
    b = o.susp.bodies
    grid = o.susp.fcm.grid
    npts = (4.0 / 3.0) * np.pi * (o.susp.fcm.rc ** 3) / grid.dV
    eps = np.finfo(np.float64).eps
    tot = 0.0
    for p in range(b.N):
        Lp = gdc.body_length(b.shapes[b.body_shape[p]], o.susp.a)
        per = 2.0 * eps * np.sqrt(npts) * np.abs(calV[p]).max()
        tot += per * (3.0 / (o.fd_delta * Lp) + 3.0 / o.fd_delta) * (3.0 if divergence == "rfd" else 1.0)
    return safety * 0.5 * o.dt * tot
