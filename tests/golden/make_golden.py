"""Writes the oracle's first gDC step of a full-size workload to a JSON
fixture under tests/golden/, for the GPU parity tests at sizes the oracle
cannot run inside a test.

It calls only the oracle (FP64, written from the paper) and the seeded input
generators; nothing here touches the HIP library.  Stored, for step 0 from
the workload's seeded initial state (noise seed of the workload):
  * nu of the step (Sec. 3, step 3) and the sum of the per-body terms d_p;
  * for a fixed sample of bodies (evenly spaced body indices): calV_p
    (eq. sol_unconst), d_p (eq. FD), the increment Y^{n+1} - Y^n and
    q^{n+1} - q^n, and the midpoint velocity V^m of step 5;
  * whole-vector norms and maxima of the increments and of calV (the scales
    the element-wise bounds of the tests are relative to);
  * the oracle's GMRES iterations and residual, and a digest of the initial
    state so that the test knows it starts from the same one.

Usage: python tests/golden/make_golden.py mixed4096 [--tol 1e-10] [--sample 512]
       python tests/golden/make_golden.py rods32768
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import workloads as wl  # noqa: E402
from oracle import fcm, gdc, rigid  # noqa: E402


def state_digest(Y, q):
    return hashlib.sha256(np.ascontiguousarray(Y).tobytes() + np.ascontiguousarray(q).tobytes()).hexdigest()


def sample_bodies(N, k):
    return np.unique(np.linspace(0, N - 1, k).astype(np.int64))


def oracle_config(w):
    p = fcm.FcmParams(fcm.Grid(w.L, w.n), w.eta, w.sigma, w.rc)
    s = rigid.Suspension(p, rigid.Bodies(w.shapes, w.body_shape), w.a)
    F = gdc.Forces(w.steric_k, w.steric_cutoff, np.asarray(w.const_force, dtype=np.float64), w.shear_rate,
                   w.sine_force)
    return gdc.Config(s, w.kT, w.dt, w.noise_seed, F)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("workload", choices=["mixed4096", "rods32768"])
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--sample", type=int, default=512)
    ap.add_argument("--workers", type=int, default=len(os.sched_getaffinity(0)))
    args = ap.parse_args()
    w = {"mixed4096": wl.mixed4096, "rods32768": wl.rods32768}[args.workload]()
    fcm.DEFAULT_WORKERS = args.workers
    Y0, q0 = wl.initial_state(w)
    cfg = oracle_config(w)
    t0 = time.time()
    Y1, q1, info = gdc.gdc_step(cfg, Y0, q0, 0, tol=args.tol)
    secs = time.time() - t0
    dY, dq = Y1 - Y0, q1 - q0
    idx = sample_bodies(w.N, args.sample)
    out = {
        "what": f"oracle gDC step 0 of {w.name} from its seeded initial state (FP64, GMRES tol {args.tol:g})",
        "workload": w.name, "N": w.N, "M": w.M, "n": list(w.n), "step": 0,
        "state_sha256": state_digest(Y0, q0),
        "gmres_tol": args.tol, "gmres_iterations": int(info["iterations"]), "gmres_relres": float(info["relres"]),
        "oracle_seconds": secs, "workers": args.workers,
        "nu": float(info["nu"]), "d_sum": float(np.sum(info["d"])),
        "norm_dY": float(np.linalg.norm(dY)), "norm_dq": float(np.linalg.norm(dq)),
        "max_dY": float(np.abs(dY).max()), "max_dq": float(np.abs(dq).max()),
        "max_calV_t": float(np.abs(info["calV"][:, :3]).max()), "max_calV_r": float(np.abs(info["calV"][:, 3:]).max()),
        "max_d": float(np.abs(info["d"]).max()),
        "max_V_t": float(np.abs(info["V"][:, :3]).max()), "max_V_r": float(np.abs(info["V"][:, 3:]).max()),
        "bodies": idx.tolist(),
        "calV": info["calV"][idx].tolist(), "d": info["d"][idx].tolist(),
        "dY": dY[idx].tolist(), "dq": dq[idx].tolist(), "V": info["V"][idx].tolist(),
    }
    path = os.path.join(HERE, f"step0_{w.name}.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=0)
    print(f"wrote {path}: nu {out['nu']:.10f}, {out['gmres_iterations']} GMRES iterations, {secs:.0f} s")


if __name__ == "__main__":
    main()
