"""Throughput of the gDC step on one MI355X: blob-steps/s with p50/p99 step
latency, on the largest suspension that fits one GPU: 32,768 rods of 10
blobs (327,680 blobs), L = 384a, grid 384^3, axes within 15 degrees of z,
background shear 0.1 and harmonic pair repulsion, dt = 0.005, FP32 grid with
FP64 body algebra and Krylov vectors.

One step is the whole hot path: stress noise and the random velocity field,
the least-squares velocity and the finite-difference drift factor, the
midpoint move, pair forces, the full saddle solve by GMRES, and the update.
Inputs stay resident in HBM (device tensors) for the timed region.

"At 1e-5 relative mobility error": the GMRES tolerance is the loosest of a
ladder (eight rungs per decade) whose FP32 body-mobility solve, on the first
state with a probe force F ~ N(0, 1) per body, stays within 1e-5 (relative
L2) of a reference solve: the library's FP64 path at 1e-12 for the 384^3
suspension (whose FP32 first step is parity-tested against the FP64 oracle
at full size), the FP64 oracle's own solve (1e-10) wherever the oracle fits
in the run (the 1,000-rod suspension and the serving buckets).

Beside the headline figure the JSON line carries:
  roofline      the step's dominant kernel (at 384^3 the inverse axis-1 pass of
                the five-pass 3D transform) against HBM peak, duration
                measured live with dispatch-stamped events on its launch
                stream;
  kernels       achieved bandwidth of spreading, averaging and each FFT pass;
  fp64_single   the same suspension on the plain FP64 path;
  rods1000      the 1,000-rod suspension (128^3), calibrated against the
                oracle, with its own roofline (inverse plane pass);
  rheology      effective viscosity of 500 rods under the sinusoidal forcing;
  serving       256 independent suspensions (N log-uniform in [8, 2048] rods,
                grids 32^3..128^3, 50 steps each) served with continuous
                batching, each grid bucket at its own calibrated tolerance:
                saturation throughput (GMRES iterations of the 32^3
                suspensions fused, the rest on concurrent streams; also all
                on streams and all fused), a Poisson sweep with p50/p99 step
                latency, and the same requests one at a time on the plain
                FP64 and FP32 paths (a sample of 16);
  cpu_baseline  the FP64 oracle on a bounded sample of the headline
                suspension (one full-size mobility apply), scaled to
                blob-steps/s.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
                       [--no-serving] [--no-extras] [--workload NAME]
       python bench.py --fusion-table   (fused against streamed batching per grid)
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "blob-steps/sec of gDC step at 1e-5 rel mobility error; p50/p99 step latency"
HBM_PEAK_GBS = 8000.0
TARGET_ERR = 1e-5

# Dominant kernel of each workload's step (largest share of GPU time in its
# kernel trace) as (probe family, kernel, algorithmic bytes per launch from G
# grid points and M blobs).  At 384^3 it is the inverse axis-1 pass of the
# five-pass transform (three half spectra of G/2 complex FP32 values read
# and written once, 24 G bytes), once per GMRES iteration and once per step
# in the noise field's transform, which gives it a slightly larger share of
# the step than the projection pass (FFT along axis 0, Stokes projection,
# inverse FFT along axis 0, also 24 G), a little longer per launch.  At 256^3 the C2R pass moves the same 24 G; at 128^3 the inverse
# plane pass of the three-pass transform reads the three half spectra and
# writes the three real components, 24 G as well.
DOMINANT = {
    "rods1000": ("fft_plane_inv", "k_plane_inv", lambda G, M: 24 * G),
    "mixed4096": ("fft_c2r", "k_c2r_axis2", lambda G, M: 24 * G),
    "rods32768": ("fft_inv1", "k_inv_axis1", lambda G, M: 24 * G),
}
# Spreading, for the kernel table: the FP32 force field written once
# (3 components x 4 B per grid point) plus, per blob, its sorted stencil
# record (32 B) and its force (3 x 8 B).
BYTES_PER_POINT = 12
BYTES_PER_BLOB = 56


def working_launches(each_ms):
    """Split probed launches into those that did the work and those that
    returned at the solver's done flag: the solver queues GMRES iteration
    k + 1 before it has read the convergence test of iteration k, so one
    launch per solve reads the flag and exits (a few microseconds against
    hundreds).  A launch is counted as working if it took at least a tenth
    of the 90th-percentile duration.  Returns (count, total ms, early-exit
    count)."""
    import numpy as np
    d = np.asarray(each_ms, dtype=np.float64)
    if d.size == 0:
        return 0, 0.0, 0
    full = d >= 0.1 * np.percentile(d, 90)
    return int(full.sum()), float(d[full].sum()), int((~full).sum())

# HBM traffic of each workload's dominant kernel per launch from two
# rocprofv3 --pmc runs of this script (FETCH_SIZE, then WRITE_SIZE, KiB per
# dispatch, averaged over the dispatches of the instantiation the timed
# region runs that did work), each scaled by the 256 MiB copy that
# --copy-calibration adds (FETCH_SIZE x 2.0, WRITE_SIZE x 1.0).  Read +
# written bytes:
#   rods1000   k_plane_inv       24,477,771 + 25,165,824
#   mixed4096  k_c2r_axis2      201,495,749 + 201,326,592 (two blocks per workgroup, 256 threads)
#   rods32768  k_inv_axis1      679,681,496 + 679,477,248 (two tiles per workgroup, 512 threads)
# A workload's entry goes back to None whenever its kernel changes, until
# the counters are taken again.
TRAFFIC_BYTES = {"rods1000": 49643595, "mixed4096": 402822341, "rods32768": 1359158744}

WORKLOAD_TEXT = {
    "rods1000": "rods1000: 1,000 rods x 10 blobs (10,000 blobs), L=128a, grid 128^3, FP32 grid / FP64 bodies "
                "and Krylov, harmonic pair repulsion 2.2a, dt=0.005",
    "mixed4096": "mixed4096: 1,366 rods(10) + 1,365 boomerangs(15) + 1,365 tetrahedra(4) (39,595 blobs), "
                 "L=256a, grid 256^3, FP32 grid / FP64 bodies, force e_z on every body, dt=0.005",
    "rods32768": "rods32768: 32,768 rods x 10 blobs (327,680 blobs), L=384a, grid 384^3, axes within 15 deg "
                 "of z, shear 0.1 + harmonic pair repulsion, FP32 grid / FP64 bodies and Krylov, dt=0.005",
}

SERVING_BUDGET = 32 << 30
SERVING_SLOTS = 16
LADDER = [float(f"{1e-3 * 10 ** (-k / 8):.2g}") for k in range(33)]   # 1e-3 .. 1e-7, ratio 10^(1/8)


def progress(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def probe_force(w):
    import numpy as np
    return np.random.default_rng(1234).standard_normal((w.N, 6))


def reference_body(g, wl, w, Y0, q0, source):
    """V = N F for the probe force: the FP64 oracle's saddle solve (GMRES to
    1e-10) or the library's FP64 path (GMRES to 1e-12)."""
    import numpy as np
    F = probe_force(w)
    if source == "oracle":
        from oracle import fcm, rigid
        fcm.DEFAULT_WORKERS = len(os.sched_getaffinity(0))
        p = fcm.FcmParams(fcm.Grid(w.L, w.n), w.eta, w.sigma, w.rc)
        susp = rigid.Suspension(p, rigid.Bodies(w.shapes, w.body_shape), w.a)
        r = rigid.blob_positions(susp.bodies, Y0, q0)
        _, V, _ = rigid.solve_saddle(susp, Y0, r, np.zeros((w.M, 3)), F, tol=1e-10)
        return V
    ref = g.Suspension(**wl.library_kwargs(w, precision="fp64", gmres_tol=1e-12, gmres_maxit=1000))
    V = ref.mobility_apply("body", Y0, q0, F)
    ref.close()
    return V


def body_error(g, wl, w, Y0, q0, Vref, tol, precision="fp32"):
    import numpy as np
    s = g.Suspension(**wl.library_kwargs(w, precision=precision, gmres_tol=tol, gmres_maxit=500))
    V = s.mobility_apply("body", Y0, q0, probe_force(w), allow_notconv=True)
    s.close()
    return float(np.linalg.norm(V - Vref) / np.linalg.norm(Vref))


def calibrate(g, wl, cases, target=TARGET_ERR):
    """The loosest ladder tolerance at which every case's FP32 body solve is
    within target of its reference.  cases: [(workload, Y0, q0, Vref)].
    Returns (tol, [error per case])."""
    for tol in LADDER:
        errs = []
        for (w, Y0, q0, Vref) in cases:
            errs.append(body_error(g, wl, w, Y0, q0, Vref, tol))
            if errs[-1] > target:
                break
        if len(errs) == len(cases) and max(errs) <= target:
            return tol, errs
    raise RuntimeError("no GMRES tolerance reaches the target mobility error")


def cpu_baseline(w, Y0, q0, gpu_iterations):
    """The FP64 oracle, as it stands, on a bounded sample of the same
    suspension: one application of its FCM mobility J L^-1 S at the full
    size (weights of all blobs, spreading, the 3D FFT solve, averaging), the
    unit of work of every GMRES iteration.  A step needs at least
    (GMRES iterations + 1) such applies (the +1 is the random-field solve),
    so blob-steps/s is bounded above by M / ((k + 1) t_apply); the oracle's
    averages, least-squares and preconditioner work are not counted."""
    import numpy as np
    from oracle import fcm, rigid
    cores = len(os.sched_getaffinity(0))
    fcm.DEFAULT_WORKERS = cores
    p = fcm.FcmParams(fcm.Grid(w.L, w.n), w.eta, w.sigma, w.rc)
    r = rigid.blob_positions(rigid.Bodies(w.shapes, w.body_shape), Y0, q0)
    lam = np.random.default_rng(7).standard_normal((w.M, 3))
    t0 = time.perf_counter()
    fcm.mobility_apply(r, lam, p)
    t_apply = time.perf_counter() - t0
    applies = float(gpu_iterations) + 1.0
    return {"value": w.M / (applies * t_apply), "unit": "blob-steps/s", "cores": cores, "kind": "oracle",
            "sample": f"one FP64 oracle mobility apply J L^-1 S on the full {w.name} suspension "
                      f"({w.M:,} blobs, grid {w.n[0]}^3): {t_apply:.1f} s on {cores} threads, scaled to a step "
                      f"of {applies:.1f} applies (the GPU's mean GMRES iterations + the random-field solve); "
                      f"an upper bound on the oracle's rate"}


def oracle_timings(wl, tol):
    """The oracle, as it stands, on the measurement configurations: seconds per
    step and blob-steps/s with all host threads, and with one thread for the
    two smallest.  1,000-rod and 4,096-body suspensions: first 3 steps; 8-rod
    suspension: 100 steps (10 on one thread); serving: the first 3 steps of 8
    requests (the smallest, the largest, 6 evenly spaced).  The 32,768-rod
    suspension is left out: at over 20 oracle minutes per step its first
    steps do not fit a bounded run."""
    import numpy as np
    from oracle import fcm, gdc, rigid
    cores = len(os.sched_getaffinity(0))

    def run(w, n_steps, workers, tol_w):
        fcm.DEFAULT_WORKERS = workers
        p = fcm.FcmParams(fcm.Grid(w.L, w.n), w.eta, w.sigma, w.rc)
        cfg = gdc.Config(rigid.Suspension(p, rigid.Bodies(w.shapes, w.body_shape), w.a), w.kT, w.dt,
                         w.noise_seed, gdc.Forces(w.steric_k, w.steric_cutoff,
                                                  np.asarray(w.const_force, dtype=np.float64), w.shear_rate,
                                                  w.sine_force))
        Y, q = wl.initial_state(w)
        t0 = time.perf_counter()
        for k in range(n_steps):
            Y, q, _ = gdc.gdc_step(cfg, Y, q, k, tol=tol_w)
        dt = time.perf_counter() - t0
        progress(f"oracle {w.name}: {n_steps} steps on {workers} threads, {dt:.1f} s")
        return {"steps": n_steps, "threads": workers, "s_per_step": dt / n_steps, "blob_steps_per_s": w.M * n_steps / dt}

    out = {"host_threads": cores, "gmres_tol": tol}
    c1 = wl.rods8()
    out["rods8"] = run(c1, 100, cores, tol)
    out["rods8_one_thread"] = run(c1, 10, 1, tol)
    c2 = wl.rods1000("fp64")
    out["rods1000"] = run(c2, 3, cores, tol)
    out["rods1000_one_thread"] = run(c2, 1, 1, tol)
    out["mixed4096"] = run(wl.mixed4096(), 3, cores, tol)
    reqs = wl.serving_requests(256)
    order = np.argsort([w.M for w in reqs])
    pick = sorted(set([int(order[0]), int(order[-1])] + [int(order[i]) for i in np.linspace(0, len(order) - 1, 8)[1:-1].astype(int)]))[:8]
    blob_steps, secs = 0, 0.0
    for i in pick:
        r = run(reqs[i], 3, cores, tol)
        blob_steps += reqs[i].M * 3
        secs += r["s_per_step"] * 3
    out["serving_sample"] = {"requests": len(pick), "steps_each": 3, "blob_steps_per_s": blob_steps / secs}
    return out


def grid_coverage(w, Y, q):
    """Fraction of grid points within the envelope cutoff of some blob (the
    part of the field an averaging pass must read)."""
    import numpy as np
    from workloads import _rodrigues_many
    n = np.asarray(w.n)
    L = np.asarray(w.L)
    dx = L / n
    ang = 2.0 * np.arccos(np.clip(q[:, 0], -1.0, 1.0))
    s = np.sin(ang / 2)
    axis = np.where(s[:, None] > 1e-15, q[:, 1:] / np.where(s[:, None] > 1e-15, s[:, None], 1.0),
                    np.array([0.0, 0.0, 1.0]))
    r = np.concatenate([Y[p] + _rodrigues_many(axis[p:p + 1], ang[p:p + 1],
                                               np.asarray(w.shapes[w.body_shape[p]]))[0]
                        for p in range(w.N)])
    mark = np.zeros(tuple(n), bool)
    P = np.ceil(w.rc / dx).astype(int)
    offs = np.stack(np.meshgrid(*[np.arange(-P[d], P[d] + 1) for d in range(3)], indexing="ij"), -1).reshape(-1, 3)
    base = np.floor(r / dx).astype(np.int64)
    for k in range(0, len(r), 2000):
        g = base[k:k + 2000, None, :] + offs[None, :, :]
        d = g * dx - r[k:k + 2000, None, :]
        inside = (d * d).sum(-1) <= w.rc * w.rc
        gi = np.mod(g[inside], n)
        mark[gi[:, 0], gi[:, 1], gi[:, 2]] = True
    return float(mark.mean())


def timed_steps(g, s, Y, q, steps, warmup):
    """Time `steps` steps as one library call (the steps are pipelined on the
    stream); per-step latencies are the gaps between consecutive completion
    times in the handle's step log within that call (steps - 1 of them)."""
    import numpy as np
    import torch
    if warmup:
        s.step(Y, q, warmup)
    torch.cuda.synchronize()
    s.step_log()   # drop earlier entries; the last completion stays as the origin
    t_start = time.perf_counter()
    st = s.step(Y, q, steps)
    torch.cuda.synchronize()
    total = time.perf_counter() - t_start
    log = np.asarray(s.step_log())
    # gaps between consecutive completions inside the timed call; the first
    # entry is the warm-up call's last completion, so the first gap would
    # also hold the host's time between the two calls
    lat = np.diff(log)[1:]
    if len(lat) != steps - 1:
        raise RuntimeError(f"step log holds {len(lat) + 1} latencies for {steps} steps")
    return total, lat, st["gmres_iterations_mean"], st


def kernel_bandwidth(g, s, Y, q, w, cov):
    """Average duration and achieved algorithmic bandwidth of each grid
    kernel family over 4 steps (dispatch-stamped HIP events on the launch
    stream)."""
    G = int(w.G)
    fams = {
        "spread": ("k_spread_tab", BYTES_PER_POINT * G + BYTES_PER_BLOB * w.M),
        "interp": ("k_interp", int(12 * cov * G) + 48 * w.M),
    }
    if max(w.n) <= 128:   # three-pass plane transforms
        fams.update({"fft_plane_fwd": ("k_plane_fwd", 24 * G), "fft_project": ("k_axis0_plane", 24 * G),
                     "fft_plane_inv": ("k_plane_inv", 24 * G)})
    else:                 # five-pass line transforms
        fams.update({"fft_r2c": ("k_r2c_axis2", 24 * G), "fft_fwd1": ("k_fwd_axis1", 24 * G),
                     "fft_project": ("k_axis0_project", 24 * G), "fft_inv1": ("k_inv_axis1", 24 * G),
                     "fft_c2r": ("k_c2r_axis2", 24 * G)})
    out = {}
    for fam, (kname, nbytes) in fams.items():
        g.probe_kernel(fam)
        s.step(Y, q, 4)
        _, _, each = g.probe_read(each=True)
        g.probe_kernel(None)
        n, ms, early = working_launches(each)
        if n == 0:
            continue
        avg = ms * 1e-3 / n
        gbs = nbytes / avg / 1e9
        out[fam] = {"kernel": kname, "launches": n, "early_exits": early, "avg_us": avg * 1e6,
                    "algorithmic_bytes": nbytes, "achieved_GBs": gbs, "frac": gbs / HBM_PEAK_GBS}
    return out


def time_workload(g, wl, name, w, Y0, q0, tol, stream, steps, warmup):
    """Times `steps` steps of workload w at GMRES tolerance tol (after
    `warmup`), with the dominant kernel probed over the timed region."""
    import numpy as np
    import torch
    s = g.Suspension(**wl.library_kwargs(w, gmres_tol=tol, gmres_maxit=500, stream=stream.cuda_stream))
    Y = torch.tensor(Y0, dtype=torch.float64, device="cuda")
    q = torch.tensor(q0, dtype=torch.float64, device="cuda")
    if warmup:
        s.step(Y, q, warmup)
    torch.cuda.synchronize()
    fam, kname, nbytes = DOMINANT[name]
    g.probe_kernel(fam)
    total, lat_ms, its, st = timed_steps(g, s, Y, q, steps, 0)
    if len(lat_ms) == 0:   # one timed step: its latency is the call's time
        lat_ms = np.array([total * 1e3])
    _, _, each = g.probe_read(each=True)
    g.probe_kernel(None)
    k_launches, k_ms, k_early = working_launches(each)
    G = int(np.prod(w.n))
    alg_bytes = nbytes(G, w.M)
    avg_s = k_ms * 1e-3 / max(k_launches, 1)
    achieved = alg_bytes / avg_s / 1e9
    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": TRAFFIC_BYTES.get(name),
                "kernel": kname, "launches": k_launches, "early_exits": k_early, "avg_us": avg_s * 1e6,
                "algorithmic_bytes": alg_bytes}
    # the whole step against the byte model of the method's grid traffic:
    # G (60 + 72 k) bytes per FP32 step with k operator applies (GMRES
    # iterations), each 3D transform counted once read and once written
    step_bytes = G * (60.0 + 72.0 * float(its))
    step_gbs = step_bytes / (total / steps) / 1e9
    res = {
        "value": w.M * steps / total, "ms_per_step": total * 1e3 / steps, "gmres_iterations_mean": float(its),
        "p50_ms": float(np.percentile(lat_ms, 50)), "p99_ms": float(np.percentile(lat_ms, 99)),
        "nu_mean": st["nu_mean"], "nu_std": st["nu_std"], "nu_min": st["nu_min"], "nu_max": st["nu_max"],
        "nu_nonpositive": st["nu_nonpositive"],
        "fft_passes": 3 if (max(w.n) <= 128 and w.n[1] == w.n[2]) else 5,
        "fft_workgroup_sizes": s.launch_config,
        "roofline": roofline,
        "step_roofline": {"model": "G (60 + 72 k) bytes per step, k = mean GMRES iterations",
                          "bytes_per_step": step_bytes, "achieved": step_gbs, "peak": HBM_PEAK_GBS,
                          "unit": "GB/s", "frac": step_gbs / HBM_PEAK_GBS},
    }
    return s, Y, q, res


def fp64_single(g, wl, w, Y0, q0, tol, stream, steps):
    """The plain FP64 path on the same suspension at the same tolerance."""
    import torch
    progress("plain FP64 path")
    s64 = g.Suspension(**wl.library_kwargs(w, precision="fp64", gmres_tol=tol, gmres_maxit=500,
                                           stream=stream.cuda_stream))
    Y64 = torch.tensor(Y0, dtype=torch.float64, device="cuda")
    q64 = torch.tensor(q0, dtype=torch.float64, device="cuda")
    t64, _, its64, _ = timed_steps(g, s64, Y64, q64, steps, 1)
    s64.close()
    return {"blob_steps_per_s": w.M * steps / t64, "ms_per_step": t64 * 1e3 / steps, "steps": steps,
            "gmres_iterations_mean": float(its64)}


def rheology_bench(g, wl, tol, stream, steps=100):
    """Effective viscosity under the sinusoidal forcing f0 sin(k y) e_x:
    eta_eff = f0 / (k^2 v_x), v_x the per-step sine amplitude of the fluid
    x-velocity averaged over the run (Sec. 6.4)."""
    import numpy as np
    import torch
    progress("rheology")
    w = wl.rheology500()
    Y0, q0 = wl.initial_state(w)
    s = g.Suspension(**wl.library_kwargs(w, gmres_tol=tol, gmres_maxit=500, stream=stream.cuda_stream))
    Y = torch.tensor(Y0, dtype=torch.float64, device="cuda")
    q = torch.tensor(q0, dtype=torch.float64, device="cuda")
    s.step(Y, q, 5)
    torch.cuda.synchronize()
    vx = []
    t0 = time.perf_counter()
    for _ in range(steps):
        vx.append(s.step(Y, q, 1)["sine_vx"])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    s.close()
    vx = np.array(vx)
    k = 2.0 * np.pi / w.L[1]
    ratio = w.sine_force / (k * k * vx.mean()) / w.eta
    se = vx.std(ddof=1) / np.sqrt(len(vx)) / vx.mean() * ratio
    return {"workload": "rheology500: 500 rods x 10 blobs (5,000 blobs, 8% volume fraction), L=64a, grid 64^3, "
                        f"f0={w.sine_force:g}, k=2pi/L, dt={w.dt:g}, pair repulsion, FP32",
            "steps": steps, "blob_steps_per_s": w.M * steps / dt,
            "v_x_mean": float(vx.mean()), "eta_eff_over_eta": float(ratio), "eta_eff_over_eta_se": float(se),
            "shear_rate": float(k * vx.mean()),
            "note": "v_x from each step's midpoint solve; a short run from a random start, not a converged "
                    "rheology measurement"}


def serving_bench(g, wl, reqs, states, budget, slots):
    """Continuous batching of the serving stream.  Each grid bucket
    (32^3 .. 128^3) runs at its own tolerance: the loosest ladder rung at
    which the bucket's smallest and largest requests both solve the body
    mobility within 1e-5 of the FP64 oracle."""
    import numpy as np
    from paper_2106_00449_amd.serving import LibraryExecutor, Request, Server, summarise

    buckets = sorted(set(int(w.n[0]) for w in reqs))
    tols, bucket_err = {}, {}
    for n in buckets:
        idx = [i for i, w in enumerate(reqs) if w.n[0] == n]
        pick = sorted(set([min(idx, key=lambda i: reqs[i].M), max(idx, key=lambda i: reqs[i].M)]))
        progress(f"serving: calibrating the {n}^3 bucket on requests {pick}")
        cases = [(reqs[i], *states[i], reference_body(g, wl, reqs[i], *states[i], "oracle")) for i in pick]
        tol, errs = calibrate(g, wl, cases)
        tols[n] = tol
        bucket_err[f"{n}^3"] = {"gmres_tol": tol, "requests": len(idx),
                                "calibrated_on": [{"request": int(i), "bodies": reqs[i].N, "rel_err": e}
                                                  for i, e in zip(pick, errs)]}

    def requests(rate):
        out = []
        for i, (w, (Y, q)) in enumerate(zip(reqs, states)):
            arr = w.extra["arrival"] / rate if rate else 0.0
            out.append(Request(i, wl.library_kwargs(w, gmres_tol=tols[w.n[0]], gmres_maxit=500), Y, q, w.steps,
                               arr, blobs=w.M))
        return out

    progress("serving: saturation run (GMRES iterations of the 32^3 suspensions fused)")
    srv = Server(hbm_budget=budget, max_slots=slots)
    t0 = time.perf_counter()
    res = srv.run(requests(None))
    sat = summarise(res, makespan=time.perf_counter() - t0)
    sat.update(peak_bytes=srv.peak_bytes, peak_slots=srv.peak_slots, fused_grids="32^3")
    sat_fused = {}
    for key, fusion in (("none", False), ("all", True)):
        progress(f"serving: saturation run, GMRES iterations fused over the resident suspensions: {key}")
        srv = Server(hbm_budget=budget, max_slots=slots, executor=LibraryExecutor(fusion=fusion))
        t0 = time.perf_counter()
        res = srv.run(requests(None))
        sat_fused[key] = summarise(res, makespan=time.perf_counter() - t0)
        sat_fused[key].update(peak_bytes=srv.peak_bytes, peak_slots=srv.peak_slots)
    rate = len(reqs) / sat["makespan_s"]
    sweep = {}
    for f in (0.5, 1.0, 2.0):
        progress(f"serving: Poisson run at {f * rate:.1f} requests/s ({f:g}x saturation)")
        srv = Server(hbm_budget=budget, max_slots=slots)
        res = srv.run(requests(f * rate))
        summ = summarise(res)
        summ.update(arrival_rate_per_s=f * rate, peak_bytes=srv.peak_bytes, peak_slots=srv.peak_slots)
        sweep[f"{f:g}x"] = summ

    # one at a time on the plain paths, same requests (a sample)
    order = np.argsort([w.M for w in reqs])
    sample = order[:: max(1, len(order) // 16)][:16]
    seq = {}
    for prec in ["fp64", "fp32"]:
        progress(f"serving: sequential {prec} sample")
        blob_steps, t_tot, lat = 0, 0.0, []
        for i in sample:
            w = reqs[i]
            Y, q = (x.copy() for x in states[i])
            s = g.Suspension(**wl.library_kwargs(w, precision=prec, gmres_tol=tols[w.n[0]], gmres_maxit=500))
            s.step(Y, q, 1)
            t0 = time.perf_counter()
            for _ in range(w.steps):
                t1 = time.perf_counter()
                s.step(Y, q, 1)
                lat.append(time.perf_counter() - t1)
            t_tot += time.perf_counter() - t0
            blob_steps += w.M * w.steps
            s.close()
        lat = np.array(lat) * 1e3
        seq[prec] = {"blob_steps_per_s": blob_steps / t_tot, "requests": len(sample),
                     "step_latency_p50_ms": float(np.percentile(lat, 50)),
                     "step_latency_p99_ms": float(np.percentile(lat, 99))}
    return {
        "workload": f"{len(reqs)} suspensions of N rods x 10 blobs, N log-uniform in [8, 2048] "
                    f"({sum(w.M for w in reqs):,} blobs), 5% blob volume fraction, grids "
                    f"{min(w.n[0] for w in reqs)}^3..{max(w.n[0] for w in reqs)}^3, 50 gDC steps each, FP32",
        "tolerance_per_bucket": bucket_err,
        "hbm_budget_bytes": budget, "max_slots": slots,
        "saturation": sat, "saturation_streams": sat_fused["none"], "saturation_fused": sat_fused["all"],
        "poisson_at_saturation_rate": sweep["1x"], "poisson_rate_sweep": sweep,
        "sequential_fp64_sample": seq["fp64"], "sequential_fp32_sample": seq["fp32"],
        "served_over_sequential_fp64": sat["blob_steps_per_s"] / seq["fp64"]["blob_steps_per_s"],
    }


def fusion_table(g, wl, reps=2, warm=4, steps=6, tol=1e-5):
    """Fused GMRES iterations against concurrent streams, per serving grid
    bucket: batch_step over the first K requests of the bucket (all of one
    grid size), `steps` timed steps after `warm`, each setting in turn and
    in alternating order over `reps` repetitions."""
    import numpy as np
    reqs = wl.serving_requests()
    out = []
    for rep in range(reps):
        for K, n in [(24, 32), (24, 48), (16, 64), (8, 96), (8, 128)]:
            ws = [w for w in reqs if w.n[0] == n][:K]
            for fusion in ((False, True) if rep % 2 == 0 else (True, False)):
                ss = []
                for w in ws:
                    Y, q = wl.initial_state(w)
                    s = g.Suspension(**wl.library_kwargs(w, gmres_tol=tol, gmres_maxit=400))
                    s.fusion = fusion
                    s.set_state(Y, q)
                    ss.append(s)
                g.batch_step(ss, [warm] * len(ss))
                t0 = time.perf_counter()
                _, stats, _ = g.batch_step(ss, [steps] * len(ss))
                dt = time.perf_counter() - t0
                blobs = sum(w.M for w in ws)
                row = {"rep": rep, "grid": n, "suspensions": len(ws), "blobs": blobs, "fused": fusion,
                       "ms": dt * 1e3, "blob_steps_per_s": blobs * steps / dt,
                       "fused_iterations": int(sum(x["fused_iterations"] for x in stats))}
                progress(f"fusion table: {row}")
                out.append(row)
                for s in ss:
                    s.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="headline only: no kernel table, FP64 path, 1,000-rod object or rheology")
    ap.add_argument("--only-headline", action="store_true",
                    help="same as --no-extras --no-serving --no-cpu-baseline")
    ap.add_argument("--serving-requests", type=int, default=256)
    ap.add_argument("--serving-slots", type=int, default=SERVING_SLOTS)
    ap.add_argument("--gmres-tol", type=float, default=0.0,
                    help="use this GMRES tolerance instead of calibrating one (profiling runs)")
    ap.add_argument("--workload", default="rods32768", choices=["rods32768", "rods1000", "mixed4096"],
                    help="suspension of the headline figure (default: the largest, 384^3)")
    ap.add_argument("--oracle-timings", action="store_true",
                    help="time the oracle on every measurement configuration instead (host only, ~20 min; "
                         "no GPU work)")
    ap.add_argument("--kernel-table", action="store_true",
                    help="with --only-headline, still measure the per-kernel bandwidth table")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one 256 MiB device copy first (counter calibration for profiling)")
    ap.add_argument("--no-graphs", action="store_true",
                    help="launch every GMRES iteration kernel by kernel (no HIP graph replay)")
    ap.add_argument("--fusion-table", action="store_true",
                    help="instead: fused GMRES iterations against concurrent streams per serving grid bucket")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(its sharding is a design, not code); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.only_headline:
        args.no_extras = args.no_serving = args.no_cpu_baseline = True

    import numpy as np
    import workloads as wl

    if args.oracle_timings:
        tol = args.gmres_tol if args.gmres_tol > 0.0 else 1e-5
        print(json.dumps({"oracle_timings": oracle_timings(wl, tol)}))
        return
    if args.fusion_table:
        import paper_2106_00449_amd as g
        g.GRAPHS_DEFAULT = not args.no_graphs
        print(json.dumps({"fusion_table": fusion_table(g, wl)}))
        return

    # initial states first, in worker processes, before anything touches the GPU
    make = {"rods1000": lambda: wl.rods1000("fp32"), "mixed4096": wl.mixed4096, "rods32768": wl.rods32768}
    w = make[args.workload]()
    Y0, q0 = wl.initial_state(w)
    c2 = None
    if not args.no_extras and args.workload != "rods1000":
        c2 = wl.rods1000("fp32")
        Y2, q2 = wl.initial_state(c2)
    reqs, states = [], []
    if not args.no_serving:
        reqs = wl.serving_requests(args.serving_requests)
        states = wl.initial_states(reqs)
    cov = grid_coverage(w, Y0, q0)

    import torch
    import paper_2106_00449_amd as g

    g.GRAPHS_DEFAULT = not args.no_graphs
    if args.copy_calibration:
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    source = "oracle" if args.workload == "rods1000" else "fp64"
    if args.gmres_tol > 0.0:
        tol, err = args.gmres_tol, None
    else:
        progress(f"calibrating the GMRES tolerance against the {source} reference")
        tol, errs = calibrate(g, wl, [(w, Y0, q0, reference_body(g, wl, w, Y0, q0, source))])
        err = errs[0]
    progress(f"tolerance {tol:g}; timing {args.steps} steps of {w.name}")
    stream = torch.cuda.current_stream()
    s, Y, q, head = time_workload(g, wl, args.workload, w, Y0, q0, tol, stream, args.steps, args.warmup)
    kernels = {}
    if not args.no_extras or args.kernel_table:
        progress("kernel bandwidths")
        kernels = kernel_bandwidth(g, s, Y, q, w, cov)
    s.close()

    out = {
        "metric": METRIC, "value": head["value"], "unit": "blob-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": head["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": WORKLOAD_TEXT[args.workload],
                   "gmres_tol": tol, "mobility_rel_err": err,
                   "mobility_reference": {"oracle": "FP64 oracle saddle solve (GMRES 1e-10)",
                                          "fp64": "the library's FP64 path (GMRES 1e-12)"}[source],
                   "gmres_iterations_mean": head["gmres_iterations_mean"],
                   "p50_ms": head["p50_ms"], "p99_ms": head["p99_ms"],
                   "nu_mean": head["nu_mean"], "nu_std": head["nu_std"], "nu_min": head["nu_min"],
                   "nu_max": head["nu_max"], "nu_nonpositive_steps": head["nu_nonpositive"],
                   "interp_grid_coverage": cov, "fft_passes": head["fft_passes"],
                   "fft_workgroup_sizes": head["fft_workgroup_sizes"],
                   "gmres_iteration_graphs": g.GRAPHS_DEFAULT},
        "roofline": head["roofline"],
        "step_roofline": head["step_roofline"],
        "kernels": kernels,
    }
    if not args.no_extras:
        out["fp64_single"] = fp64_single(g, wl, w, Y0, q0, tol, stream, max(5, args.steps // 4))
        if c2 is not None:
            progress("1,000-rod suspension: calibrating against the oracle")
            tol2, errs2 = calibrate(g, wl, [(c2, Y2, q2, reference_body(g, wl, c2, Y2, q2, "oracle"))])
            s2, _, _, r2 = time_workload(g, wl, "rods1000", c2, Y2, q2, tol2, stream, 30, 3)
            s2.close()
            r2.update(workload=WORKLOAD_TEXT["rods1000"], gmres_tol=tol2, mobility_rel_err=errs2[0],
                      mobility_reference="FP64 oracle saddle solve (GMRES 1e-10)")
            out["rods1000"] = r2
        out["rheology"] = rheology_bench(g, wl, 1e-5, stream)
    if reqs:
        progress(f"serving {len(reqs)} requests")
        out["serving"] = serving_bench(g, wl, reqs, states, SERVING_BUDGET, args.serving_slots)
    if not args.no_cpu_baseline:
        progress("oracle on the host")
        out["cpu_baseline"] = cpu_baseline(w, Y0, q0, head["gmres_iterations_mean"])
    print(json.dumps(out))


if __name__ == "__main__":
    main()
