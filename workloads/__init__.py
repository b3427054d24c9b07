"""Seeded synthetic inputs shared by the tests, the oracle runs and the bench.

This module only builds inputs: body shapes (body-frame blob offsets),
suspension parameters, and non-overlapping initial positions and
orientations.  It holds none of the method's arithmetic (no mobility, no
noise of the method, no time stepping); the placement check rotates blob
offsets with its own axis-angle (Rodrigues) routine, used for nothing else.
Both the HIP library and the oracle recompute blob positions themselves.

Workloads (sizes of the five suspensions the paper's method is exercised on):
  rods8        8 rods x 5 blobs, L = 32a, grid 48^3, dt = 0.01, no forces, FP64
  rods1000     1,000 rods x 10 blobs, L = 128a, grid 128^3, dt = 0.005,
               harmonic blob-pair repulsion (cutoff 2.2a)
  mixed4096    1,366 rods(10) + 1,365 boomerangs(15) + 1,365 tetrahedra(4),
               L = 256a, grid 256^3, constant force e_z on every body
  serving      256 requests of N rods (10 blobs), N log-uniform in [8, 2048],
               box at 5% blob volume fraction, grid from {32,48,64,96,128}
  rods32768    32,768 rods x 10 blobs, L = 384a, grid 384^3, axes within 15
               degrees of z, shear rate 0.1 plus the pair repulsion
  rheology500  500 rods x 10 blobs, L = 64a, grid 64^3, sinusoidal forcing
               f0 sin(2 pi y / L) e_x of the fluid (effective viscosity)
Common: a = 1, eta = 1/(6 pi), kT = 1, sigma = a/sqrt(pi), cutoff 3a.
"""

from dataclasses import dataclass, field
import math

import numpy as np

A = 1.0
ETA = 1.0 / (6.0 * math.pi)
KT = 1.0
SIGMA = A / math.sqrt(math.pi)


# ------------------------------------------------------------------ shapes

def _centred(b):
    b = np.asarray(b, dtype=np.float64)
    return b - b.mean(axis=0)


def rod(n_blobs, spacing=2.0 * A):
    """Straight rod of collinear blobs along the body z axis."""
    return _centred([[0.0, 0.0, spacing * i] for i in range(n_blobs)])


def boomerang(spacing=A):
    """L-shaped boomerang: a corner blob plus 7 blobs along each of the body
    x and y axes at the given spacing (15 blobs, two 8-blob arms)."""
    pts = [[0.0, 0.0, 0.0]]
    pts += [[spacing * i, 0.0, 0.0] for i in range(1, 8)]
    pts += [[0.0, spacing * i, 0.0] for i in range(1, 8)]
    return _centred(pts)


def tetrahedron(edge=2.0 * A):
    """Regular tetrahedron of 4 blobs with the given edge length."""
    s = edge / (2.0 * math.sqrt(2.0))
    return _centred([[s, s, s], [s, -s, -s], [-s, s, -s], [-s, -s, s]])


# ------------------------------------------------------------------ configs

@dataclass
class Workload:
    name: str
    L: tuple
    n: tuple
    shapes: list
    body_shape: np.ndarray
    dt: float
    steps: int
    noise_seed: int
    placement_seed: int
    precision: str = "fp32"
    a: float = A
    sigma: float = SIGMA
    rc: float = 3.0 * A
    eta: float = ETA
    kT: float = KT
    steric_k: float = 0.0
    steric_cutoff: float = 0.0
    const_force: tuple = (0.0, 0.0, 0.0, 0.0, 0.0, 0.0)
    shear_rate: float = 0.0
    sine_force: float = 0.0          # f0 of the rheology forcing f0 sin(2 pi y / L_y) e_x
    channel: bool = False            # slip walls at y = 0 and y = L_y/2 (images in the upper half)
    wall_k: float = 0.0              # blob-wall harmonic repulsion of the channel
    wall_cutoff: float = 0.0
    nematic_cap_deg: float = 0.0     # 0: orientations uniform on S^3
    placement: str = "sequential"    # or "batch" (see initial_state)
    extra: dict = field(default_factory=dict)

    @property
    def N(self):
        return int(len(self.body_shape))

    @property
    def M(self):
        return int(sum(len(self.shapes[s]) for s in self.body_shape))

    @property
    def G(self):
        return int(np.prod(self.n))


def _steric():
    b = 2.2 * A
    return dict(steric_k=40.0 * KT / (A * b), steric_cutoff=b)


def rods8():
    return Workload("rods8", (32.0,) * 3, (48,) * 3, [rod(5)], np.zeros(8, np.int64),
                    dt=0.01, steps=100, noise_seed=0, placement_seed=1000, precision="fp64")


def rods1000(precision="fp32"):
    return Workload("rods1000", (128.0,) * 3, (128,) * 3, [rod(10)], np.zeros(1000, np.int64),
                    dt=0.005, steps=1000, noise_seed=2, placement_seed=1002,
                    precision=precision, **_steric())


def mixed4096():
    body_shape = np.concatenate([np.zeros(1366, np.int64), np.ones(1365, np.int64),
                                 np.full(1365, 2, np.int64)])
    return Workload("mixed4096", (256.0,) * 3, (256,) * 3,
                    [rod(10), boomerang(), tetrahedron()], body_shape,
                    dt=0.005, steps=100, noise_seed=3, placement_seed=1003,
                    const_force=(0.0, 0.0, 1.0, 0.0, 0.0, 0.0), placement="batch")


def rods32768(steric=True):
    kw = _steric() if steric else {}
    return Workload("rods32768", (384.0,) * 3, (384,) * 3, [rod(10)],
                    np.zeros(32768, np.int64), dt=0.005, steps=10000, noise_seed=5,
                    placement_seed=1005, shear_rate=0.1, nematic_cap_deg=15.0, placement="batch", **kw)


def rheology500(sine_force=0.002):
    """Sinusoidal-forcing rheology: 500 rods x 10 blobs (8% blob volume
    fraction), L = 64a, grid 64^3, fluid forced by f0 sin(2 pi y / L) e_x;
    the paper's suspension (Sec. 6.4) is the same forcing on a denser box of
    19-blob particles whose geometry the text does not give."""
    return Workload("rheology500", (64.0,) * 3, (64,) * 3, [rod(10)], np.zeros(500, np.int64),
                    dt=0.005, steps=200, noise_seed=6, placement_seed=1006, sine_force=sine_force,
                    placement="batch", **_steric())


def small_case(name="tiny", n_bodies=4, n=16, L=16.0, shapes=None, body_shape=None,
               precision="fp64", seed=7, **kw):
    """Small suspensions for parity tests (oracle runs in seconds)."""
    shapes = shapes if shapes is not None else [rod(3)]
    if body_shape is None:
        body_shape = np.arange(n_bodies) % len(shapes)
    Ls = tuple(L) if isinstance(L, (tuple, list)) else (float(L),) * 3
    ns = tuple(n) if isinstance(n, (tuple, list)) else (int(n),) * 3
    return Workload(name, Ls, ns, shapes, np.asarray(body_shape, np.int64), dt=kw.pop("dt", 0.01),
                    steps=kw.pop("steps", 3), noise_seed=seed, placement_seed=seed + 1000,
                    precision=precision, **kw)


def serving_requests(n_requests=256, seed=4):
    """The serving stream: N log-uniform in [8, 2048] rods of 10 blobs, box at
    5% volume fraction, grid the smallest of {32,48,64,96,128} >= L/a,
    50 steps, noise seed = request index, Poisson arrivals at unit rate."""
    rng = np.random.default_rng(seed)
    grids = [32, 48, 64, 96, 128]
    out = []
    t = 0.0
    for r in range(n_requests):
        N = int(round(math.exp(rng.uniform(math.log(8), math.log(2048)))))
        L = (10 * N * (4.0 / 3.0) * math.pi * A ** 3 / 0.05) ** (1.0 / 3.0)
        n = next(g for g in grids if g >= L / A)
        t += rng.exponential(1.0)
        w = Workload(f"req{r}", (L,) * 3, (n,) * 3, [rod(10)], np.zeros(N, np.int64),
                     dt=0.005, steps=50, noise_seed=r, placement_seed=10000 + r, placement="batch")
        w.extra["arrival"] = t
        out.append(w)
    return out


# ------------------------------------------------------- initial placement

def _rodrigues(axis, angle, v):
    """Rotate vectors v (k, 3) about the unit axis by angle (right hand)."""
    c, s = math.cos(angle), math.sin(angle)
    return v * c + np.cross(axis, v) * s + np.outer(v @ axis, axis) * (1.0 - c)


def _random_orientation(rng, cap_deg):
    """(quaternion, axis, angle).  cap_deg = 0: uniform on S^3 (normalised
    four normals); otherwise the body z axis uniform in the cap of half-angle
    cap_deg about the lab z axis (no spin: rods are symmetric about it)."""
    if cap_deg <= 0.0:
        q = rng.standard_normal(4)
        q /= np.linalg.norm(q)
        if q[0] < 0:
            q = -q
        angle = 2.0 * math.acos(min(1.0, q[0]))
        v = q[1:]
        nv = np.linalg.norm(v)
        axis = v / nv if nv > 0 else np.array([0.0, 0.0, 1.0])
        return q, axis, angle
    cmin = math.cos(math.radians(cap_deg))
    ct = rng.uniform(cmin, 1.0)
    phi = rng.uniform(0.0, 2.0 * math.pi)
    e = np.array([math.sqrt(1 - ct * ct) * math.cos(phi), math.sqrt(1 - ct * ct) * math.sin(phi), ct])
    axis = np.cross([0.0, 0.0, 1.0], e)
    na = np.linalg.norm(axis)
    angle = math.acos(ct)
    axis = axis / na if na > 1e-15 else np.array([1.0, 0.0, 0.0])
    q = np.concatenate([[math.cos(angle / 2)], math.sin(angle / 2) * axis])
    return q, axis, angle


def initial_state(w: Workload, min_dist=2.0 * A, max_tries=2000):
    """Centres uniform in the box, orientations as described, no blob within
    min_dist (minimum image) of a blob of another body.  Returns Y (N, 3) and
    q (N, 4), FP64.

    placement "sequential": bodies are placed one after the other, each
    redrawn until it clears every body placed before it.  "batch": all bodies
    are drawn at once, then every body that overlaps a lower-numbered one is
    redrawn, until none overlaps (vectorised; for the large suspensions)."""
    if w.placement == "batch":
        return _batch_placement(w, min_dist, max_tries)
    rng = np.random.default_rng(w.placement_seed)
    L = np.asarray(w.L, dtype=np.float64)
    cell = max(min_dist, 1e-9)
    nc = np.maximum((L // cell).astype(int), 1)
    bins = {}
    Y = np.zeros((w.N, 3))
    Q = np.zeros((w.N, 4))

    def key(p):
        return tuple((np.floor(p / (L / nc)).astype(int)) % nc)

    for p in range(w.N):
        b = w.shapes[w.body_shape[p]]
        for _ in range(max_tries):
            c = rng.uniform(0.0, 1.0, 3) * L
            q, axis, angle = _random_orientation(rng, w.nematic_cap_deg)
            pts = c + _rodrigues(axis, angle, b)
            ok = True
            for x in pts:
                k = key(x - L * np.floor(x / L))
                for dk in np.ndindex(3, 3, 3):
                    kk = tuple((np.array(k) + np.array(dk) - 1) % nc)
                    for y in bins.get(kk, ()):
                        d = x - y
                        d -= L * np.round(d / L)
                        if d @ d < min_dist * min_dist:
                            ok = False
                            break
                    if not ok:
                        break
                if not ok:
                    break
            if ok:
                break
        else:
            raise RuntimeError(f"could not place body {p} of {w.name}")
        Y[p], Q[p] = c, q
        for x in pts:
            xw = x - L * np.floor(x / L)
            bins.setdefault(key(xw), []).append(xw)
    return Y, Q


def _draw_bodies(rng, k, L, cap_deg):
    """k centres uniform in the box and k orientations: quaternions (k, 4)
    and the matching (axis, angle) pairs."""
    c = rng.uniform(0.0, 1.0, (k, 3)) * L
    if cap_deg <= 0.0:
        q = rng.standard_normal((k, 4))
        q /= np.linalg.norm(q, axis=1, keepdims=True)
        q[q[:, 0] < 0] *= -1.0
        angle = 2.0 * np.arccos(np.minimum(1.0, q[:, 0]))
        nv = np.linalg.norm(q[:, 1:], axis=1, keepdims=True)
        axis = np.where(nv > 0, q[:, 1:] / np.where(nv > 0, nv, 1.0), np.array([0.0, 0.0, 1.0]))
    else:
        cmin = math.cos(math.radians(cap_deg))
        ct = rng.uniform(cmin, 1.0, k)
        phi = rng.uniform(0.0, 2.0 * math.pi, k)
        st = np.sqrt(1.0 - ct * ct)
        e = np.stack([st * np.cos(phi), st * np.sin(phi), ct], axis=1)
        axis = np.cross(np.array([0.0, 0.0, 1.0]), e)
        na = np.linalg.norm(axis, axis=1, keepdims=True)
        angle = np.arccos(ct)
        axis = np.where(na > 1e-15, axis / np.where(na > 1e-15, na, 1.0), np.array([1.0, 0.0, 0.0]))
        q = np.concatenate([np.cos(angle / 2)[:, None], np.sin(angle / 2)[:, None] * axis], axis=1)
    return c, q, axis, angle


def _rodrigues_many(axis, angle, b):
    """Rotate the body-frame offsets b (nb, 3) of k bodies: (k, nb, 3)."""
    c = np.cos(angle)[:, None, None]
    s = np.sin(angle)[:, None, None]
    ax = axis[:, None, :]
    v = b[None, :, :]
    return v * c + np.cross(ax, v) * s + (v @ axis[:, :, None]) * ax * (1.0 - c)


def _close_pairs(p, ref, L, nc, min_dist):
    """Index pairs (i, j) with p[i] within min_dist of ref[j] (minimum image),
    found through a cell list of ref (cells of at least min_dist)."""
    def cells(x):
        w = x - L * np.floor(x / L)
        c = np.minimum((w / (L / nc)).astype(np.int64), nc - 1)
        return w, c
    pw, pc = cells(p)
    rw, rc = cells(ref)
    rid = (rc[:, 0] * nc[1] + rc[:, 1]) * nc[2] + rc[:, 2]
    order = np.argsort(rid, kind="stable")
    srid = rid[order]
    out_i, out_j = [], []
    for d in np.ndindex(3, 3, 3):
        nb = (pc + np.array(d) - 1) % nc
        nid = (nb[:, 0] * nc[1] + nb[:, 1]) * nc[2] + nb[:, 2]
        lo = np.searchsorted(srid, nid, "left")
        hi = np.searchsorted(srid, nid, "right")
        k = lo[:, None] + np.arange(max(int((hi - lo).max(initial=0)), 1))[None, :]
        ok = k < hi[:, None]
        cj = order[np.minimum(np.where(ok, k, 0), len(order) - 1)]
        dv = pw[:, None, :] - rw[cj]
        dv -= L * np.round(dv / L)
        close = ok & (np.einsum("ijk,ijk->ij", dv, dv) < min_dist * min_dist)
        i, jj = np.nonzero(close)
        out_i.append(i)
        out_j.append(cj[i, jj])
    return np.concatenate(out_i), np.concatenate(out_j)


def _batch_placement(w, min_dist, max_rounds):
    rng = np.random.default_rng(w.placement_seed)
    L = np.asarray(w.L, dtype=np.float64)
    N = w.N
    nc = np.maximum((L // max(min_dist, 1e-9)).astype(int), 1)
    if np.any(nc < 3):
        raise ValueError("batch placement needs a box of at least three cells per axis")
    bshape = np.asarray(w.body_shape)
    nbs = np.array([len(w.shapes[s]) for s in bshape])
    off = np.concatenate([[0], np.cumsum(nbs)])
    blob_body = np.repeat(np.arange(N), nbs)
    Y = np.zeros((N, 3))
    Q = np.zeros((N, 4))
    pos = np.zeros((int(off[-1]), 3))
    todo = np.arange(N)
    for _ in range(max_rounds):
        for s in np.unique(bshape[todo]):
            grp = todo[bshape[todo] == s]
            nb = len(w.shapes[s])
            c, q, axis, angle = _draw_bodies(rng, len(grp), L, w.nematic_cap_deg)
            Y[grp], Q[grp] = c, q
            idx = off[grp][:, None] + np.arange(nb)[None, :]
            pos[idx.ravel()] = (c[:, None, :] + _rodrigues_many(axis, angle, np.asarray(w.shapes[s]))).reshape(-1, 3)
        # a drawn body that overlaps a kept body, or a lower-numbered drawn
        # body, is drawn again (kept bodies never move)
        drawn = np.zeros(N, bool)
        drawn[todo] = True
        rows = np.nonzero(drawn[blob_body])[0]
        i, j = _close_pairs(pos[rows], pos, L, nc, min_dist)
        bi, bj = blob_body[rows[i]], blob_body[j]
        hit = (bi != bj) & (~drawn[bj] | (bj < bi))
        todo = np.unique(bi[hit])
        if todo.size == 0:
            return Y, Q
    raise RuntimeError(f"could not place the bodies of {w.name}")


def initial_states(ws, processes=None):
    """initial_state of each workload, computed in worker processes (fork;
    call it before the process touches a GPU)."""
    import multiprocessing as mp
    import os
    n = processes or min(16, len(os.sched_getaffinity(0)))
    if n <= 1 or len(ws) <= 1:
        return [initial_state(w) for w in ws]
    with mp.get_context("fork").Pool(n) as pool:
        return pool.map(initial_state, ws, chunksize=1)


def library_kwargs(w: Workload, **over):
    """Keyword arguments of paper_2106_00449_amd.Suspension for a workload."""
    kw = dict(L=w.L, n=w.n, shapes=w.shapes, body_shape=w.body_shape, a=w.a, sigma=w.sigma,
              trunc=w.rc, eta=w.eta, kT=w.kT, dt=w.dt, precision=w.precision, seed=w.noise_seed,
              steric_k=w.steric_k, steric_cutoff=w.steric_cutoff, const_force=w.const_force,
              shear_rate=w.shear_rate, sine_force=w.sine_force, channel=w.channel, wall_k=w.wall_k,
              wall_cutoff=w.wall_cutoff)
    kw.update(over)
    return kw
