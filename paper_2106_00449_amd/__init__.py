"""Python binding of libgdc, the MI355X (gfx950) HIP library for the
generalised drift-correcting (gDC) Brownian-dynamics step of rigid multiblob
particles with fluctuating FCM hydrodynamics (arXiv 2106.00449).

Argument marshalling only: every step of the method runs in the library's
HIP kernels behind the C ABI of include/gdc.h.  Arrays may be NumPy arrays
(host memory; the library copies) or CUDA/HIP torch tensors (device memory,
used in place on the handle's stream).  There is no CPU fallback: if the
library is missing, importing this module raises.
"""

import ctypes
import os

import numpy as np

__all__ = ["Suspension", "GdcError", "LIB_PATH", "lib", "batch_step", "footprint",
           "GDC_FP32", "GDC_FP64", "GDC_BLOB", "GDC_BODY",
           "GDC_SCHEME_GDC", "GDC_SCHEME_EM", "GDC_DIV_FD", "GDC_DIV_RFD"]

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libgdc.so")

GDC_OK, GDC_EINVAL, GDC_ENOMEM, GDC_ENOTCONV, GDC_ENUMERIC, GDC_EDEVICE = 0, -1, -2, -3, -4, -5
GDC_FP32, GDC_FP64 = 0, 1
GDC_HOST, GDC_DEVICE = 0, 1
GDC_BLOB, GDC_BODY = 0, 1
GDC_SCHEME_GDC, GDC_SCHEME_EM = 0, 1
GDC_DIV_FD, GDC_DIV_RFD = 0, 1
GDC_UNTIL_ALL, GDC_UNTIL_ANY = 0, 1

_NAMES = {GDC_EINVAL: "GDC_EINVAL", GDC_ENOMEM: "GDC_ENOMEM", GDC_ENOTCONV: "GDC_ENOTCONV",
          GDC_ENUMERIC: "GDC_ENUMERIC", GDC_EDEVICE: "GDC_EDEVICE"}


class GdcError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_NAMES.get(code, code)}: {msg}")
        self.code = code


class _Shape(ctypes.Structure):
    _fields_ = [("n_blobs", ctypes.c_int), ("b", ctypes.POINTER(ctypes.c_double))]


class _Forces(ctypes.Structure):
    _fields_ = [("steric_k", ctypes.c_double), ("steric_cutoff", ctypes.c_double),
                ("const_force", ctypes.c_double * 6), ("shear_rate", ctypes.c_double),
                ("sine_force", ctypes.c_double), ("wall_k", ctypes.c_double), ("wall_cutoff", ctypes.c_double)]


class _Config(ctypes.Structure):
    _fields_ = [("L", ctypes.c_double * 3), ("n", ctypes.c_int * 3),
                ("a", ctypes.c_double), ("sigma", ctypes.c_double), ("trunc", ctypes.c_double),
                ("eta", ctypes.c_double), ("kT", ctypes.c_double), ("dt", ctypes.c_double),
                ("fd_delta", ctypes.c_double), ("gmres_tol", ctypes.c_double),
                ("gmres_maxit", ctypes.c_int), ("gmres_restart", ctypes.c_int),
                ("precision", ctypes.c_int), ("scheme", ctypes.c_int), ("divergence", ctypes.c_int),
                ("channel", ctypes.c_int),
                ("seed", ctypes.c_uint64),
                ("n_shapes", ctypes.c_int), ("shapes", ctypes.POINTER(_Shape)),
                ("n_bodies", ctypes.c_int), ("body_shape", ctypes.POINTER(ctypes.c_int)),
                ("forces", _Forces), ("device", ctypes.c_int), ("stream", ctypes.c_void_p)]


class _Stats(ctypes.Structure):
    _fields_ = [("steps_done", ctypes.c_int), ("gmres_iterations", ctypes.c_int),
                ("gmres_relres", ctypes.c_double), ("nu", ctypes.c_double),
                ("nu_nonpositive", ctypes.c_int), ("ms", ctypes.c_double),
                ("sine_vx", ctypes.c_double), ("gmres_iterations_mean", ctypes.c_double),
                ("nu_mean", ctypes.c_double), ("nu_std", ctypes.c_double), ("nu_min", ctypes.c_double),
                ("nu_max", ctypes.c_double), ("status", ctypes.c_int), ("fused_iterations", ctypes.c_int)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_2106_00449_amd.build` (hipcc, gfx950)")
    L = ctypes.CDLL(LIB_PATH)
    P, D, I, U64, U32 = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_int, ctypes.c_uint64, ctypes.c_uint32
    L.gdc_init.argtypes = [ctypes.POINTER(_Config), ctypes.POINTER(P)]
    L.gdc_free.argtypes = [P]
    L.gdc_free.restype = None
    L.gdc_last_error.restype = ctypes.c_char_p
    L.gdc_mobility_apply.argtypes = [P, I, P, P, P, P, I]
    L.gdc_step.argtypes = [P, I, P, P, I, ctypes.POINTER(_Stats)]
    L.gdc_get_step.argtypes = [P, ctypes.POINTER(U64)]
    L.gdc_set_step.argtypes = [P, U64]
    L.gdc_fluct_velocity.argtypes = [P, U64, P, I]
    L.gdc_predictor.argtypes = [P, P, P, U64, P, P, I]
    L.gdc_philox_normals.argtypes = [P, U64, U32, U64, U32, I, D]
    L.gdc_philox_normals_noalloc.argtypes = [P, U64, U32, U64, U32, I, D]
    L.gdc_probe_kernel.argtypes = [ctypes.c_char_p]
    L.gdc_probe_read.argtypes = [D, ctypes.POINTER(ctypes.c_longlong), ctypes.POINTER(ctypes.c_float),
                                 ctypes.c_longlong]
    L.gdc_set_state.argtypes = [P, P, P, I]
    L.gdc_get_state.argtypes = [P, P, P, I]
    L.gdc_batch_step.argtypes = [ctypes.POINTER(P), I, ctypes.POINTER(I), I, ctypes.c_double,
                                 ctypes.POINTER(_Stats)]
    L.gdc_step_log.argtypes = [P, D, I, ctypes.POINTER(I)]
    L.gdc_footprint.argtypes = [ctypes.POINTER(_Config), ctypes.POINTER(ctypes.c_size_t)]
    L.gdc_device_bytes.argtypes = [P, ctypes.POINTER(ctypes.c_size_t)]
    L.gdc_get_launch_config.argtypes = [P, ctypes.POINTER(I), I]
    L.gdc_set_graphs.argtypes = [P, I]
    L.gdc_get_graphs.argtypes = [P, ctypes.POINTER(I)]
    L.gdc_set_fusion.argtypes = [P, I]
    L.gdc_get_fusion.argtypes = [P, ctypes.POINTER(I)]
    L.gdc_set_launch_config.argtypes = [P, ctypes.POINTER(I), I]
    for name in ["gdc_init", "gdc_mobility_apply", "gdc_step", "gdc_get_step", "gdc_set_step",
                 "gdc_fluct_velocity", "gdc_predictor", "gdc_philox_normals", "gdc_philox_normals_noalloc",
                 "gdc_probe_kernel",
                 "gdc_probe_read", "gdc_set_state", "gdc_get_state", "gdc_batch_step", "gdc_step_log",
                 "gdc_footprint", "gdc_device_bytes",
                 "gdc_get_launch_config", "gdc_set_launch_config", "gdc_set_graphs", "gdc_get_graphs",
                 "gdc_set_fusion", "gdc_get_fusion"]:
        getattr(L, name).restype = ctypes.c_int
    return L


lib = _load()


def _check(rc):
    if rc != GDC_OK:
        raise GdcError(rc, lib.gdc_last_error().decode())


def _is_torch(x):
    return type(x).__module__.startswith("torch")


class _Arg:
    """Marshals one array argument: host NumPy (copied to contiguous FP64) or
    a device torch tensor (FP64, contiguous, used in place)."""

    def __init__(self, x, shape, writable=False):
        self.torch = _is_torch(x)
        if self.torch:
            if x.dtype.__str__() != "torch.float64" or not x.is_contiguous() or not x.is_cuda:
                raise TypeError("device arrays must be contiguous float64 torch tensors on the GPU")
            if tuple(x.shape) != tuple(shape):
                raise ValueError(f"expected shape {shape}, got {tuple(x.shape)}")
            self.arr = x
            self.ptr = ctypes.c_void_p(x.data_ptr())
        else:
            a = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
            if a.shape != tuple(shape):
                a = a.reshape(shape)
            self.arr = a
            self.ptr = a.ctypes.data_as(ctypes.c_void_p)

    @property
    def memspace(self):
        return GDC_DEVICE if self.torch else GDC_HOST


def _memspace(*args):
    ms = {a.memspace for a in args}
    if len(ms) != 1:
        raise TypeError("mix of host and device arrays in one call")
    return ms.pop()


def probe_kernel(family):
    """Time every later launch of one kernel family with HIP events."""
    _check(lib.gdc_probe_kernel(family.encode() if family else None))


PROBE_CAPACITY = 8192


def probe_read(each=False):
    """(total ms, launches) of the probed family since the last read; with
    each=True also the per-launch durations (ms, launch order)."""
    ms = ctypes.c_double()
    n = ctypes.c_longlong()
    buf = (ctypes.c_float * PROBE_CAPACITY)() if each else None
    _check(lib.gdc_probe_read(ctypes.byref(ms), ctypes.byref(n), buf, PROBE_CAPACITY if each else 0))
    if not each:
        return ms.value, n.value
    return ms.value, n.value, np.array(buf[:min(n.value, PROBE_CAPACITY)], dtype=np.float64)


def _make_config(L, n, shapes, body_shape, *, a=1.0, sigma=0.0, trunc=0.0,
                 eta=1.0 / (6.0 * np.pi), kT=1.0, dt=0.01, fd_delta=0.0, gmres_tol=0.0,
                 gmres_maxit=0, gmres_restart=0, precision="fp32", scheme="gdc",
                 divergence="fd", seed=0, steric_k=0.0, steric_cutoff=0.0,
                 const_force=(0, 0, 0, 0, 0, 0), shear_rate=0.0, sine_force=0.0, channel=False, wall_k=0.0,
                 wall_cutoff=0.0, device=0, stream=None):
    """A gdc_config and the arrays it points into (kept alive by the caller).
    channel=True: the slip channel (walls at y = 0 and y = L[1]/2)."""
    shape_arrays = [np.ascontiguousarray(np.asarray(s, dtype=np.float64).reshape(-1, 3)) for s in shapes]
    bshape = np.ascontiguousarray(np.asarray(body_shape, dtype=np.int32))
    sh = (_Shape * len(shapes))()
    for i, s in enumerate(shape_arrays):
        sh[i].n_blobs = s.shape[0]
        sh[i].b = s.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    c = _Config()
    Ls = np.broadcast_to(np.asarray(L, dtype=np.float64), (3,))
    ns = np.broadcast_to(np.asarray(n, dtype=np.int64), (3,))
    for d in range(3):
        c.L[d] = float(Ls[d])
        c.n[d] = int(ns[d])
    c.a, c.sigma, c.trunc, c.eta, c.kT, c.dt = a, sigma, trunc, eta, kT, dt
    c.fd_delta, c.gmres_tol, c.gmres_maxit, c.gmres_restart = fd_delta, gmres_tol, gmres_maxit, gmres_restart
    c.precision = {"fp32": GDC_FP32, "fp64": GDC_FP64}[precision]
    c.scheme = {"gdc": GDC_SCHEME_GDC, "em": GDC_SCHEME_EM}[scheme]
    c.divergence = {"fd": GDC_DIV_FD, "rfd": GDC_DIV_RFD}[divergence]
    c.channel = 1 if channel else 0
    c.seed = int(seed)
    c.n_shapes = len(shapes)
    c.shapes = ctypes.cast(sh, ctypes.POINTER(_Shape))
    c.n_bodies = int(bshape.size)
    c.body_shape = bshape.ctypes.data_as(ctypes.POINTER(ctypes.c_int))
    c.forces.steric_k, c.forces.steric_cutoff = steric_k, steric_cutoff
    for k in range(6):
        c.forces.const_force[k] = float(const_force[k])
    c.forces.shear_rate = shear_rate
    c.forces.sine_force = sine_force
    c.forces.wall_k, c.forces.wall_cutoff = wall_k, wall_cutoff
    c.device = int(device)
    c.stream = stream
    keep = {"shapes": shape_arrays, "body_shape": bshape, "shapes_c": sh, "N": int(bshape.size),
            "M": int(sum(shape_arrays[s].shape[0] for s in bshape)), "n": tuple(int(x) for x in ns)}
    return c, keep


def footprint(L, n, shapes, body_shape, **kw):
    """Device bytes a Suspension with these arguments would hold (no device
    is touched)."""
    c, keep = _make_config(L, n, shapes, body_shape, **kw)
    b = ctypes.c_size_t()
    _check(lib.gdc_footprint(ctypes.byref(c), ctypes.byref(b)))
    return int(b.value)


def batch_step(susps, steps, until="all", max_ms=0.0):
    """Advance resident suspensions together (gdc_batch_step).

    steps: steps still to take per suspension.  Returns (steps left,
    per-suspension statistics, return code).  A suspension's own outcome is
    its statistics' "status" (GDC_OK, GDC_ENOTCONV or GDC_ENUMERIC), so the
    step errors of one suspension are returned, not raised; argument and
    device errors raise."""
    nh = len(susps)
    hs = (ctypes.c_void_p * max(nh, 1))(*[s._h for s in susps])
    st_in = (ctypes.c_int * max(nh, 1))(*[int(x) for x in steps])
    stats = (_Stats * max(nh, 1))()
    rc = lib.gdc_batch_step(hs, nh, st_in, {"all": GDC_UNTIL_ALL, "any": GDC_UNTIL_ANY}[until],
                            float(max_ms), stats)
    if rc not in (GDC_OK, GDC_ENOTCONV, GDC_ENUMERIC):
        _check(rc)
    out = [{"steps_done": x.steps_done, "gmres_iterations": x.gmres_iterations,
            "gmres_relres": x.gmres_relres, "nu": x.nu, "nu_nonpositive": x.nu_nonpositive,
            "ms": x.ms, "sine_vx": x.sine_vx, "gmres_iterations_mean": x.gmres_iterations_mean,
            "nu_mean": x.nu_mean, "nu_std": x.nu_std, "nu_min": x.nu_min, "nu_max": x.nu_max,
            "status": x.status, "fused_iterations": x.fused_iterations}
           for x in stats[:nh]]
    return [int(x) for x in st_in[:nh]], out, rc


# whether new suspensions replay GMRES iterations from HIP graphs
GRAPHS_DEFAULT = True


class Suspension:
    """A suspension of rigid multiblob bodies in a periodic box on one GPU.

    shapes: list of (n_b, 3) body-frame blob offsets; body_shape: (N,) ints.
    graphs: replay GMRES iterations from captured HIP graphs (None: the
    module's GRAPHS_DEFAULT).  Remaining keyword arguments follow gdc_config
    (include/gdc.h)."""

    def __init__(self, L, n, shapes, body_shape, graphs=None, **kw):
        c, keep = _make_config(L, n, shapes, body_shape, **kw)
        self._keep = keep
        self._cfg = c
        self.N = keep["N"]
        self.M = keep["M"]
        self.n = keep["n"]
        self.precision = kw.get("precision", "fp32")
        h = ctypes.c_void_p()
        _check(lib.gdc_init(ctypes.byref(c), ctypes.byref(h)))
        self._h = h
        on = GRAPHS_DEFAULT if graphs is None else graphs
        if not on:
            self.graphs = False

    def close(self):
        if getattr(self, "_h", None):
            lib.gdc_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # --------------------------------------------------------------- calls
    def mobility_apply(self, mode, Y, q, x, out=None, allow_notconv=False):
        """mode "blob": M_FCM lambda (M x 3); mode "body": N F (N x 6)."""
        m = {"blob": GDC_BLOB, "body": GDC_BODY}[mode]
        shp = (self.M, 3) if m == GDC_BLOB else (self.N, 6)
        aY, aq, ax = _Arg(Y, (self.N, 3)), _Arg(q, (self.N, 4)), _Arg(x, shp)
        ms = _memspace(aY, aq, ax)
        if out is None:
            if ms == GDC_DEVICE:
                import torch
                out = torch.empty(shp, dtype=torch.float64, device=ax.arr.device)
            else:
                out = np.empty(shp)
        ao = _Arg(out, shp, writable=True)
        rc = lib.gdc_mobility_apply(self._h, m, aY.ptr, aq.ptr, ax.ptr, ao.ptr, ms)
        if not (allow_notconv and rc == GDC_ENOTCONV):
            _check(rc)
        return out

    def step(self, Y, q, n_steps=1):
        """Advances Y (N x 3) and q (N x 4) in place; returns the statistics."""
        if not _is_torch(Y):
            if not (isinstance(Y, np.ndarray) and Y.dtype == np.float64 and Y.flags.c_contiguous
                    and isinstance(q, np.ndarray) and q.dtype == np.float64 and q.flags.c_contiguous):
                raise TypeError("step updates Y and q in place: pass contiguous float64 arrays")
        aY, aq = _Arg(Y, (self.N, 3), True), _Arg(q, (self.N, 4), True)
        ms = _memspace(aY, aq)
        st = _Stats()
        rc = lib.gdc_step(self._h, int(n_steps), aY.ptr, aq.ptr, ms, ctypes.byref(st))
        stats = {"steps_done": st.steps_done, "gmres_iterations": st.gmres_iterations,
                 "gmres_relres": st.gmres_relres, "nu": st.nu, "nu_nonpositive": st.nu_nonpositive,
                 "ms": st.ms, "sine_vx": st.sine_vx, "gmres_iterations_mean": st.gmres_iterations_mean,
                 "nu_mean": st.nu_mean, "nu_std": st.nu_std, "nu_min": st.nu_min, "nu_max": st.nu_max,
                 "rc": rc}
        if rc != GDC_ENOTCONV:
            _check(rc)
        return stats

    def set_state(self, Y, q):
        """Make (Y, q) the resident state (for batch_step)."""
        aY, aq = _Arg(Y, (self.N, 3)), _Arg(q, (self.N, 4))
        _check(lib.gdc_set_state(self._h, aY.ptr, aq.ptr, _memspace(aY, aq)))

    def get_state(self):
        """The resident state (Y (N x 3), q (N x 4)) as host arrays."""
        Y = np.empty((self.N, 3))
        q = np.empty((self.N, 4))
        _check(lib.gdc_get_state(self._h, Y.ctypes.data_as(ctypes.c_void_p), q.ctypes.data_as(ctypes.c_void_p),
                                 GDC_HOST))
        return Y, q

    def step_log(self, cap=1 << 16):
        """Completion times (ms, monotonic clock) logged since the last read;
        the first entry is the previous read's last one (or the set_state
        time)."""
        buf = np.empty(cap)
        cnt = ctypes.c_int()
        _check(lib.gdc_step_log(self._h, buf.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), cap,
                                ctypes.byref(cnt)))
        return buf[:cnt.value].copy()

    FFT_PASSES = ("plane_fwd", "proj_plane", "plane_inv", "r2c", "fwd1", "proj", "inv1", "c2r")

    @property
    def launch_config(self):
        """Workgroup sizes of the FFT passes (dict), as tuned at set-up."""
        buf = (ctypes.c_int * 8)()
        _check(lib.gdc_get_launch_config(self._h, buf, 8))
        return dict(zip(self.FFT_PASSES, list(buf)))

    @launch_config.setter
    def launch_config(self, cfg):
        cur = self.launch_config
        cur.update(cfg)
        buf = (ctypes.c_int * 8)(*[int(cur[k]) for k in self.FFT_PASSES])
        _check(lib.gdc_set_launch_config(self._h, buf, 8))

    @property
    def device_bytes(self):
        b = ctypes.c_size_t()
        _check(lib.gdc_device_bytes(self._h, ctypes.byref(b)))
        return int(b.value)

    @property
    def graphs(self):
        """Whether GMRES iterations are replayed from captured HIP graphs."""
        on = ctypes.c_int()
        _check(lib.gdc_get_graphs(self._h, ctypes.byref(on)))
        return bool(on.value)

    @graphs.setter
    def graphs(self, on):
        _check(lib.gdc_set_graphs(self._h, 1 if on else 0))

    @property
    def fusion(self):
        """Whether batch_step fuses this suspension's GMRES iterations with
        other suspensions' (one launch per kernel for all of them)."""
        on = ctypes.c_int()
        _check(lib.gdc_get_fusion(self._h, ctypes.byref(on)))
        return bool(on.value)

    @fusion.setter
    def fusion(self, on):
        _check(lib.gdc_set_fusion(self._h, 1 if on else 0))

    @property
    def step_counter(self):
        v = ctypes.c_uint64()
        _check(lib.gdc_get_step(self._h, ctypes.byref(v)))
        return int(v.value)

    @step_counter.setter
    def step_counter(self, value):
        _check(lib.gdc_set_step(self._h, int(value)))

    def fluct_velocity(self, step):
        """The random velocity field of step `step`, (3, n0, n1, n2) FP64."""
        out = np.empty((3,) + self.n)
        _check(lib.gdc_fluct_velocity(self._h, int(step), out.ctypes.data_as(ctypes.c_void_p), GDC_HOST))
        return out

    def predictor(self, Y, q, step):
        """(calV (N x 6), d (N)) of steps 1-3 at (Y, q) for step `step`."""
        aY, aq = _Arg(Y, (self.N, 3)), _Arg(q, (self.N, 4))
        calV = np.empty((self.N, 6))
        d = np.empty(self.N)
        _check(lib.gdc_predictor(self._h, aY.ptr, aq.ptr, int(step), calV.ctypes.data_as(ctypes.c_void_p),
                                 d.ctypes.data_as(ctypes.c_void_p), GDC_HOST))
        return calV, d

    def philox_normals(self, seed, c1, step, c0_begin, count):
        out = np.empty((count, 4))
        _check(lib.gdc_philox_normals(self._h, int(seed), int(c1), int(step), int(c0_begin), int(count),
                                      out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return out

    def philox_normals_noalloc(self, seed, c1, step, c0_begin, count):
        """philox_normals staged through the library's fixed per-GPU array
        (no device allocation; count <= 65536)."""
        out = np.empty((count, 4))
        _check(lib.gdc_philox_normals_noalloc(self._h, int(seed), int(c1), int(step), int(c0_begin), int(count),
                                              out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return out
