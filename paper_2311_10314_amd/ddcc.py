"""Thin Python binding of libddcc.so (include/ddcc.h).

Argument marshalling only: every step of the scheme runs in the HIP
library. Importing this module loads the in-tree libddcc.so and raises if it
is missing; there is no fallback implementation.

The module-level functions carry the C names (ddcc_create, ddcc_step, ...).
`Sim` wraps one context for convenience: numpy arrays for the host calls,
torch CUDA tensors (float64, contiguous) for the *_dev calls.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libddcc.so")

DDCC_OK = 0
DDCC_E_INVAL = 1
DDCC_E_STATE = 2
DDCC_E_NOMEM = 3
DDCC_E_HIP = 4
DDCC_E_NONFINITE = 5
DDCC_E_UNSUPPORTED = 6

LATTICES = {"D2Q9": 0, "D3Q7": 1, "D3Q15": 2, "D3Q19": 3}
FP64, FP32, FP16, BF16 = 0, 1, 2, 3
PRECISIONS = {"fp64": FP64, "fp32": FP32, "fp16": FP16, "bf16": BF16}
MAX_PHASES = 4
RATE_SLOTS = ("0", "1", "21", "22", "3", "4")


class ddcc_params(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int), ("nx", ctypes.c_int), ("ny", ctypes.c_int),
        ("nz", ctypes.c_int), ("nphase", ctypes.c_int),
        ("lattice_f", ctypes.c_int), ("lattice_g", ctypes.c_int),
        ("precision", ctypes.c_int),
        ("d0", ctypes.c_double), ("eps", ctypes.c_double),
        ("m0", ctypes.c_double), ("rho0", ctypes.c_double),
        ("psi_min", ctypes.c_double), ("lam", ctypes.c_double),
        ("sigma", (ctypes.c_double * MAX_PHASES) * MAX_PHASES),
        ("rho", ctypes.c_double * MAX_PHASES),
        ("nu", ctypes.c_double * MAX_PHASES),
        ("eta", ctypes.c_double * MAX_PHASES),
        ("s_f", ctypes.c_double * 6), ("s_g", ctypes.c_double * 6),
        ("accel", ctypes.c_double * 3),
        ("force", ctypes.c_double * 3),
    ]


class DDCCError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("ddcc error %d: %s" % (code, msg))
        self.code = code


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            "libddcc.so is not built (%s); run "
            "`python -m paper_2311_10314_amd.build`" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    dp = P(ctypes.c_double)
    vp = ctypes.c_void_p
    ctx = vp
    sig = {
        "ddcc_default_params": (ctypes.c_int, [P(ddcc_params)]),
        "ddcc_create": (ctypes.c_int, [P(ddcc_params), vp, P(vp)]),
        "ddcc_init_geometry": (ctypes.c_int, [ctx, dp, dp]),
        "ddcc_init_geometry_dev": (ctypes.c_int, [ctx, vp, vp]),
        "ddcc_init_geometry_walls": (ctypes.c_int, [ctx, ctypes.c_int, dp,
                                                    dp]),
        "ddcc_init_fields": (ctypes.c_int, [ctx, dp, dp, dp]),
        "ddcc_init_fields_dev": (ctypes.c_int, [ctx, vp, vp, vp]),
        "ddcc_step": (ctypes.c_int, [ctx, ctypes.c_int64]),
        "ddcc_read_moments": (ctypes.c_int, [ctx, dp, dp, dp]),
        "ddcc_read_moments_dev": (ctypes.c_int, [ctx, vp, vp, vp]),
        "ddcc_mass": (ctypes.c_int, [ctx, dp]),
        "ddcc_mass_noalloc": (ctypes.c_int, [ctx, vp, vp]),
        "ddcc_time": (ctypes.c_int64, [ctx]),
        "ddcc_save": (ctypes.c_int, [ctx, vp, P(ctypes.c_size_t)]),
        "ddcc_load": (ctypes.c_int, [ctx, vp, ctypes.c_size_t]),
        "ddcc_sync": (ctypes.c_int, [ctx]),
        "ddcc_set_tile": (ctypes.c_int, [ctx, ctypes.c_int, ctypes.c_int]),
        "ddcc_autotune": (ctypes.c_int, [ctx, ctypes.c_int, P(ctypes.c_int)]),
        "ddcc_set_diagnostics": (ctypes.c_int, [ctx, ctypes.c_int]),
        "ddcc_diagnostics": (ctypes.c_int, [ctx, dp, P(ctypes.c_int64),
                                            P(ctypes.c_int64)]),
        "ddcc_adjoint": (ctypes.c_int, [ctx, ctypes.c_int64, ctypes.c_int,
                                        ctypes.c_int, dp, dp, dp, dp]),
        "ddcc_objective": (ctypes.c_int, [ctx, ctypes.c_int, dp, dp]),
        "ddcc_last_error": (ctypes.c_char_p, [ctx]),
        "ddcc_destroy": (None, [ctx]),
        "ddcc_version": (ctypes.c_char_p, []),
        "ddcc_batch_create": (ctypes.c_int, [P(ddcc_params), ctypes.c_int,
                                             P(ctypes.c_int), P(ctypes.c_int),
                                             vp, P(vp)]),
        "ddcc_batch_set_params": (ctypes.c_int, [vp, ctypes.c_int,
                                                 P(ddcc_params)]),
        "ddcc_batch_init_geometry": (ctypes.c_int, [vp, ctypes.c_int, dp, dp]),
        "ddcc_batch_init_fields": (ctypes.c_int, [vp, ctypes.c_int, dp, dp,
                                                  dp]),
        "ddcc_batch_step": (ctypes.c_int, [vp, ctypes.c_int64]),
        "ddcc_batch_read_moments": (ctypes.c_int, [vp, ctypes.c_int, dp, dp,
                                                   dp]),
        "ddcc_batch_mass": (ctypes.c_int, [vp, ctypes.c_int, dp]),
        "ddcc_batch_set_tile": (ctypes.c_int, [vp, ctypes.c_int]),
        "ddcc_batch_autotune": (ctypes.c_int, [vp, ctypes.c_int,
                                               P(ctypes.c_int)]),
        "ddcc_batch_set_graph": (ctypes.c_int, [vp, ctypes.c_int]),
        "ddcc_batch_sync": (ctypes.c_int, [vp]),
        "ddcc_batch_time": (ctypes.c_int64, [vp]),
        "ddcc_batch_last_error": (ctypes.c_char_p, [vp]),
        "ddcc_batch_destroy": (None, [vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


LIB = _load()

# C-named entry points
ddcc_default_params = LIB.ddcc_default_params
ddcc_create = LIB.ddcc_create
ddcc_init_geometry = LIB.ddcc_init_geometry
ddcc_init_geometry_dev = LIB.ddcc_init_geometry_dev
ddcc_init_geometry_walls = LIB.ddcc_init_geometry_walls
ddcc_init_fields = LIB.ddcc_init_fields
ddcc_init_fields_dev = LIB.ddcc_init_fields_dev
ddcc_step = LIB.ddcc_step
ddcc_read_moments = LIB.ddcc_read_moments
ddcc_read_moments_dev = LIB.ddcc_read_moments_dev
ddcc_mass = LIB.ddcc_mass
ddcc_mass_noalloc = LIB.ddcc_mass_noalloc
ddcc_time = LIB.ddcc_time
ddcc_save = LIB.ddcc_save
ddcc_load = LIB.ddcc_load
ddcc_sync = LIB.ddcc_sync
ddcc_set_tile = LIB.ddcc_set_tile
ddcc_autotune = LIB.ddcc_autotune
ddcc_set_diagnostics = LIB.ddcc_set_diagnostics
ddcc_diagnostics = LIB.ddcc_diagnostics
ddcc_adjoint = LIB.ddcc_adjoint
ddcc_objective = LIB.ddcc_objective
ddcc_last_error = LIB.ddcc_last_error
ddcc_destroy = LIB.ddcc_destroy
ddcc_version = LIB.ddcc_version
ddcc_batch_create = LIB.ddcc_batch_create
ddcc_batch_set_params = LIB.ddcc_batch_set_params
ddcc_batch_init_geometry = LIB.ddcc_batch_init_geometry
ddcc_batch_init_fields = LIB.ddcc_batch_init_fields
ddcc_batch_step = LIB.ddcc_batch_step
ddcc_batch_read_moments = LIB.ddcc_batch_read_moments
ddcc_batch_mass = LIB.ddcc_batch_mass
ddcc_batch_set_tile = LIB.ddcc_batch_set_tile
ddcc_batch_autotune = LIB.ddcc_batch_autotune
ddcc_batch_set_graph = LIB.ddcc_batch_set_graph
ddcc_batch_sync = LIB.ddcc_batch_sync
ddcc_batch_time = LIB.ddcc_batch_time
ddcc_batch_last_error = LIB.ddcc_batch_last_error
ddcc_batch_destroy = LIB.ddcc_batch_destroy


def make_params(dim, shape, nphase, lattice_f, lattice_g, precision="fp64",
                **prm):
    """Fill a ddcc_params from plain numbers (lattice units). `shape` is the
    array shape (ny, nx) or (nz, ny, nx); keys as in workloads.default_params:
    d0, eps, eps0 (penalty lam = 1/eps0^3 unless lam is given), m0, rho0,
    psi_min, sigma, rho, nu, eta, s_f, s_g (dicts by slot name), accel,
    force."""
    p = ddcc_params()
    LIB.ddcc_default_params(ctypes.byref(p))
    p.dim = dim
    if dim == 2:
        p.ny, p.nx = shape
        p.nz = 1
    else:
        p.nz, p.ny, p.nx = shape
    p.nphase = nphase
    p.lattice_f = LATTICES[lattice_f]
    p.lattice_g = LATTICES[lattice_g]
    p.precision = PRECISIONS[precision] if isinstance(precision, str) \
        else int(precision)
    for key in ("d0", "eps", "m0", "rho0", "psi_min"):
        if key in prm:
            setattr(p, key, float(prm[key]))
    if prm.get("lam") is not None:
        p.lam = float(prm["lam"])
    elif prm.get("eps0") is not None:
        p.lam = 1.0 / float(prm["eps0"]) ** 3
    if "sigma" in prm:
        s = np.asarray(prm["sigma"], dtype=np.float64)
        for i in range(MAX_PHASES):
            for j in range(MAX_PHASES):
                p.sigma[i][j] = s[i, j] if (i < nphase and j < nphase) else \
                    (0.0 if i == j else 1.0)
    for key in ("rho", "nu", "eta"):
        if key in prm and prm[key] is not None:
            v = np.broadcast_to(np.asarray(prm[key], dtype=np.float64),
                                (nphase,))
            arr = getattr(p, key)
            for i in range(nphase):
                arr[i] = v[i]
    for key in ("s_f", "s_g"):
        if key in prm:
            arr = getattr(p, key)
            for slot, val in prm[key].items():
                arr[RATE_SLOTS.index(slot)] = float(val)
    for key in ("accel", "force"):
        if key in prm and prm[key] is not None:
            arr = getattr(p, key)
            for a, v in enumerate(prm[key]):
                arr[a] = float(v)
    return p


def centroid_weight(shape):
    """w(x) = x, the node index along x (the last array axis)."""
    return np.ascontiguousarray(np.broadcast_to(
        np.arange(shape[-1], dtype=np.float64), shape))


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _c64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class Sim:
    """One library context. Raises DDCCError on any non-zero return code."""

    def __init__(self, params, stream=None):
        self.params = params
        self.dim = params.dim
        self.nphase = params.nphase
        self.shape = ((params.ny, params.nx) if params.dim == 2 else
                      (params.nz, params.ny, params.nx))
        h = ctypes.c_void_p()
        st = ctypes.c_void_p(stream) if stream is not None else None
        rc = LIB.ddcc_create(ctypes.byref(params), st, ctypes.byref(h))
        if rc != DDCC_OK:
            raise DDCCError(rc, "ddcc_create failed")
        self._h = h

    @classmethod
    def from_workload(cls, wl, precision="fp64", stream=None):
        p = make_params(wl.dim, wl.shape, wl.nphase, wl.lattice_f,
                        wl.lattice_g, precision, **wl.params)
        s = cls(p, stream)
        if getattr(wl, "walls", None):
            s.init_geometry_walls([w[0] for w in wl.walls],
                                  [w[1] for w in wl.walls])
        else:
            s.init_geometry(wl.psi, wl.cos_theta_iN)
        s.init_fields(wl.C0, wl.u0, wl.P0)
        return s

    def _check(self, rc):
        if rc != DDCC_OK:
            raise DDCCError(rc, LIB.ddcc_last_error(self._h).decode())

    def init_geometry(self, psi, cos_theta=None):
        psi = _c64(psi)
        ct = None if cos_theta is None else _c64(cos_theta)
        self._check(LIB.ddcc_init_geometry(self._h, _dptr(psi),
                                           None if ct is None else _dptr(ct)))

    def init_fields(self, C, u=None, P=None):
        C = _c64(C)
        u = None if u is None else _c64(u)
        P = None if P is None else _c64(P)
        self._check(LIB.ddcc_init_fields(
            self._h, _dptr(C), None if u is None else _dptr(u),
            None if P is None else _dptr(P)))

    def init_geometry_walls(self, psis, cos_thetas=None):
        """psis: K arrays psi_k; cos_thetas: K arrays cos theta^k_iN (or
        None for 90 degrees)."""
        psi = _c64(np.stack(psis))
        ct = None if cos_thetas is None else _c64(np.stack(cos_thetas))
        self._check(LIB.ddcc_init_geometry_walls(
            self._h, len(psis), _dptr(psi), None if ct is None else _dptr(ct)))

    def init_geometry_dev(self, psi, cos_theta=None):
        self._check(LIB.ddcc_init_geometry_dev(
            self._h, psi.data_ptr(),
            None if cos_theta is None else cos_theta.data_ptr()))

    def init_fields_dev(self, C, u=None, P=None):
        self._check(LIB.ddcc_init_fields_dev(
            self._h, C.data_ptr(), None if u is None else u.data_ptr(),
            None if P is None else P.data_ptr()))

    def step(self, n=1):
        self._check(LIB.ddcc_step(self._h, int(n)))

    def read_moments(self):
        C = np.empty((self.nphase,) + self.shape)
        u = np.empty((self.dim,) + self.shape)
        P = np.empty(self.shape)
        self._check(LIB.ddcc_read_moments(self._h, _dptr(C), _dptr(u),
                                          _dptr(P)))
        return C, u, P

    def read_moments_dev(self, C, u, P):
        self._check(LIB.ddcc_read_moments_dev(self._h, C.data_ptr(),
                                              u.data_ptr(), P.data_ptr()))

    def mass(self):
        m = np.empty(self.nphase)
        self._check(LIB.ddcc_mass(self._h, _dptr(m)))
        return m

    def mass_noalloc(self, mass_dev, nonfinite_dev=None):
        """ddcc_mass_noalloc into device tensors (float64 [nphase], int32
        [1] or None); asynchronous on the context stream."""
        self._check(LIB.ddcc_mass_noalloc(
            self._h, mass_dev.data_ptr(),
            None if nonfinite_dev is None else nonfinite_dev.data_ptr()))

    @property
    def time(self):
        return int(LIB.ddcc_time(self._h))

    def save(self):
        nb = ctypes.c_size_t(0)
        self._check(LIB.ddcc_save(self._h, None, ctypes.byref(nb)))
        buf = np.empty(nb.value, dtype=np.uint8)
        self._check(LIB.ddcc_save(self._h, buf.ctypes.data_as(ctypes.c_void_p),
                                  ctypes.byref(nb)))
        return buf

    def load(self, buf):
        buf = np.ascontiguousarray(buf, dtype=np.uint8)
        self._check(LIB.ddcc_load(self._h, buf.ctypes.data_as(ctypes.c_void_p),
                                  buf.nbytes))

    def sync(self):
        self._check(LIB.ddcc_sync(self._h))

    def set_tile(self, tx=0, ty=0):
        self._check(LIB.ddcc_set_tile(self._h, int(tx), int(ty)))

    def set_diagnostics(self, every):
        """Per-phase masses and a non-finite check every `every` steps,
        inside the step stream (0: off)."""
        self._check(LIB.ddcc_set_diagnostics(self._h, int(every)))

    def diagnostics(self):
        """(masses of the last check, its step, first step whose check saw
        a non-finite population or -1)."""
        m = np.empty(self.nphase)
        tc = ctypes.c_int64(0)
        tn = ctypes.c_int64(0)
        self._check(LIB.ddcc_diagnostics(self._h, _dptr(m), ctypes.byref(tc),
                                         ctypes.byref(tn)))
        return m, tc.value, tn.value

    def autotune(self, steps=5):
        """Time each tile height on the current state, keep the fastest and
        restore the state; returns the chosen height."""
        ty = ctypes.c_int(0)
        self._check(LIB.ddcc_autotune(self._h, int(steps), ctypes.byref(ty)))
        return ty.value

    def adjoint(self, nsteps, interval=100, phase=0, weight=None):
        """ddcc_adjoint: J and its gradients (dJ/dcos theta_iN of shape
        (nphase - 1,) + shape, dJ/dpsi of shape `shape`) over the next
        nsteps steps; weight defaults to the node index along x (J is then
        the centroid x of `phase`). The context advances by nsteps."""
        w = centroid_weight(self.shape) if weight is None else _c64(weight)
        J = ctypes.c_double(0.0)
        gc = np.empty((self.nphase - 1,) + self.shape)
        gp = np.empty(self.shape)
        self._check(LIB.ddcc_adjoint(self._h, int(nsteps), int(interval),
                                     int(phase), _dptr(w), ctypes.byref(J),
                                     _dptr(gc), _dptr(gp)))
        return J.value, gc, gp

    def objective(self, phase=0, weight=None):
        """ddcc_objective: sum w phi C_k / sum phi C_k on the current state
        (weight defaults to the node index along x)."""
        w = centroid_weight(self.shape) if weight is None else _c64(weight)
        J = ctypes.c_double(0.0)
        self._check(LIB.ddcc_objective(self._h, int(phase), _dptr(w),
                                       ctypes.byref(J)))
        return J.value

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            LIB.ddcc_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """A batch of independent 2D instances (ddcc_batch_*). Instance i has
    the grid shapes[i] = (ny, nx); arrays are per instance, as for Sim."""

    def __init__(self, params, shapes, stream=None):
        self.params = params
        self.nphase = params.nphase
        self.shapes = [tuple(int(v) for v in sh) for sh in shapes]
        ny = (ctypes.c_int * len(shapes))(*[sh[0] for sh in self.shapes])
        nx = (ctypes.c_int * len(shapes))(*[sh[1] for sh in self.shapes])
        h = ctypes.c_void_p()
        st = ctypes.c_void_p(stream) if stream is not None else None
        rc = LIB.ddcc_batch_create(ctypes.byref(params), len(shapes), nx, ny,
                                   st, ctypes.byref(h))
        if rc != DDCC_OK:
            raise DDCCError(rc, "ddcc_batch_create failed")
        self._h = h

    @classmethod
    def from_workloads(cls, wls, precision="fp32", stream=None):
        """All workloads must share N; an instance whose method parameters
        differ from the first one's gets its own (ddcc_batch_set_params)."""
        w0 = wls[0]
        p = make_params(2, w0.shape, w0.nphase, "D2Q9", "D2Q9", precision,
                        **w0.params)
        b = cls(p, [w.shape for w in wls], stream)
        for i, w in enumerate(wls):
            if w.params != w0.params:
                b.set_params(i, make_params(2, w.shape, w.nphase, "D2Q9",
                                            "D2Q9", precision, **w.params))
            b.init_geometry(i, w.psi, w.cos_theta_iN)
            b.init_fields(i, w.C0, w.u0, w.P0)
        return b

    def set_params(self, i, params):
        """Method parameters of instance i (a ddcc_params with the batch's
        dim, N, lattices and precision); call before its init_fields."""
        self._check(LIB.ddcc_batch_set_params(self._h, int(i),
                                              ctypes.byref(params)))

    def _check(self, rc):
        if rc != DDCC_OK:
            raise DDCCError(rc, LIB.ddcc_batch_last_error(self._h).decode())

    def init_geometry(self, i, psi, cos_theta=None):
        psi = _c64(psi)
        ct = None if cos_theta is None else _c64(cos_theta)
        self._check(LIB.ddcc_batch_init_geometry(
            self._h, int(i), _dptr(psi), None if ct is None else _dptr(ct)))

    def init_fields(self, i, C, u=None, P=None):
        C = _c64(C)
        u = None if u is None else _c64(u)
        P = None if P is None else _c64(P)
        self._check(LIB.ddcc_batch_init_fields(
            self._h, int(i), _dptr(C), None if u is None else _dptr(u),
            None if P is None else _dptr(P)))

    def step(self, n=1):
        self._check(LIB.ddcc_batch_step(self._h, int(n)))

    def read_moments(self, i):
        sh = self.shapes[i]
        C = np.empty((self.nphase,) + sh)
        u = np.empty((2,) + sh)
        P = np.empty(sh)
        self._check(LIB.ddcc_batch_read_moments(self._h, int(i), _dptr(C),
                                                _dptr(u), _dptr(P)))
        return C, u, P

    def mass(self, i):
        m = np.empty(self.nphase)
        self._check(LIB.ddcc_batch_mass(self._h, int(i), _dptr(m)))
        return m

    def set_tile(self, ty):
        self._check(LIB.ddcc_batch_set_tile(self._h, int(ty)))

    def autotune(self, steps=5):
        ty = ctypes.c_int(0)
        self._check(LIB.ddcc_batch_autotune(self._h, int(steps),
                                            ctypes.byref(ty)))
        return ty.value

    def set_graph(self, steps_per_graph):
        self._check(LIB.ddcc_batch_set_graph(self._h, int(steps_per_graph)))

    def sync(self):
        self._check(LIB.ddcc_batch_sync(self._h))

    @property
    def time(self):
        return int(LIB.ddcc_batch_time(self._h))

    @property
    def nodes(self):
        return int(sum(a * b for a, b in self.shapes))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            LIB.ddcc_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
