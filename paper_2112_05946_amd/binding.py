"""ctypes binding of libfrsg.so: argument marshalling only.

Every numerical step runs in the HIP library; this module converts a
configuration dictionary into the C problem struct, checks tensor shapes,
dtypes and devices, and passes raw device pointers and the current HIP stream.
If the library is missing, importing a Solver raises: there is no fallback.
"""

import ctypes
import os

import numpy as np

from . import inputs

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfrsg.so")

ABI_VERSION = 5
STATUS = {0: "OK", -1: "EINVAL", -2: "EUNSUPPORTED", -3: "EDEVICE", -4: "ENONFINITE", -5: "ENOTREALIZABLE",
          -6: "EABI"}
EQUATION = {"advection": 0, "burgers": 1, "euler1d": 2, "euler2d": 3}
BC = {"periodic": 0, "dirichlet": 1, "outflow": 2, "reflect": 3}
FILTER = {"none": 0, "exp": 1, "l2": 2, "lasso": 3}
FLUX = {"rusanov": 0, "hll": 1}
INTEGRATOR = {"ssprk3": 0, "rk4": 1, "bs3": 2, "tsit5": 3}
SENSOR = {"always": 0, "detector": 1}
PRECISION = {"fp64": 0, "fp32": 1, "bf16": 2}
ELEMENT = {"quad": 0, "tri": 1}


class FrsgError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s (%d): %s" % (STATUS.get(status, "?"), status, msg))
        self.status = status


class Problem(ctypes.Structure):
    _fields_ = [
        ("abi_version", ctypes.c_int32), ("equation", ctypes.c_int32),
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("xlo", ctypes.c_double), ("xhi", ctypes.c_double), ("ylo", ctypes.c_double), ("yhi", ctypes.c_double),
        ("bc", ctypes.c_int32 * 4), ("bc_state", (ctypes.c_double * 4) * 4),
        ("fr_degree", ctypes.c_int32), ("rdim", ctypes.c_int32), ("gpc_order", ctypes.c_int32),
        ("nq1d", ctypes.c_int32), ("adv_speed", ctypes.c_double), ("gamma", ctypes.c_double),
        ("filter", ctypes.c_int32), ("alpha", ctypes.c_double), ("s", ctypes.c_double),
        ("nstar", ctypes.c_double),
        ("eps1", ctypes.c_double), ("eps2", ctypes.c_double),
        ("sensor", ctypes.c_int32), ("s0", ctypes.c_double), ("kappa", ctypes.c_double),
        ("limiter", ctypes.c_int32), ("cfl", ctypes.c_double), ("precision", ctypes.c_int32),
        ("flux", ctypes.c_int32), ("integrator", ctypes.c_int32),
        ("element", ctypes.c_int32), ("n_tri", ctypes.c_int32),
        ("tri_xy", ctypes.c_void_p), ("tri_nbr", ctypes.c_void_p), ("tri_nbr_face", ctypes.c_void_p),
    ]


class Info(ctypes.Structure):
    _fields_ = [
        ("n_elem", ctypes.c_int64), ("nsp", ctypes.c_int32), ("n_modes", ctypes.c_int32),
        ("n_nodes", ctypes.c_int32), ("n_states", ctypes.c_int32), ("n_dof", ctypes.c_int64),
        ("state_bytes", ctypes.c_int64), ("flags_len", ctypes.c_int64), ("workspace_bytes", ctypes.c_int64),
    ]


class PassTime(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_int64), ("total_ms", ctypes.c_double),
                ("alg_bytes", ctypes.c_double)]


# (name, restype, argtypes) of every symbol in include/fr_sg.h
_VP = ctypes.c_void_p
SYMBOLS = [
    ("fr_sg_workspace_size", ctypes.c_int32, [ctypes.POINTER(Problem), ctypes.POINTER(ctypes.c_int64)]),
    ("fr_sg_init", ctypes.c_int32, [ctypes.POINTER(Problem), _VP, _VP, ctypes.c_int64, ctypes.POINTER(_VP)]),
    ("fr_sg_init_static", ctypes.c_int32, [ctypes.POINTER(Problem), _VP, ctypes.POINTER(_VP)]),
    ("fr_sg_query", ctypes.c_int32, [_VP, ctypes.POINTER(Info)]),
    ("fr_sg_set_stream", ctypes.c_int32, [_VP, _VP]),
    ("fr_sg_points", ctypes.c_int32, [_VP, _VP, _VP, _VP]),
    ("fr_sg_project", ctypes.c_int32, [_VP, _VP, _VP]),
    ("fr_sg_limit", ctypes.c_int32, [_VP, _VP, _VP]),
    ("fr_sg_rhs", ctypes.c_int32, [_VP, _VP, _VP]),
    ("fr_sg_step", ctypes.c_int32, [_VP, _VP, ctypes.c_double, _VP, _VP]),
    ("fr_sg_steps", ctypes.c_int32, [_VP, _VP, ctypes.c_int32, _VP, _VP]),
    ("fr_sg_adjoint_step", ctypes.c_int32, [_VP, _VP, _VP, ctypes.c_double, _VP, _VP]),
    ("fr_sg_step_stages", ctypes.c_int32, [_VP, _VP, ctypes.c_double, _VP, _VP, _VP, _VP]),
    ("fr_sg_adjoint_step_stages", ctypes.c_int32, [_VP, _VP, _VP, _VP, _VP, ctypes.c_double, _VP, _VP]),
    ("fr_sg_sync", ctypes.c_int32, [_VP]),
    ("fr_sg_timing_enable", ctypes.c_int32, [_VP, ctypes.c_int32]),
    ("fr_sg_timing_read", ctypes.c_int32, [_VP, ctypes.POINTER(PassTime), ctypes.c_int32,
                                           ctypes.POINTER(ctypes.c_int32)]),
    ("fr_sg_destroy", ctypes.c_int32, [_VP]),
    ("fr_sg_last_error", ctypes.c_char_p, [_VP]),
    ("fr_sg_copy", ctypes.c_int32, [_VP, _VP, ctypes.c_int64, _VP]),
]

_lib = None


def load_library(path=LIB_PATH):
    """Load libfrsg.so and declare its symbols; raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise FileNotFoundError("libfrsg.so not built (run __graft_entry__.build()): " + path)
    lib = ctypes.CDLL(path)
    for name, res, args in SYMBOLS:
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def problem_from_config(cfg, precision="fp64"):
    P = Problem()
    P.abi_version = ABI_VERSION
    P.equation = EQUATION[cfg["equation"]]
    P.nx = int(cfg["nx"])
    P.ny = int(cfg.get("ny", 1))
    P.xlo, P.xhi = float(cfg.get("xlo", 0.0)), float(cfg.get("xhi", 1.0))
    P.ylo, P.yhi = float(cfg.get("ylo", 0.0)), float(cfg.get("yhi", 1.0))
    bc = cfg.get("bc", ["periodic"] * 4)
    for i in range(4):
        P.bc[i] = BC[bc[i]]
    st = cfg.get("bc_state", [[0.0] * 4] * 4)
    for i in range(4):
        for s in range(4):
            P.bc_state[i][s] = float(st[i][s]) if s < len(st[i]) else 0.0
    P.fr_degree = int(cfg["p"])
    P.rdim = int(cfg.get("rdim", 1))
    P.gpc_order = int(cfg["gpc_order"])
    P.nq1d = int(cfg["nq1d"])
    P.adv_speed = float(cfg.get("adv_speed", 1.0))
    P.gamma = float(cfg.get("gamma", 1.4))
    P.filter = FILTER[cfg.get("filter", "none")]
    P.flux = FLUX[cfg.get("flux", "rusanov")]
    P.integrator = INTEGRATOR[cfg.get("integrator", "ssprk3")]
    P.alpha = float(cfg.get("alpha", 36.0))
    P.s = float(cfg.get("s", 8.0))
    P.nstar = float(cfg.get("nstar", 0.0))
    P.eps1 = float(cfg.get("eps1", 0.6))
    P.eps2 = float(cfg.get("eps2", 0.6))
    P.sensor = SENSOR[cfg.get("sensor", "detector")]
    P.s0 = float(cfg.get("s0", -1.0))
    P.kappa = float(cfg.get("kappa", 4.0))
    P.limiter = 1 if cfg.get("limiter", False) else 0
    P.cfl = float(cfg.get("cfl", 0.3))
    P.precision = PRECISION[precision]
    P.element = ELEMENT[cfg.get("element", "quad")]
    if P.element == ELEMENT["tri"]:
        # host arrays read by fr_sg_init only; the struct keeps them alive until then
        mesh = cfg["mesh"]
        xy = np.ascontiguousarray(mesh["xy"], dtype=np.float64)
        nb = np.ascontiguousarray(mesh["nbr"], dtype=np.int32)
        nf = np.ascontiguousarray(mesh["nbr_face"], dtype=np.int32)
        if xy.shape != (len(xy), 3, 2) or nb.shape != (len(xy), 3) or nf.shape != (len(xy), 3):
            raise ValueError("triangle mesh arrays must be xy [E, 3, 2], nbr [E, 3], nbr_face [E, 3]")
        P.n_tri = len(xy)
        P.tri_xy = xy.ctypes.data
        P.tri_nbr = nb.ctypes.data
        P.tri_nbr_face = nf.ctypes.data
        P._mesh_arrays = (xy, nb, nf)
    return P


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def device_copy(src, dst, stream=None):
    """dst <- src with the library's streaming copy kernel (fr_sg_copy): contiguous
    float64 CUDA tensors of equal size, enqueued on `stream` (default: torch's current
    stream).  A measurement utility: the bandwidth reference of the benchmark."""
    import torch
    if not (src.is_cuda and dst.is_cuda and src.dtype == torch.float64 and dst.dtype == torch.float64
            and src.is_contiguous() and dst.is_contiguous() and src.numel() == dst.numel()):
        raise ValueError("device_copy needs contiguous float64 CUDA tensors of equal size")
    lib = load_library()
    s = stream if stream is not None else torch.cuda.current_stream(src.device)
    st = lib.fr_sg_copy(_ptr(src), _ptr(dst), src.numel(), ctypes.c_void_p(s.cuda_stream))
    if st != 0:
        raise FrsgError(st, lib.fr_sg_last_error(None).decode())


class Solver:
    """One FR-SG problem on the current HIP device and stream."""

    def __init__(self, cfg, precision="fp64", stream=None, static_workspace=False):
        import torch

        self._torch = torch
        self.lib = load_library()
        self.cfg = dict(cfg)
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device")
        self.device = torch.device("cuda", torch.cuda.current_device())
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._stream = s
        self._ctx = ctypes.c_void_p()
        prob = problem_from_config(cfg, precision)
        if static_workspace:
            # the library's fixed per-GPU array (fr_sg_init_static): nothing is allocated
            self.workspace = None
            st = self.lib.fr_sg_init_static(ctypes.byref(prob), ctypes.c_void_p(s.cuda_stream),
                                            ctypes.byref(self._ctx))
            if st != 0:
                raise FrsgError(st, self.lib.fr_sg_last_error(None).decode())
            self._finish_init()
            return
        # the caller owns the workspace: a torch byte buffer of the size the library asks for
        nbytes = ctypes.c_int64()
        st = self.lib.fr_sg_workspace_size(ctypes.byref(prob), ctypes.byref(nbytes))
        if st != 0:
            raise FrsgError(st, self.lib.fr_sg_last_error(None).decode())
        with torch.cuda.stream(s):
            self.workspace = torch.empty(max(int(nbytes.value), 256), dtype=torch.uint8, device=self.device)
        st = self.lib.fr_sg_init(ctypes.byref(prob), ctypes.c_void_p(s.cuda_stream),
                                 ctypes.c_void_p(self.workspace.data_ptr()), ctypes.c_int64(self.workspace.numel()),
                                 ctypes.byref(self._ctx))
        if st != 0:
            raise FrsgError(st, self.lib.fr_sg_last_error(None).decode())
        self._finish_init()

    def _finish_init(self):
        info = Info()
        self._check(self.lib.fr_sg_query(self._ctx, ctypes.byref(info)))
        self.info = {f: getattr(info, f) for f, _ in Info._fields_}
        self.shape = (info.n_states, info.n_modes, int(info.n_elem), info.nsp)
        self.E = int(info.n_elem)

    # -- helpers ---------------------------------------------------------------
    def _check(self, st):
        if st != 0:
            raise FrsgError(st, self.lib.fr_sg_last_error(self._ctx).decode())

    def _state(self, t, name):
        torch = self._torch
        if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or t.device != self.device \
                or tuple(t.shape) != self.shape or not t.is_contiguous():
            raise ValueError("%s must be a contiguous float64 %s tensor of shape %s" % (name, self.device, self.shape))
        return t

    def _aux(self, t, dtype, n, name):
        """A caller-supplied output buffer: contiguous, on this device, of dtype, >= n entries."""
        if t is None:
            return None
        torch = self._torch
        if not isinstance(t, torch.Tensor) or t.dtype != dtype or t.device != self.device \
                or not t.is_contiguous() or t.numel() < n:
            raise ValueError("%s must be a contiguous %s %s tensor of at least %d entries"
                             % (name, dtype, self.device, n))
        return t

    def empty_state(self):
        return self._torch.empty(self.shape, dtype=self._torch.float64, device=self.device)

    # -- API -------------------------------------------------------------------
    def points(self):
        n = self.E * self.shape[3]
        x = np.zeros(n)
        y = np.zeros(n)
        z = np.zeros(self.info["n_nodes"] * int(self.cfg.get("rdim", 1)))
        self._check(self.lib.fr_sg_points(self._ctx, x.ctypes.data_as(ctypes.c_void_p),
                                          y.ctypes.data_as(ctypes.c_void_p), z.ctypes.data_as(ctypes.c_void_p)))
        rd = int(self.cfg.get("rdim", 1))
        return x.reshape(self.E, -1), y.reshape(self.E, -1), z.reshape(-1, rd)

    def project(self, u0_nodal, out=None):
        torch = self._torch
        S, M, E, nsp = self.shape
        need = (S, self.info["n_nodes"], E, nsp)
        if tuple(u0_nodal.shape) != need or u0_nodal.dtype != torch.float64 or not u0_nodal.is_contiguous():
            raise ValueError("u0_nodal must be contiguous float64 of shape %s" % (need,))
        out = self.empty_state() if out is None else self._state(out, "out")
        self._check(self.lib.fr_sg_project(self._ctx, _ptr(u0_nodal), _ptr(out)))
        return out

    def initial_state(self, ic=None, limit=True):
        """Evaluate the named analytic initial data at the library's points and project it."""
        torch = self._torch
        ic = ic or self.cfg["ic"]
        x, y, z = self.points()
        Nq = z.shape[0]
        X = np.broadcast_to(x[None], (Nq,) + x.shape)
        Y = np.broadcast_to(y[None], (Nq,) + y.shape)
        Z = np.broadcast_to(z[:, None, None, :], (Nq,) + x.shape + (z.shape[1],))
        U0 = inputs.initial_condition(ic, X, Y, Z, float(self.cfg.get("gamma", 1.4)))
        U0 = torch.from_numpy(np.ascontiguousarray(U0)).to(self.device)
        u = self.project(U0)
        if limit:
            self.limit(u)
        return u

    def limit(self, u, flags=None):
        self._state(u, "u")
        self._aux(flags, self._torch.uint8, self.E, "flags")
        self._check(self.lib.fr_sg_limit(self._ctx, _ptr(u), _ptr(flags)))
        return flags

    def rhs(self, u, out=None):
        self._state(u, "u")
        out = self.empty_state() if out is None else self._state(out, "out")
        self._check(self.lib.fr_sg_rhs(self._ctx, _ptr(u), _ptr(out)))
        return out

    def step(self, u, dt=None, dt_used=None, flags=None):
        """In-place SSP-RK3 step; dt None => CFL.  Returns (dt_used, flags) device tensors."""
        torch = self._torch
        self._state(u, "u")
        if dt_used is None:
            dt_used = torch.empty(1, dtype=torch.float64, device=self.device)
        if flags is None:
            flags = torch.empty(4 * self.E, dtype=torch.uint8, device=self.device)
        self._aux(dt_used, torch.float64, 1, "dt_used")
        self._aux(flags, torch.uint8, 4 * self.E, "flags")
        self._check(self.lib.fr_sg_step(self._ctx, _ptr(u), float(dt) if dt else 0.0, _ptr(dt_used), _ptr(flags)))
        return dt_used, flags

    def steps(self, u, nsteps, dt_used=None, flags=None):
        """nsteps in-place CFL steps; the CFL maximum of each later step comes from the step before."""
        self._state(u, "u")
        n = max(int(nsteps), 0)
        self._aux(dt_used, self._torch.float64, n, "dt_used")
        self._aux(flags, self._torch.uint8, 4 * self.E * n, "flags")
        self._check(self.lib.fr_sg_steps(self._ctx, _ptr(u), int(nsteps), _ptr(dt_used), _ptr(flags)))

    def adjoint_step(self, u_n, flags_n, dt, lam, dparams=None):
        """lam <- (d u_{n+1}/d u_n)^T lam at the step's filter flags and dt (in place);
        dparams (device float64[2] or None) accumulates d/d(adv_speed, gamma)."""
        self._state(u_n, "u_n")
        self._state(lam, "lam")
        torch = self._torch
        if flags_n is not None and (flags_n.dtype != torch.uint8 or flags_n.numel() != 4 * self.E
                                    or flags_n.device != self.device or not flags_n.is_contiguous()):
            raise ValueError("flags_n must be a contiguous uint8 device tensor of 4*E entries")
        if dparams is not None and (dparams.dtype != torch.float64 or dparams.numel() != 2
                                    or dparams.device != self.device):
            raise ValueError("dparams must be a float64 device tensor of 2 entries")
        self._check(self.lib.fr_sg_adjoint_step(self._ctx, _ptr(u_n), _ptr(flags_n), float(dt), _ptr(lam),
                                                _ptr(dparams)))
        return lam

    def step_stages(self, u, w1, w2, dt=None, dt_used=None, flags=None):
        """step() that also leaves the first and second stage states in w1 and w2."""
        torch = self._torch
        self._state(u, "u")
        self._state(w1, "w1")
        self._state(w2, "w2")
        if dt_used is None:
            dt_used = torch.empty(1, dtype=torch.float64, device=self.device)
        if flags is None:
            flags = torch.empty(4 * self.E, dtype=torch.uint8, device=self.device)
        self._aux(dt_used, torch.float64, 1, "dt_used")
        self._aux(flags, torch.uint8, 4 * self.E, "flags")
        self._check(self.lib.fr_sg_step_stages(self._ctx, _ptr(u), float(dt) if dt else 0.0, _ptr(dt_used),
                                               _ptr(flags), _ptr(w1), _ptr(w2)))
        return dt_used, flags

    def adjoint_step_stages(self, u_n, w1, w2, flags_n, dt, lam, dparams=None):
        """adjoint_step() from the stage states step_stages() left (no recomputation)."""
        self._state(u_n, "u_n")
        self._state(w1, "w1")
        self._state(w2, "w2")
        self._state(lam, "lam")
        torch = self._torch
        if flags_n is not None and (flags_n.dtype != torch.uint8 or flags_n.numel() != 4 * self.E
                                    or flags_n.device != self.device or not flags_n.is_contiguous()):
            raise ValueError("flags_n must be a contiguous uint8 device tensor of 4*E entries")
        if dparams is not None and (dparams.dtype != torch.float64 or dparams.numel() != 2
                                    or dparams.device != self.device):
            raise ValueError("dparams must be a float64 device tensor of 2 entries")
        self._check(self.lib.fr_sg_adjoint_step_stages(self._ctx, _ptr(u_n), _ptr(w1), _ptr(w2), _ptr(flags_n),
                                                       float(dt), _ptr(lam), _ptr(dparams)))
        return lam

    def timing(self, enable=True):
        self._check(self.lib.fr_sg_timing_enable(self._ctx, 1 if enable else 0))

    def timing_read(self):
        """{pass name: (launches, total_ms, algorithmic bytes per launch)}; synchronises."""
        buf = (PassTime * 64)()
        n = ctypes.c_int32()
        self._check(self.lib.fr_sg_timing_read(self._ctx, buf, 64, ctypes.byref(n)))
        return {buf[i].name.decode(): (int(buf[i].launches), float(buf[i].total_ms), float(buf[i].alg_bytes))
                for i in range(n.value)}

    def sync(self):
        self._check(self.lib.fr_sg_sync(self._ctx))

    def close(self):
        if self._ctx:
            self.lib.fr_sg_destroy(self._ctx)
            self._ctx = ctypes.c_void_p()
        self.workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
