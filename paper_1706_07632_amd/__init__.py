"""Python binding of libmgwr (argument marshalling only).

Every step of the solver runs in the HIP kernels of libmgwr.so; this module
only converts arguments, owns the torch workspace tensor that backs a plan,
and raises on non-OK status codes.  It fails loudly when the library has not
been built: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libmgwr.so")

MGWR_OK = 0
MGWR_ERR_INVALID_ARG = 1
MGWR_ERR_STATE = 2
MGWR_ERR_HIP = 3
MGWR_ERR_NOT_CONVERGED = 4
MGWR_ERR_NONFINITE = 5
MGWR_ERR_MODEL = 6
MGWR_FP64 = 0
MGWR_MIXED_FP32 = 1
MGWR_MIXED_BF16 = 2
MGWR_GUESS_IN_U = 1
MGWR_WARM_START = 2
MGWR_WARM_RES0 = 4

EXPORTED = [
    "mgwr_params_default", "mgwr_plan_create", "mgwr_plan_workspace_bytes", "mgwr_plan_bind",
    "mgwr_solve", "mgwr_residual", "mgwr_hmatvec", "mgwr_htrsm", "mgwr_plan_get_info",
    "mgwr_plan_get_mesh", "mgwr_plan_export_dense", "mgwr_plan_set_progress_limit", "mgwr_plan_destroy",
    "mgwr_last_error",
    "mgwr_timing_enable", "mgwr_timing_get", "mgwr_batch_create", "mgwr_batch_workspace_bytes",
    "mgwr_batch_bind", "mgwr_batch_solve", "mgwr_batch_timing", "mgwr_batch_destroy",
    "mgwr_net_create", "mgwr_net_param_count", "mgwr_net_workspace_bytes", "mgwr_net_bind",
    "mgwr_net_sync_weights", "mgwr_net_forward", "mgwr_net_gradient", "mgwr_net_set_finest",
    "mgwr_net_adam_step", "mgwr_net_destroy",
    "mgwr_plan_set_warm_start", "mgwr_batch_set_graph", "mgwr_batch_graph_replays", "mgwr_plan_autotune",
    "mgwr_plan_set_staging", "mgwr_plan_tuned", "mgwr_plan_set_layout", "mgwr_apply_A", "mgwr_model_describe",
    "mgwr_model_load", "mgwr_set_xcd_queues", "mgwr_xcd_queues_in_use",
    "mgwr_solve_static",
]

KERNEL_CLASSES = ["smooth64", "defect64", "smooth32", "defect32", "restrict", "prolong", "pipe64", "coarse", "side"]
NCLASSES = len(KERNEL_CLASSES)


class MgwrError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"mgwr error {code}: {msg}")
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("n", ctypes.c_int), ("length", ctypes.c_double),
                ("M", ctypes.c_int), ("T", ctypes.c_double), ("alpha", ctypes.c_double),
                ("r", ctypes.c_double), ("k", ctypes.c_int), ("leaf", ctypes.c_int),
                ("nu1", ctypes.c_int), ("nu2", ctypes.c_int), ("gamma", ctypes.c_int),
                ("max_cycles", ctypes.c_int), ("precision", ctypes.c_int), ("inner_cycles", ctypes.c_int),
                ("schedule", ctypes.c_int), ("eta", ctypes.c_double), ("cluster", ctypes.c_int)]


class Stats(ctypes.Structure):
    _fields_ = [("cycles", ctypes.c_int), ("refinements", ctypes.c_int), ("res0", ctypes.c_double),
                ("bnorm", ctypes.c_double), ("res", ctypes.c_double), ("avg_factor", ctypes.c_double),
                ("history", ctypes.c_double * 64), ("used_warm_start", ctypes.c_int), ("warm_res0", ctypes.c_double),
                ("setup_ms", ctypes.c_double), ("solve_ms", ctypes.c_double)]

    def as_dict(self):
        d = {f: getattr(self, f) for f, _ in self._fields_ if f != "history"}
        steps = self.refinements if self.refinements else self.cycles
        d["history"] = [self.history[i] for i in range(min(steps, 64))]
        return d


class Timing(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_longlong * NCLASSES), ("ms", ctypes.c_double * NCLASSES),
                ("flops", ctypes.c_double * NCLASSES), ("bytes", ctypes.c_double * NCLASSES)]

    def as_dict(self):
        return {name: {"launches": self.launches[i], "ms": self.ms[i], "flops": self.flops[i],
                       "bytes": self.bytes[i]} for i, name in enumerate(KERNEL_CLASSES)}


class ModelInfo(ctypes.Structure):
    _fields_ = [("layers", ctypes.c_int), ("channels", ctypes.c_int * 17), ("nsignal", ctypes.c_int),
                ("nslices", ctypes.c_int), ("rows", ctypes.c_int * 64), ("h_min", ctypes.c_double),
                ("nparam", ctypes.c_longlong)]

    def as_dict(self):
        return {"layers": self.layers, "channels": [self.channels[i] for i in range(self.layers + 1)],
                "nsignal": self.nsignal, "nslices": self.nslices,
                "rows": [self.rows[i] for i in range(self.nslices)], "h_min": self.h_min, "nparam": self.nparam}


class PlanInfo(ctypes.Structure):
    _fields_ = [("M", ctypes.c_int), ("nleaf", ctypes.c_int), ("nclusters", ctypes.c_int),
                ("ndense", ctypes.c_int), ("nrk", ctypes.c_int), ("nzclusters", ctypes.c_int),
                ("nslots", ctypes.c_int), ("window", ctypes.c_int), ("levels", ctypes.c_int),
                ("k", ctypes.c_int), ("stored_entries", ctypes.c_longlong), ("shift0", ctypes.c_double),
                ("layout", ctypes.c_int), ("nf64leaves", ctypes.c_int)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_lib = None


def lib():
    """The loaded libmgwr (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1706_07632_amd.build` "
                          "or __graft_entry__.build()")
    L = ctypes.CDLL(LIB_PATH)
    vp, dp, ip = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_int
    L.mgwr_params_default.argtypes = [ctypes.POINTER(Params)]
    L.mgwr_params_default.restype = None
    L.mgwr_plan_create.argtypes = [ctypes.POINTER(Params), dp, ctypes.POINTER(vp)]
    L.mgwr_plan_workspace_bytes.argtypes = [vp, ctypes.POINTER(ctypes.c_size_t)]
    L.mgwr_plan_bind.argtypes = [vp, vp, ctypes.c_size_t, vp]
    L.mgwr_solve.argtypes = [vp, vp, vp, ctypes.c_double, vp, ctypes.c_uint, ctypes.POINTER(Stats)]
    L.mgwr_residual.argtypes = [vp, vp, vp, vp, vp, dp]
    L.mgwr_hmatvec.argtypes = [vp, vp, vp, ip]
    L.mgwr_htrsm.argtypes = [vp, ip, vp, vp, ip]
    L.mgwr_plan_get_info.argtypes = [vp, ctypes.POINTER(PlanInfo)]
    L.mgwr_plan_get_mesh.argtypes = [vp, dp, dp]
    L.mgwr_plan_export_dense.argtypes = [vp, dp]
    L.mgwr_plan_destroy.argtypes = [vp]
    L.mgwr_plan_set_progress_limit.argtypes = [vp, ctypes.c_uint]
    L.mgwr_timing_enable.argtypes = [vp, ip]
    L.mgwr_timing_get.argtypes = [vp, ctypes.POINTER(Timing)]
    L.mgwr_batch_create.argtypes = [ip, ctypes.POINTER(vp), ctypes.POINTER(vp)]
    L.mgwr_batch_workspace_bytes.argtypes = [vp, ctypes.POINTER(ctypes.c_size_t)]
    L.mgwr_batch_bind.argtypes = [vp, vp, ctypes.c_size_t, vp]
    L.mgwr_batch_solve.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.c_double,
                                   ctypes.POINTER(vp), ctypes.c_uint, ctypes.POINTER(Stats)]
    L.mgwr_batch_timing.argtypes = [vp, ip, ctypes.POINTER(Timing)]
    L.mgwr_batch_destroy.argtypes = [vp]
    L.mgwr_batch_set_graph.argtypes = [vp, ip]
    L.mgwr_batch_graph_replays.argtypes = [vp, ctypes.POINTER(ctypes.c_longlong)]
    L.mgwr_plan_autotune.argtypes = [vp, vp, vp, ctypes.c_double, vp, ctypes.POINTER(ctypes.c_int)]
    L.mgwr_plan_set_staging.argtypes = [vp, ctypes.c_int, ctypes.c_int]
    L.mgwr_plan_set_layout.argtypes = [vp, ctypes.c_int]
    ipp = ctypes.POINTER(ctypes.c_int)
    L.mgwr_set_xcd_queues.argtypes = [ip, ipp]
    L.mgwr_xcd_queues_in_use.argtypes = [vp, ipp]
    L.mgwr_plan_tuned.argtypes = [vp, ipp, ipp, ipp]
    L.mgwr_net_create.argtypes = [ip, ctypes.POINTER(ctypes.c_int), ip, ctypes.POINTER(vp)]
    L.mgwr_net_param_count.argtypes = [vp, ctypes.POINTER(ctypes.c_size_t)]
    L.mgwr_net_workspace_bytes.argtypes = [vp, ctypes.c_longlong, ctypes.POINTER(ctypes.c_size_t)]
    L.mgwr_net_bind.argtypes = [vp, vp, ctypes.c_longlong, vp, ctypes.c_size_t, vp]
    L.mgwr_net_sync_weights.argtypes = [vp]
    L.mgwr_net_forward.argtypes = [vp, vp, ip, ip, ip, ctypes.c_double, vp]
    L.mgwr_net_gradient.argtypes = [vp, vp, vp, ip, ip, ip, ctypes.c_double, vp, ctypes.POINTER(ctypes.c_double)]
    L.mgwr_net_set_finest.argtypes = [vp, ctypes.c_double]
    L.mgwr_net_adam_step.argtypes = [vp, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float, ip]
    L.mgwr_net_destroy.argtypes = [vp]
    L.mgwr_plan_set_warm_start.argtypes = [vp, vp, ip, ctypes.POINTER(ctypes.c_int)]
    L.mgwr_apply_A.argtypes = [vp, vp, vp]
    L.mgwr_solve_static.argtypes = [vp, vp, vp, vp, ctypes.c_double, vp, ctypes.c_uint, ctypes.POINTER(Stats)]
    L.mgwr_model_describe.argtypes = [ctypes.c_char_p, ctypes.c_size_t, ctypes.POINTER(ModelInfo)]
    L.mgwr_model_load.argtypes = [vp, vp, ctypes.c_char_p, ctypes.c_size_t]
    L.mgwr_last_error.argtypes = []
    L.mgwr_last_error.restype = ctypes.c_char_p
    for name in EXPORTED:
        fn = getattr(L, name)
        if name not in ("mgwr_params_default", "mgwr_last_error"):
            fn.restype = ctypes.c_int
    _lib = L
    return L


def _check(rc, ok=(MGWR_OK,)):
    if rc not in ok:
        raise MgwrError(rc, lib().mgwr_last_error().decode())
    return rc


def _dptr(x):
    return None if x is None else ctypes.c_void_p(x.data_ptr())


def _require(x, name, shape, dtype=None):
    import torch
    dtype = torch.float64 if dtype is None else dtype
    if not x.is_cuda:
        raise ValueError(f"{name} must be a ROCm device tensor")
    if x.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}")
    if not x.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if tuple(x.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(x.shape)}, expected {tuple(shape)}")


class Plan:
    """H-matrix MGWR plan for one (mesh, alpha, k, grid).

    dim, n, M, alpha, k: problem and rank; r / T build the graded mesh unless
    an explicit mesh `t` (length M+1, host array) is given.
    """

    def __init__(self, dim, n, M, alpha, k=10, r=1.0, T=1.0, length=1.0, t=None, leaf=16,
                 nu1=1, nu2=1, gamma=1, max_cycles=50, precision="fp64", inner_cycles=1,
                 schedule="auto", eta=1.0, cluster="index"):
        import numpy as np
        L = lib()
        p = Params()
        L.mgwr_params_default(ctypes.byref(p))
        p.dim, p.n, p.M, p.alpha, p.k = int(dim), int(n), int(M), float(alpha), int(k)
        p.r, p.T, p.length, p.leaf = float(r), float(T), float(length), int(leaf)
        p.nu1, p.nu2, p.gamma, p.max_cycles = int(nu1), int(nu2), int(gamma), int(max_cycles)
        p.precision = {"fp64": MGWR_FP64, "mixed": MGWR_MIXED_FP32, "fp32": MGWR_MIXED_FP32,
                       "mixed_bf16": MGWR_MIXED_BF16, "bf16": MGWR_MIXED_BF16}[precision]
        p.inner_cycles = int(inner_cycles)
        p.schedule = {"auto": 0, "staged": 1, "pipelined": 2}[schedule]
        p.eta = float(eta)
        p.cluster = {"index": 0, "geometric": 1}[cluster]
        self.params = p
        self.dim, self.n, self.M = int(dim), int(n), int(M)
        self.N = self.n ** self.dim
        handle = ctypes.c_void_p()
        tp = None
        if t is not None:
            self._t_host = np.ascontiguousarray(np.asarray(t, dtype=np.float64))
            if self._t_host.shape != (self.M + 1,):
                raise ValueError("t must have M+1 entries")
            tp = self._t_host.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        _check(L.mgwr_plan_create(ctypes.byref(p), tp, ctypes.byref(handle)))
        self._h = handle
        self._ws = None
        self._stream = None

    # -- host facts ---------------------------------------------------------
    def info(self):
        inf = PlanInfo()
        _check(lib().mgwr_plan_get_info(self._h, ctypes.byref(inf)))
        return inf.as_dict()

    def mesh(self):
        import numpy as np
        t = np.empty(self.M + 1)
        a1 = np.empty(self.M)
        _check(lib().mgwr_plan_get_mesh(self._h, t.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                        a1.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return t, a1

    def export_dense(self):
        import numpy as np
        R = np.empty((self.M, self.M))
        _check(lib().mgwr_plan_export_dense(self._h, R.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return R

    def workspace_bytes(self):
        b = ctypes.c_size_t()
        _check(lib().mgwr_plan_workspace_bytes(self._h, ctypes.byref(b)))
        return b.value

    # -- device ---------------------------------------------------------------
    def bind(self, device=None, stream=None):
        import torch
        dev = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        with torch.cuda.device(dev):
            nbytes = self.workspace_bytes()
            self._ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
            base = self._ws.data_ptr()
            aligned = (base + 255) & ~255
            self._stream = torch.cuda.current_stream(dev) if stream is None else stream
            _check(lib().mgwr_plan_bind(self._h, ctypes.c_void_p(aligned), nbytes,
                                        ctypes.c_void_p(self._stream.cuda_stream)))
        self.device = dev
        return self

    def autotune(self, f, g=None, tol=1e-8, u=None):
        """Measure the schedules (and the staged schedule's prefetch and
        coarse level, see tuned()) on f and keep the fastest, also for later
        plans of the same shape; returns "staged" or "pipelined"."""
        import torch
        _require(f, "f", (self.M, self.N))
        if g is not None:
            _require(g, "g", (self.N,))
        if u is None:
            u = torch.empty_like(f)
        chosen = ctypes.c_int()
        _check(lib().mgwr_plan_autotune(self._h, _dptr(f), _dptr(g), float(tol), _dptr(u), ctypes.byref(chosen)))
        return {1: "staged", 2: "pipelined"}[chosen.value]

    def set_warm_start(self, net, rows):
        """Attach a bound Net as the initial-guess predictor (rows: the time
        rows of its input/output slices)."""
        rows = [int(r) for r in rows]
        arr = (ctypes.c_int * len(rows))(*rows)
        _check(lib().mgwr_plan_set_warm_start(self._h, None if net is None else net._h, len(rows), arr))
        self._net = net

    def solve(self, f, g=None, tol=1e-10, u=None, guess=False, allow_unconverged=False, warm_start=False,
              warm_res0=False):
        """warm_start: start from the attached network's prediction;
        warm_res0: also evaluate that prediction's float64 residual."""
        import torch
        _require(f, "f", (self.M, self.N))
        if g is not None:
            _require(g, "g", (self.N,))
        if u is None:
            u = torch.empty((self.M, self.N), dtype=torch.float64, device=f.device)
        _require(u, "u", (self.M, self.N))
        st = Stats()
        fl = ((MGWR_GUESS_IN_U if guess else 0) | (MGWR_WARM_START if warm_start else 0) |
              (MGWR_WARM_RES0 if warm_res0 else 0))
        rc = lib().mgwr_solve(self._h, _dptr(f), _dptr(g), float(tol), _dptr(u), fl, ctypes.byref(st))
        _check(rc, ok=(MGWR_OK, MGWR_ERR_NOT_CONVERGED) if allow_unconverged else (MGWR_OK,))
        return u, st.as_dict()

    def solve_static(self, f, g=None, tol=1e-10, u=None, guess=False, allow_unconverged=False, stream=None):
        """mgwr_solve with the library's static device array as the workspace
        (no allocation by the library; the plan need not be bound)."""
        import torch
        _require(f, "f", (self.M, self.N))
        if g is not None:
            _require(g, "g", (self.N,))
        if u is None:
            u = torch.empty((self.M, self.N), dtype=torch.float64, device=f.device)
        _require(u, "u", (self.M, self.N))
        if stream is None:
            stream = torch.cuda.current_stream(f.device)
        st = Stats()
        fl = MGWR_GUESS_IN_U if guess else 0
        rc = lib().mgwr_solve_static(self._h, ctypes.c_void_p(stream.cuda_stream), _dptr(f), _dptr(g), float(tol),
                                     _dptr(u), fl, ctypes.byref(st))
        _check(rc, ok=(MGWR_OK, MGWR_ERR_NOT_CONVERGED) if allow_unconverged else (MGWR_OK,))
        return u, st.as_dict()

    def residual(self, f, u, g=None, out=None, want_norm=True):
        _require(f, "f", (self.M, self.N))
        _require(u, "u", (self.M, self.N))
        if g is not None:
            _require(g, "g", (self.N,))
        if out is not None:
            _require(out, "out", (self.M, self.N))
        nrm = ctypes.c_double(0.0)
        _check(lib().mgwr_residual(self._h, _dptr(f), _dptr(g), _dptr(u), _dptr(out),
                                   ctypes.byref(nrm) if want_norm else None))
        return out, (nrm.value if want_norm else None)

    def hmatvec(self, x, y=None):
        import torch
        ncols = x.shape[1]
        _require(x, "x", (self.M, ncols))
        if y is None:
            y = torch.empty_like(x)
        _require(y, "y", (self.M, ncols))
        _check(lib().mgwr_hmatvec(self._h, _dptr(x), _dptr(y), int(ncols)))
        return y

    def apply_A(self, u, out=None):
        """out = A u (the float64 space-time operator: R~ in time plus the
        spatial stencil)."""
        import torch
        _require(u, "u", (self.M, self.N))
        if out is None:
            out = torch.empty_like(u)
        _require(out, "out", (self.M, self.N))
        _check(lib().mgwr_apply_A(self._h, _dptr(u), _dptr(out)))
        return out

    def load_model(self, net, blob):
        """Load a weight blob (model_blob) into the bound Net and attach it for
        warm-started solves (mgwr_model_load)."""
        blob = bytes(blob)
        _check(lib().mgwr_model_load(self._h, None if net is None else net._h, blob, len(blob)))
        self._net = net

    def htrsm(self, b, level=0, x=None):
        import torch
        ncols = b.shape[1]
        _require(b, "b", (self.M, ncols))
        if x is None:
            x = torch.empty_like(b)
        _require(x, "x", (self.M, ncols))
        _check(lib().mgwr_htrsm(self._h, int(level), _dptr(b), _dptr(x), int(ncols)))
        return x

    def timing(self, enable=None):
        """enable=True/False switches live event timing (True clears it);
        enable=None returns the accumulated per-kernel-class counters."""
        if enable is not None:
            _check(lib().mgwr_timing_enable(self._h, 1 if enable else 0))
            return None
        tm = Timing()
        _check(lib().mgwr_timing_get(self._h, ctypes.byref(tm)))
        return tm.as_dict()

    def set_staging(self, prefetch: int = 0, coarse_level: int = -1):
        """Staged-schedule knobs: march prefetch (0 by mesh length, 1 shallow,
        2 deep) and the level the coarse pipelined launch starts at (-1 by
        rule, 0 none)."""
        _check(lib().mgwr_plan_set_staging(self._h, int(prefetch), int(coarse_level)))
        return self

    LAYOUTS = {"auto": -1, "natural": 0, "split": 1}

    def set_layout(self, layout: str = "auto"):
        """Storage of a 2D plan's arrays inside its solves: "split" (each
        time row holds the first colour's points, then the second's),
        "natural", or "auto" (the autotuner's choice, else split).  The
        caller's arrays are always in natural order."""
        if layout not in self.LAYOUTS:
            raise ValueError(f"layout must be one of {sorted(self.LAYOUTS)}")
        _check(lib().mgwr_plan_set_layout(self._h, self.LAYOUTS[layout]))
        return self

    def tuned(self):
        """{"schedule", "prefetch", "coarse_level"} a solve uses now."""
        s, p, c = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check(lib().mgwr_plan_tuned(self._h, ctypes.byref(s), ctypes.byref(p), ctypes.byref(c)))
        return {"schedule": {1: "staged", 2: "pipelined"}[s.value],
                "prefetch": {0: "by_length", 1: "shallow", 2: "deep"}[p.value], "coarse_level": c.value}

    def xcd_queues_in_use(self):
        """Whether this (bound) plan's pipelined launches deal their work
        items to per-XCD queues."""
        v = ctypes.c_int()
        _check(lib().mgwr_xcd_queues_in_use(self._h, ctypes.byref(v)))
        return bool(v.value)

    def set_progress_limit(self, polls: int):
        """Bound on the polls of one progress wait of a pipelined launch
        (default 4194304); beyond it the solve fails with MGWR_ERR_HIP."""
        _check(lib().mgwr_plan_set_progress_limit(self._h, int(polls)))
        return self

    def close(self):
        if getattr(self, "_h", None):
            lib().mgwr_plan_destroy(self._h)
            self._h = None
        self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Several bound plans solved together: the instances with a pipelined
    schedule in one merged launch (replayed from a HIP graph when `graph`
    is on and nothing changed), the others side by side on worker streams
    (one by one when two entries share a plan, or for warm-started solves)."""

    def __init__(self, plans, graph=False):
        self.plans = list(plans)
        arr = (ctypes.c_void_p * len(self.plans))(*[p._h.value for p in self.plans])
        h = ctypes.c_void_p()
        _check(lib().mgwr_batch_create(len(self.plans), arr, ctypes.byref(h)))
        self._h = h
        self._ws = None
        self.set_graph(graph)

    def set_graph(self, enable):
        _check(lib().mgwr_batch_set_graph(self._h, 1 if enable else 0))

    def graph_replays(self):
        n = ctypes.c_longlong()
        _check(lib().mgwr_batch_graph_replays(self._h, ctypes.byref(n)))
        return n.value

    def bind(self, stream=None):
        import torch
        dev = self.plans[0].device
        with torch.cuda.device(dev):
            b = ctypes.c_size_t()
            _check(lib().mgwr_batch_workspace_bytes(self._h, ctypes.byref(b)))
            self._ws = torch.empty(b.value + 256, dtype=torch.uint8, device=dev)
            aligned = (self._ws.data_ptr() + 255) & ~255
            self._stream = torch.cuda.current_stream(dev) if stream is None else stream
            _check(lib().mgwr_batch_bind(self._h, ctypes.c_void_p(aligned), b.value,
                                         ctypes.c_void_p(self._stream.cuda_stream)))
        return self

    def solve(self, fs, gs=None, tol=1e-10, us=None, guess=False, allow_unconverged=False, warm_start=False,
              warm_res0=False):
        import torch
        n = len(self.plans)
        if us is None:
            us = [torch.empty((p.M, p.N), dtype=torch.float64, device=f.device) for p, f in zip(self.plans, fs)]
        for p, f, u in zip(self.plans, fs, us):
            _require(f, "f", (p.M, p.N))
            _require(u, "u", (p.M, p.N))
        fa = (ctypes.c_void_p * n)(*[f.data_ptr() for f in fs])
        ua = (ctypes.c_void_p * n)(*[u.data_ptr() for u in us])
        ga = None
        if gs is not None:
            for p, g in zip(self.plans, gs):
                if g is not None:
                    _require(g, "g", (p.N,))
            ga = (ctypes.c_void_p * n)(*[None if g is None else g.data_ptr() for g in gs])
        st = (Stats * n)()
        fl = ((MGWR_GUESS_IN_U if guess else 0) | (MGWR_WARM_START if warm_start else 0) |
              (MGWR_WARM_RES0 if warm_res0 else 0))
        rc = lib().mgwr_batch_solve(self._h, fa, ga, float(tol), ua, fl, st)
        _check(rc, ok=(MGWR_OK, MGWR_ERR_NOT_CONVERGED) if allow_unconverged else (MGWR_OK,))
        return us, [s.as_dict() for s in st]

    def timing(self, enable=None):
        tm = Timing()
        _check(lib().mgwr_batch_timing(self._h, -1 if enable is None else (1 if enable else 0), ctypes.byref(tm)))
        return tm.as_dict()

    def close(self):
        if getattr(self, "_h", None):
            lib().mgwr_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Net:
    """Band-pyramid convolution network of the learned initial guess.

    `channels` = [c_0, ..., c_L] of the 3x3 convolution stack; the input
    tensor has c_0 - 1 channels, the first `nsignal` of which are split into
    spatial bands (the last one of c_0 is the level value the library adds).
    Weights live in the float32 tensor `params` (master copy); the library
    keeps bfloat16 copies for the forward and data-gradient passes."""

    def __init__(self, channels, nsignal, max_bhw, device=None, seed=0):
        import torch
        self.channels = [int(c) for c in channels]
        self.nsignal = int(nsignal)
        arr = (ctypes.c_int * len(self.channels))(*self.channels)
        h = ctypes.c_void_p()
        _check(lib().mgwr_net_create(len(self.channels) - 1, arr, self.nsignal, ctypes.byref(h)))
        self._h = h
        n = ctypes.c_size_t()
        _check(lib().mgwr_net_param_count(self._h, ctypes.byref(n)))
        self.nparam = n.value
        dev = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        self.params = torch.zeros(self.nparam, dtype=torch.float32, device=dev)
        b = ctypes.c_size_t()
        _check(lib().mgwr_net_workspace_bytes(self._h, int(max_bhw), ctypes.byref(b)))
        self._ws = torch.empty(b.value + 256, dtype=torch.uint8, device=dev)
        aligned = (self._ws.data_ptr() + 255) & ~255
        self._stream = torch.cuda.current_stream(dev)
        _check(lib().mgwr_net_bind(self._h, ctypes.c_void_p(self.params.data_ptr()), int(max_bhw),
                                   ctypes.c_void_p(aligned), b.value, ctypes.c_void_p(self._stream.cuda_stream)))
        self.max_bhw = int(max_bhw)
        self.step = 0
        self.init_params(seed)

    @property
    def in_channels(self):
        return self.channels[0] - 1

    def layout(self):
        """[(weight offset, weight shape, bias offset, bias size)] per layer."""
        out, off = [], 0
        for cin, cout in zip(self.channels[:-1], self.channels[1:]):
            out.append((off, (cout, cin, 3, 3), off + cout * cin * 9, cout))
            off += cout * cin * 9 + cout
        return out

    def init_params(self, seed=0):
        """Uniform weights with variance 1/fan_in, zero biases (host RNG)."""
        import numpy as np
        host = np.zeros(self.nparam, dtype=np.float32)
        rng = np.random.default_rng(seed)
        for woff, shape, boff, nb in self.layout():
            cnt = int(np.prod(shape))
            host[woff:woff + cnt] = rng.uniform(-1, 1, cnt) * np.sqrt(3.0 / (shape[1] * 9))
        self.set_params(host)

    def set_params(self, values):
        import torch
        self.params.copy_(torch.as_tensor(values, dtype=torch.float32))
        _check(lib().mgwr_net_sync_weights(self._h))
        self.step = 0

    def set_finest(self, h_min):
        """Leave out the bands finer than spacing h_min (0 keeps all)."""
        _check(lib().mgwr_net_set_finest(self._h, float(h_min)))
        self.h_min = float(h_min)

    def forward(self, x, h):
        import torch
        B, C, H, W = x.shape
        _require(x, "x", (B, self.in_channels, H, W), torch.float32)
        y = torch.empty((B, self.channels[-1], H, W), dtype=torch.float32, device=x.device)
        _check(lib().mgwr_net_forward(self._h, _dptr(x), B, H, W, float(h), _dptr(y)))
        return y

    def gradient(self, x, target, h):
        import torch
        B, C, H, W = x.shape
        _require(x, "x", (B, self.in_channels, H, W), torch.float32)
        _require(target, "target", (B, self.channels[-1], H, W), torch.float32)
        g = torch.empty(self.nparam, dtype=torch.float32, device=x.device)
        loss = ctypes.c_double()
        _check(lib().mgwr_net_gradient(self._h, _dptr(x), _dptr(target), B, H, W, float(h), _dptr(g),
                                       ctypes.byref(loss)))
        return loss.value, g

    def train_step(self, x, target, h, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, want_loss=False):
        import torch
        B, C, H, W = x.shape
        _require(x, "x", (B, self.in_channels, H, W), torch.float32)
        _require(target, "target", (B, self.channels[-1], H, W), torch.float32)
        loss = ctypes.c_double()
        _check(lib().mgwr_net_gradient(self._h, _dptr(x), _dptr(target), B, H, W, float(h), None,
                                       ctypes.byref(loss) if want_loss else None))
        self.step += 1
        _check(lib().mgwr_net_adam_step(self._h, float(lr), float(beta1), float(beta2), float(eps), self.step))
        return loss.value if want_loss else None

    def close(self):
        if getattr(self, "_h", None):
            lib().mgwr_net_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _fnv1a64(data: bytes) -> int:
    """64-bit FNV-1a (the weight blob's checksum)."""
    h = 0xcbf29ce484222325
    for byte in memoryview(data).cast("B"):
        h = ((h ^ byte) * 0x100000001b3) & 0xFFFFFFFFFFFFFFFF
    return h


def model_blob(channels, nsignal, rows, h_min, params) -> bytes:
    """Serialise network weights into the self-describing blob that
    mgwr_model_load reads (layout in include/mgwr.h)."""
    import struct

    import numpy as np
    ch = [int(c) for c in channels]
    rows = [int(r) for r in rows]
    w = np.ascontiguousarray(np.asarray(params, dtype="<f4"))
    body = b"MGWRNET1" + struct.pack("<ii", 1, len(ch) - 1) + struct.pack(f"<{len(ch)}i", *ch)
    body += struct.pack("<ii", int(nsignal), len(rows)) + struct.pack(f"<{len(rows)}i", *rows)
    body += struct.pack("<dq", float(h_min), int(w.size)) + w.tobytes()
    return body + struct.pack("<Q", _fnv1a64(body))


def set_xcd_queues(enable: bool) -> bool:
    """Per-XCD work queues of the pipelined launches (process-wide, on by
    default); returns the previous setting."""
    prev = ctypes.c_int()
    _check(lib().mgwr_set_xcd_queues(1 if enable else 0, ctypes.byref(prev)))
    return bool(prev.value)


def describe_model(blob):
    """Shape of a weight blob as the library reads it (raises MgwrError with
    code MGWR_ERR_MODEL if it is missing or corrupt)."""
    blob = bytes(blob) if blob is not None else b""
    info = ModelInfo()
    _check(lib().mgwr_model_describe(blob if blob else None, len(blob), ctypes.byref(info)))
    return info.as_dict()
