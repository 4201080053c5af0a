"""ctypes binding of ``libhipmsat.so`` (declared in ``include/hipmsat.h``).

Argument marshalling only: every step of the solve loop runs in the HIP
library.  PyTorch provides device tensors and the current stream.  Loading
fails loudly when the built library is missing; there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
import threading
from dataclasses import dataclass, field

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
# HIPMSAT_LIB names another build of the same library (the sanitized host build)
LIB_PATH = os.environ.get("HIPMSAT_LIB") or os.path.join(_PKG, "libhipmsat.so")

HMS_OK = 0
ERRORS = {
    -1: "HMS_ERR_ARG", -2: "HMS_ERR_PARSE", -3: "HMS_ERR_LITERAL_RANGE", -4: "HMS_ERR_DEVICE",
    -5: "HMS_ERR_NOMEM", -6: "HMS_ERR_NONFINITE", -7: "HMS_ERR_CANCELLED", -8: "HMS_ERR_IO",
    -9: "HMS_ERR_TOO_LARGE",
}
ADAM, SGD = 0, 1
LOSS_UNSAT, LOSS_ALL = 0, 1

# schedule id of the resident solver (whole loop in one workgroup per restart);
# other ids are a kernel table index | rows per work unit << 8
RESIDENT = 255


class HipMsatError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code
        self.name = ERRORS.get(code, str(code))


class CnfInfo(C.Structure):
    _fields_ = [("n_vars", C.c_int32), ("n_clauses", C.c_int32), ("n_lits", C.c_int64),
                ("nnz", C.c_int64), ("n_empty", C.c_int32), ("n_taut", C.c_int32),
                ("n_active", C.c_int32), ("n_heavy", C.c_int32), ("struct_bytes", C.c_int64),
                ("state_bytes_r1", C.c_int64), ("weighted", C.c_int32), ("total_weight", C.c_int64),
                ("plan_threads", C.c_int32), ("slot_bytes", C.c_int64)]


class SolveState(C.Structure):
    _fields_ = [("x", C.c_void_p), ("m", C.c_void_p), ("v", C.c_void_p), ("best_assignment", C.c_void_p),
                ("best", C.c_void_p), ("best_step", C.c_void_p), ("step", C.c_int32), ("pad", C.c_int32)]


class SolveParams(C.Structure):
    _fields_ = [("steps", C.c_int32), ("restarts", C.c_int32), ("eval_every", C.c_int32),
                ("optimizer", C.c_int32), ("seed", C.c_uint64), ("lr", C.c_float),
                ("beta1", C.c_float), ("beta2", C.c_float), ("eps", C.c_float),
                ("loss_mode", C.c_int32), ("schedule", C.c_int32), ("use_graph", C.c_int32),
                ("autotune", C.c_int32), ("time_limit_s", C.c_double), ("x0", C.c_void_p),
                ("stream", C.c_void_p), ("cancel", C.c_void_p), ("resume", C.c_void_p)]


class SolveResult(C.Structure):
    _fields_ = [("best_cost", C.c_int64), ("best_restart", C.c_int32), ("best_step", C.c_int32),
                ("steps_done", C.c_int32), ("schedule", C.c_int32), ("final_loss", C.c_double),
                ("best_assignment", C.c_void_p), ("restart_best", C.c_void_p),
                ("restart_step", C.c_void_p), ("restart_loss", C.c_void_p),
                ("x_final", C.c_void_p), ("device_ms", C.c_double), ("state", C.c_void_p),
                ("trace", C.c_void_p), ("trace_cap", C.c_int32), ("trace_len", C.c_int32)]


# hms_trace_point: one counted iterate of one restart
TRACE_DTYPE = np.dtype([("step", np.int32), ("pad", np.int32), ("cost", np.int64), ("loss", np.float64)])


class PlanView(C.Structure):
    _fields_ = [("n", C.c_int32), ("m", C.c_int32), ("mk", C.c_int32), ("c_tiles", C.c_int32),
                ("n_act", C.c_int32), ("n_heavy", C.c_int32), ("seg_rows", C.c_int32),
                ("seg_tiles", C.c_int32), ("v_tiles", C.c_int32), ("n_empty", C.c_int32),
                ("n_taut", C.c_int32), ("tile_rows", C.c_int32), ("seg_len", C.c_int32), ("split_len", C.c_int32),
                ("nnz", C.c_int64), ("c_ent_len", C.c_int64), ("v_ent_len", C.c_int64),
                ("c_tile", C.c_void_p), ("c_ent", C.c_void_p), ("c_row_orig", C.c_void_p),
                ("v_tile", C.c_void_p), ("v_ent", C.c_void_p), ("seg_first", C.c_void_p),
                ("seg_row", C.c_void_p), ("var_old", C.c_void_p), ("c_slot", C.c_void_p),
                ("priv", C.c_void_p)]


EXPORTS = ["hms_load_cnf", "hms_load_cnf_dimacs", "hms_cnf_info_get", "hms_free_cnf",
           "hms_solve_params_default", "hms_solve", "hms_evaluate", "hms_eval_relaxed",
           "hms_last_error", "hms_version", "hms_plan_view_build", "hms_plan_view_free",
           "hms_time_kernels", "hms_tune", "hms_adjoint_bytes", "hms_forward", "hms_backward",
           "hms_solve_batch", "hms_tune_candidates", "hms_load_wcnf", "hms_eval_relaxed_noalloc",
           "hms_schedule_count", "hms_cnf_slot_map"]

_lib = None
_lib_lock = threading.Lock()


def lib():
    """Load the library (raises if it has not been built)."""
    if _lib is not None:
        return _lib
    with _lib_lock:
        return _lib if _lib is not None else _load()


def _load():
    global _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2402_03640_amd.build`")
    # torch first: it brings its own HIP runtime (same soname), which the
    # library then binds to, so the process holds one runtime whatever the
    # import order of the caller (a runtime loaded ahead of torch's bundled
    # libraries can leave the device unusable)
    import torch  # noqa: F401
    L = C.CDLL(LIB_PATH)
    P, I32, I64 = C.c_void_p, C.c_int32, C.c_int64
    L.hms_load_cnf.argtypes = [I32, P, I64, P, C.POINTER(P)]
    L.hms_load_cnf_dimacs.argtypes = [C.c_char_p, P, C.POINTER(P)]
    L.hms_load_wcnf.argtypes = [I32, P, I64, P, P, C.POINTER(P)]
    L.hms_cnf_info_get.argtypes = [P, C.POINTER(CnfInfo)]
    L.hms_free_cnf.argtypes = [P]
    L.hms_free_cnf.restype = None
    L.hms_solve_params_default.argtypes = [C.POINTER(SolveParams)]
    L.hms_solve_params_default.restype = None
    L.hms_solve.argtypes = [P, C.POINTER(SolveParams), C.POINTER(SolveResult)]
    L.hms_evaluate.argtypes = [P, P, P, P]
    L.hms_time_kernels.argtypes = [P, C.POINTER(SolveParams), I32, P, P, P]
    L.hms_tune.argtypes = [P, C.POINTER(SolveParams), I32, P, P]
    L.hms_adjoint_bytes.argtypes = [P, I32, P]
    L.hms_solve_batch.argtypes = [P, P, I32, P, P]
    L.hms_forward.argtypes = [P, P, I32, I32, P, P, P, P]
    L.hms_backward.argtypes = [P, P, I32, I32, P, P, P, P]
    L.hms_eval_relaxed.argtypes = [P, P, I32, I32, P, P, P, P]
    L.hms_eval_relaxed_noalloc.argtypes = [P, P, I32, I32, P, P, P, P]
    L.hms_last_error.argtypes = []
    L.hms_last_error.restype = C.c_char_p
    L.hms_version.argtypes = []
    L.hms_version.restype = C.c_char_p
    L.hms_plan_view_build.argtypes = [I32, P, I64, C.POINTER(PlanView)]
    L.hms_plan_view_free.argtypes = [C.POINTER(PlanView)]
    L.hms_cnf_slot_map.argtypes = [P, P, I64, P]
    L.hms_cnf_slot_map.restype = I32
    L.hms_plan_view_free.restype = None
    L.hms_tune_candidates.argtypes = [I32, I32, P, I32, P]
    L.hms_schedule_count.argtypes = []
    L.hms_schedule_count.restype = I32
    for name in ("hms_load_cnf", "hms_load_wcnf", "hms_load_cnf_dimacs", "hms_cnf_info_get", "hms_solve",
                 "hms_evaluate", "hms_eval_relaxed", "hms_eval_relaxed_noalloc", "hms_plan_view_build", "hms_time_kernels", "hms_tune", "hms_adjoint_bytes",
                 "hms_forward", "hms_backward", "hms_solve_batch", "hms_tune_candidates"):
        getattr(L, name).restype = I32
    _lib = L
    return L


def _check(rc: int):
    if rc != HMS_OK:
        raise HipMsatError(rc, lib().hms_last_error().decode())


def _stream_ptr(stream):
    """hipStream_t of a torch stream (default: torch's current stream)."""
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(stream.cuda_stream)


def _lits(lits) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(lits, dtype=np.int32))


def _device_points(x, cnf, name: str):
    """x as its [n][R] view, after checking it can be handed to the kernels:
    a contiguous float32 tensor on the instance's device with n rows."""
    import torch
    if not isinstance(x, torch.Tensor) or not x.is_cuda or x.dtype != torch.float32:
        raise TypeError(f"{name} must be a float32 tensor on the GPU")
    if x.device.index != cnf.device:
        raise ValueError(f"{name} is on device {x.device.index}, the instance on device {cnf.device}")
    if not x.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    X = x if x.dim() == 2 else (x.view(-1, 1) if x.dim() == 1 else None)
    if X is None or X.shape[0] != cnf.n or X.shape[1] < 1:
        raise ValueError(f"{name} must have shape [{cnf.n}] or [{cnf.n}][R], got {tuple(x.shape)}")
    return X


class Cnf:
    """A loaded instance (owns its device structure)."""

    def __init__(self, handle: C.c_void_p):
        self._h = handle
        info = CnfInfo()
        _check(lib().hms_cnf_info_get(self._h, C.byref(info)))
        self.info = {k: getattr(info, k) for k, _ in CnfInfo._fields_}
        self.n = info.n_vars
        self.m = info.n_clauses
        import torch
        self.device = torch.cuda.current_device()  # where the library put the instance

    @property
    def handle(self):
        return self._h

    def slot_map(self) -> np.ndarray:
        """The occurrence map built on the device (layout tests; see
        ``hms_cnf_slot_map``); empty when the instance has none."""
        n = C.c_int64()
        _check(lib().hms_cnf_slot_map(self._h, None, 0, C.byref(n)))
        out = np.zeros(n.value, dtype=np.uint32)
        if n.value:
            _check(lib().hms_cnf_slot_map(self._h, out.ctypes.data_as(C.c_void_p), out.size, C.byref(n)))
        return out

    def free(self):
        if self._h is not None and self._h.value:
            lib().hms_free_cnf(self._h)
        self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.free()


def load_cnf(n_vars: int, lits, stream=None, weights=None) -> Cnf:
    """Load a DIMACS-style flat literal array (clauses ended by 0); `weights`
    (one positive integer per clause) makes it a weighted MaxSAT instance."""
    a = _lits(lits)
    h = C.c_void_p()
    if weights is not None:
        w = np.ascontiguousarray(weights, dtype=np.int64)
        m = int(np.count_nonzero(a == 0))
        if w.ndim != 1 or w.size != m:
            raise ValueError(f"{w.size} clause weights for {m} clauses")
    if weights is None:
        _check(lib().hms_load_cnf(int(n_vars), a.ctypes.data_as(C.c_void_p), a.size,
                                  _stream_ptr(stream), C.byref(h)))
    else:
        _check(lib().hms_load_wcnf(int(n_vars), a.ctypes.data_as(C.c_void_p), a.size,
                                   w.ctypes.data_as(C.c_void_p), _stream_ptr(stream), C.byref(h)))
    return Cnf(h)


def load_cnf_dimacs(path: str, stream=None) -> Cnf:
    h = C.c_void_p()
    _check(lib().hms_load_cnf_dimacs(os.fsencode(path), _stream_ptr(stream), C.byref(h)))
    return Cnf(h)


@dataclass
class SolverState:
    """The state Algorithm 1 carries between iterations (``hms_solve_state``):
    relaxed values and Adam moments (device float32 [n][R]), each restart's
    best rounded iterate (device uint8 [R][n]), its cost and step (host), and
    the iterations taken.  ``solve(..., want_state=True)`` returns one;
    ``solve(..., resume=state)`` continues from it."""
    x: object
    m: object
    v: object
    best_assignment: object
    best: np.ndarray
    best_step: np.ndarray
    step: int

    @classmethod
    def empty(cls, n: int, restarts: int):
        import torch
        R = int(restarts)
        f = lambda: torch.empty((n, R), dtype=torch.float32, device="cuda")  # noqa: E731
        return cls(f(), f(), f(), torch.empty((R, n), dtype=torch.uint8, device="cuda"),
                   np.zeros(R, dtype=np.int64), np.zeros(R, dtype=np.int32), 0)

    def _struct(self) -> SolveState:
        st = SolveState()
        for k in ("x", "m", "v", "best_assignment"):
            t = getattr(self, k)
            setattr(st, k, None if t is None else t.data_ptr())
        for k, dt in (("best", np.int64), ("best_step", np.int32)):
            a = np.ascontiguousarray(getattr(self, k), dtype=dt)
            setattr(self, k, a)
            setattr(st, k, a.ctypes.data)
        st.step = int(self.step)
        return st


@dataclass
class SolveOutput:
    best_cost: int
    best_restart: int
    best_step: int
    steps_done: int
    schedule: int
    final_loss: float
    device_ms: float
    best_assignment: np.ndarray
    restart_best: np.ndarray
    restart_step: np.ndarray
    restart_loss: np.ndarray
    x_final: object = field(default=None)
    state: object = field(default=None)
    trace: object = field(default=None)  # [counts][R] TRACE_DTYPE records, oldest first


def _params(cnf, steps, restarts, eval_every, seed, optimizer, lr, beta1, beta2, eps, loss_mode,
            schedule, use_graph, time_limit_s, x0, stream, autotune=True):
    R = int(restarts)
    p = SolveParams()
    lib().hms_solve_params_default(C.byref(p))
    p.steps, p.restarts, p.eval_every, p.optimizer = int(steps), R, int(eval_every), int(optimizer)
    p.seed = int(seed) & (2 ** 64 - 1)
    p.lr, p.beta1, p.beta2, p.eps = lr, beta1, beta2, eps
    p.loss_mode, p.schedule, p.use_graph = int(loss_mode), int(schedule), int(bool(use_graph))
    p.time_limit_s = float(time_limit_s)
    p.autotune = int(bool(autotune))
    if x0 is not None:
        X0 = _device_points(x0, cnf, "x0")
        if X0.shape[1] != R:
            raise ValueError(f"x0 has {X0.shape[1]} columns for {R} restarts")
        p.x0 = X0.data_ptr()
    p.stream = _stream_ptr(stream)
    return p


def time_kernels(cnf: Cnf, restarts: int = 1, iters: int = 50, seed: int = 0, optimizer: int = ADAM,
                 lr: float = 1e-4, loss_mode: int = LOSS_UNSAT, schedule: int = 0, stream=None):
    """Average device ms per launch of the forward kernel, the backward kernels
    and a whole step (HIP events on the launch stream)."""
    p = _params(cnf, 1, restarts, 1, seed, optimizer, lr, 0.9, 0.999, 1e-8, loss_mode, schedule,
                False, 0.0, None, stream)
    f, b, st = C.c_double(), C.c_double(), C.c_double()
    _check(lib().hms_time_kernels(cnf.handle, C.byref(p), int(iters), C.byref(f), C.byref(b),
                                  C.byref(st)))
    return f.value, b.value, st.value


def tune(cnf: Cnf, restarts: int = 1, iters: int = 6, optimizer: int = ADAM, lr: float = 1e-4,
         loss_mode: int = LOSS_UNSAT, stream=None, eval_every: int = 1):
    """Time every schedule for this restart count; returns (schedule id, ms per step).
    ``eval_every`` is the counting period the resident solver is timed with."""
    p = _params(cnf, 1, restarts, int(eval_every), 0, optimizer, lr, 0.9, 0.999, 1e-8, loss_mode, 0, False, 0.0,
                None, stream)
    code, ms = C.c_int32(), C.c_double()
    _check(lib().hms_tune(cnf.handle, C.byref(p), int(iters), C.byref(code), C.byref(ms)))
    return code.value, ms.value


def tune_candidates(restarts: int = 1, loss_mode: int = LOSS_UNSAT) -> list[int]:
    """Schedule ids the autotuner times for this restart count (host only)."""
    cnt = C.c_int32()
    _check(lib().hms_tune_candidates(int(restarts), int(loss_mode), None, 0, C.byref(cnt)))
    buf = (C.c_int32 * max(cnt.value, 1))()
    _check(lib().hms_tune_candidates(int(restarts), int(loss_mode), C.cast(buf, C.c_void_p), cnt.value,
                                     C.byref(cnt)))
    return [int(buf[i]) for i in range(cnt.value)]


def schedule_count() -> int:
    """Number of kernel table entries: schedule table indices are 1..count."""
    return int(lib().hms_schedule_count())


class CancelFlag:
    """A host flag a running ``solve`` polls at its counting boundaries; set
    it from another thread to stop the solve (HMS_ERR_CANCELLED, with the
    best so far on the raised error's ``result``)."""

    def __init__(self):
        self._v = C.c_int32(0)

    def set(self):
        self._v.value = 1

    @property
    def address(self):
        return C.addressof(self._v)


def solve(cnf: Cnf, steps: int = 1000, restarts: int = 1, eval_every: int = 1, seed: int = 0,
          optimizer: int = ADAM, lr: float = 1e-4, beta1: float = 0.9, beta2: float = 0.999,
          eps: float = 1e-8, loss_mode: int = LOSS_UNSAT, schedule: int = 0, use_graph: bool = True,
          time_limit_s: float = 0.0, x0=None, want_x: bool = False, stream=None,
          autotune: bool = True, cancel: CancelFlag | None = None, resume: SolverState | None = None,
          want_state: bool = False, trace_cap: int = 0) -> SolveOutput:
    """Algorithm 1 over ``restarts`` relaxed points (see ``hms_solve``).
    ``resume`` continues from a ``SolverState``; ``want_state`` returns the
    state after the last step as ``output.state``; ``trace_cap`` > 0 returns
    the (step, cost, loss) of the last ``trace_cap`` counted iterates of each
    restart as ``output.trace`` ([counts][R] records of TRACE_DTYPE)."""
    R = int(restarts)
    p = _params(cnf, steps, restarts, eval_every, seed, optimizer, lr, beta1, beta2, eps, loss_mode,
                schedule, use_graph, time_limit_s, x0, stream, autotune)
    if cancel is not None:
        p.cancel = cancel.address
    keep = []  # structs and arrays the call reads, alive until it returns
    if resume is not None:
        for k in ("x", "m", "v"):
            t = getattr(resume, k)
            if t is not None:
                _device_points(t, cnf, f"resume.{k}")
                if t.view(cnf.n, -1).shape[1] != R:
                    raise ValueError(f"resume.{k} has {t.view(cnf.n, -1).shape[1]} columns for {R} restarts")
        ba = resume.best_assignment
        if ba is not None and (not ba.is_cuda or ba.dtype.itemsize != 1 or not ba.is_contiguous()
                               or ba.numel() != R * cnf.n):
            raise ValueError(f"resume.best_assignment must be a contiguous byte tensor of {R} x {cnf.n} on the GPU")
        rstruct = resume._struct()
        keep.append(rstruct)
        p.resume = C.addressof(rstruct)
    res = SolveResult()
    trace = None
    if trace_cap:
        trace = np.zeros((int(trace_cap), R), dtype=TRACE_DTYPE)
        res.trace = trace.ctypes.data
        res.trace_cap = int(trace_cap)
    out_state = None
    if want_state:
        out_state = SolverState.empty(cnf.n, R)
        if optimizer != ADAM:
            out_state.m = out_state.v = None
        ostruct = out_state._struct()
        keep.append(ostruct)
        res.state = C.addressof(ostruct)
    ba = np.zeros(max(cnf.n, 1), dtype=np.uint8)
    rb = np.zeros(R, dtype=np.int64)
    rs = np.zeros(R, dtype=np.int32)
    rl = np.zeros(R, dtype=np.float64)
    res.best_assignment = ba.ctypes.data
    res.restart_best = rb.ctypes.data
    res.restart_step = rs.ctypes.data
    res.restart_loss = rl.ctypes.data
    xf = None
    if want_x:
        import torch
        xf = torch.empty((cnf.n, R), dtype=torch.float32, device="cuda")
        res.x_final = xf.data_ptr()
    rc = lib().hms_solve(cnf.handle, C.byref(p), C.byref(res))
    if rc != HMS_OK and rc not in (-6, -7):
        _check(rc)
    if out_state is not None:
        out_state.step = int(ostruct.step)
    out = SolveOutput(res.best_cost, res.best_restart, res.best_step, res.steps_done, res.schedule,
                      res.final_loss, res.device_ms, ba[:cnf.n].copy(), rb, rs, rl, xf, out_state,
                      None if trace is None else trace[:res.trace_len].copy())
    if rc in (-6, -7):  # non-finite loss or cancelled: the result holds the best so far
        err = HipMsatError(rc, lib().hms_last_error().decode())
        err.result = out
        raise err
    return out


def solve_batch(cnfs, steps=1000, restarts=1, eval_every=1, seeds=0, optimizer: int = ADAM,
                lr: float = 1e-4, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8,
                loss_mode: int = LOSS_UNSAT, schedule: int = 0, stream=None, want_x: bool = False):
    """Solve many instances in one call (see ``hms_solve_batch``).  Scalar
    arguments apply to every instance; lists give one value per instance.
    Returns one SolveOutput per instance (``status`` set on each; ``x_final``
    a device tensor when ``want_x``)."""
    cnfs = list(cnfs)
    N = len(cnfs)

    def per(v):
        return list(v) if isinstance(v, (list, tuple)) else [v] * N

    steps, restarts, eval_every, seeds = per(steps), per(restarts), per(eval_every), per(seeds)
    optimizer, lr, loss_mode, schedule = per(optimizer), per(lr), per(loss_mode), per(schedule)
    beta1, beta2, eps = per(beta1), per(beta2), per(eps)
    params = (SolveParams * N)()
    results = (SolveResult * N)()
    statuses = (C.c_int32 * N)()
    bufs = []
    for i, cnf in enumerate(cnfs):
        p = _params(cnf, steps[i], restarts[i], eval_every[i], seeds[i], optimizer[i], lr[i], beta1[i],
                    beta2[i], eps[i], loss_mode[i], schedule[i], True, 0.0, None, stream, False)
        params[i] = p
        R = int(restarts[i])
        ba = np.zeros(max(cnf.n, 1), dtype=np.uint8)
        rb = np.zeros(R, dtype=np.int64)
        rs = np.zeros(R, dtype=np.int32)
        rl = np.zeros(R, dtype=np.float64)
        results[i].best_assignment = ba.ctypes.data
        results[i].restart_best = rb.ctypes.data
        results[i].restart_step = rs.ctypes.data
        results[i].restart_loss = rl.ctypes.data
        xf = None
        if want_x:
            import torch
            xf = torch.empty((cnf.n, R), dtype=torch.float32, device="cuda")
            results[i].x_final = xf.data_ptr()
        bufs.append((ba, rb, rs, rl, xf))
    handles = (C.c_void_p * N)(*[c.handle.value for c in cnfs])
    rc = lib().hms_solve_batch(handles, params, N, results, statuses)
    outs = []
    for i, cnf in enumerate(cnfs):
        ba, rb, rs, rl, xf = bufs[i]
        r = results[i]
        o = SolveOutput(r.best_cost, r.best_restart, r.best_step, r.steps_done, r.schedule,
                        r.final_loss, r.device_ms, ba[:cnf.n].copy(), rb, rs, rl, xf)
        o.status = int(statuses[i])
        outs.append(o)
    if rc != HMS_OK and rc != -6:
        _check(rc)
    return outs


def evaluate(cnf: Cnf, assignment, stream=None) -> int:
    """Unsatisfied clauses of a 0/1 assignment (host array of n entries)."""
    a = np.ascontiguousarray(np.asarray(assignment) != 0, dtype=np.uint8)
    if a.shape != (cnf.n,):
        raise ValueError(f"assignment must have {cnf.n} entries, got shape {a.shape}")
    out = C.c_int64()
    _check(lib().hms_evaluate(cnf.handle, a.ctypes.data_as(C.c_void_p), C.byref(out),
                              _stream_ptr(stream)))
    return int(out.value)


def eval_relaxed(cnf: Cnf, x, loss_mode: int = LOSS_UNSAT, want_grad: bool = True, grad_out=None,
                 stream=None):
    """Loss, gradient and unsat count at relaxed points x (cuda float32 [n][R]).

    Returns (loss: float64[R], grad: torch [n][R] or None, unsat: int64[R])."""
    import torch
    X = _device_points(x, cnf, "x")
    R = X.shape[1]
    loss = np.zeros(R, dtype=np.float64)
    unsat = np.zeros(R, dtype=np.int64)
    g = None
    if want_grad:
        g = torch.empty_like(X) if grad_out is None else _device_points(grad_out, cnf, "grad_out")
        if g.shape != X.shape:
            raise ValueError(f"grad_out must have the shape of x, {tuple(X.shape)}")
    _check(lib().hms_eval_relaxed(cnf.handle, C.c_void_p(X.data_ptr()), R, int(loss_mode),
                                  loss.ctypes.data_as(C.c_void_p),
                                  C.c_void_p(g.data_ptr()) if g is not None else None,
                                  unsat.ctypes.data_as(C.c_void_p), _stream_ptr(stream)))
    return loss, g, unsat


def eval_relaxed_noalloc(cnf: Cnf, x, loss_out=None, grad_out=None, unsat_out=None, loss_mode: int = LOSS_UNSAT,
                         stream=None):
    """``hms_eval_relaxed_noalloc``: the evaluation of ``eval_relaxed`` into
    caller device tensors (loss float64 [R], grad float32 [n][R], unsat int64
    [R]; each may be None), with no allocation and no wait in the library."""
    import torch
    X = _device_points(x, cnf, "x")
    R = X.shape[1]

    def dev(t, dtype, shape, name):
        if t is None:
            return None
        if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != dtype or not t.is_contiguous() \
                or tuple(t.shape) != shape or t.device.index != cnf.device:
            raise ValueError(f"{name} must be a contiguous {dtype} tensor of shape {shape} on the instance's GPU")
        return C.c_void_p(t.data_ptr())

    _check(lib().hms_eval_relaxed_noalloc(cnf.handle, C.c_void_p(X.data_ptr()), R, int(loss_mode),
                                          dev(loss_out, torch.float64, (R,), "loss_out"),
                                          dev(grad_out, torch.float32, tuple(X.shape), "grad_out"),
                                          dev(unsat_out, torch.int64, (R,), "unsat_out"), _stream_ptr(stream)))


def version() -> str:
    return lib().hms_version().decode()


class Plan:
    """Host-only copy of an instance plan (tests of the layouts; no device)."""

    def __init__(self, n_vars: int, lits):
        a = _lits(lits)
        v = PlanView()
        _check(lib().hms_plan_view_build(int(n_vars), a.ctypes.data_as(C.c_void_p), a.size,
                                         C.byref(v)))
        try:
            for k, _ in PlanView._fields_:
                if k not in ("c_tile", "c_ent", "c_row_orig", "v_tile", "v_ent", "seg_first",
                             "seg_row", "var_old", "c_slot", "priv"):
                    setattr(self, k, getattr(v, k))

            def arr(ptr, count, dt):
                if count == 0 or not ptr:
                    return np.zeros(0, dtype=dt)
                buf = (C.c_char * (count * np.dtype(dt).itemsize)).from_address(ptr)
                return np.frombuffer(buf, dtype=dt).copy()

            self.c_tile = arr(v.c_tile, v.c_tiles * 4, np.uint32).reshape(-1, 4)
            self.c_ent = arr(v.c_ent, v.c_ent_len, np.uint32)
            self.c_row_orig = arr(v.c_row_orig, v.c_tiles * v.tile_rows, np.int32)
            self.v_tile = arr(v.v_tile, v.v_tiles * 4, np.uint32).reshape(-1, 4)
            self.v_ent = arr(v.v_ent, v.v_ent_len, np.uint32)
            self.seg_first = arr(v.seg_first, v.n_heavy + 1 if v.n_heavy else 0, np.int32)
            self.seg_row = arr(v.seg_row, v.seg_rows, np.int32)
            self.var_old = arr(v.var_old, v.n, np.int32)
            self.c_slot = arr(v.c_slot, v.c_ent_len, np.uint32)
        finally:
            lib().hms_plan_view_free(C.byref(v))
