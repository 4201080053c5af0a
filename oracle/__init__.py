"""Python view of the FP64 CPU oracle (``oracle.c``).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg of
the benchmark use it; the HIP library never does.  Build with :func:`build`
(gcc, no GPU needed).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
# HIPMSAT_ORACLE_LIB names another build (the sanitized one of build(sanitize=True))
_LIB = os.environ.get("HIPMSAT_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")

UNSAT, ALL = 0, 1
ADAM, SGD = 0, 1


def build(force: bool = True, sanitize: bool = False, out: str | None = None) -> str:
    """Compile ``oracle.c`` with gcc (plain IEEE FP64, no contraction); with
    ``sanitize`` under ASan and UBSan (load it through HIPMSAT_ORACLE_LIB with
    gcc's libasan and libubsan preloaded)."""
    lib_path = out or _LIB
    if force or not os.path.exists(lib_path):
        tmp = lib_path + ".tmp"
        san = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-fno-sanitize-recover=undefined",
               "-g"] if sanitize else []
        subprocess.check_call([
            "gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
            "-fno-fast-math", "-Wall"] + san + ["-o", tmp, _SRC, "-lm"])
        os.replace(tmp, lib_path)
    return lib_path


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = C.CDLL(_LIB)
        P, I32, I64, U64, D = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64, C.c_double
        L.oracle_build.argtypes = [I32, P, I64, C.POINTER(P)]
        L.oracle_build.restype = C.c_int
        L.oracle_free.argtypes = [P]
        L.oracle_free.restype = None
        L.oracle_n.argtypes = [P]; L.oracle_n.restype = I32
        L.oracle_m.argtypes = [P]; L.oracle_m.restype = I32
        L.oracle_count.argtypes = [P, P]; L.oracle_count.restype = I64
        L.oracle_unsat_mask.argtypes = [P, P, P]; L.oracle_unsat_mask.restype = None
        L.oracle_loss_grad_d.argtypes = [P, P, C.c_int, P, P, P, P]
        L.oracle_loss_grad_d.restype = D
        L.oracle_loss_grad_f.argtypes = [P, P, C.c_int, P, P, P, P]
        L.oracle_loss_grad_f.restype = D
        L.oracle_adam_step.argtypes = [I32, P, P, P, P, I32, D, D, D, D]
        L.oracle_adam_step.restype = None
        L.oracle_sgd_step.argtypes = [I32, P, P, D]
        L.oracle_sgd_step.restype = None
        L.oracle_splitmix64.argtypes = [U64, U64]; L.oracle_splitmix64.restype = U64
        L.oracle_init_x.argtypes = [I32, I32, U64, P]; L.oracle_init_x.restype = None
        L.oracle_solve.argtypes = [P, I32, I32, I32, U64, I32, D, D, D, D, I32, P, I32,
                                   P, P, P, P, P, P]
        L.oracle_solve.restype = I64
        L.oracle_run.argtypes = [P, I32, I32, I32, I32, D, D, D, D, I32, I32, P, P, P, P, P, P, P, P]
        L.oracle_run.restype = C.c_int
        L.oracle_init_state.argtypes = [P, I32, U64, P, P, P, P, P, P, P, P]
        L.oracle_init_state.restype = None
        L.oracle_bruteforce.argtypes = [P, P, P, P]
        L.oracle_bruteforce.restype = C.c_int
        L.oracle_set_weights.argtypes = [P, P]
        L.oracle_set_weights.restype = C.c_int
        L.oracle_total_weight.argtypes = [P]
        L.oracle_total_weight.restype = I64
        L.oracle_num_threads.argtypes = []
        L.oracle_num_threads.restype = C.c_int
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


class OracleError(RuntimeError):
    def __init__(self, code):
        super().__init__(f"oracle error {code}")
        self.code = code


class OracleCNF:
    """A canonicalized CNF held by the oracle."""

    def __init__(self, n_vars: int, lits, weights=None):
        """weights: one positive integer per clause (weighted MaxSAT), or None
        for weight 1 everywhere."""
        self._lits = np.ascontiguousarray(lits, dtype=np.int32)
        h = C.c_void_p()
        rc = lib().oracle_build(int(n_vars), _ptr(self._lits), self._lits.size, C.byref(h))
        if rc != 0:
            raise OracleError(rc)
        self._h = h
        self.n = lib().oracle_n(h)
        self.m = lib().oracle_m(h)
        if weights is not None:
            self._w = np.ascontiguousarray(weights, dtype=np.int64)
            assert self._w.shape == (self.m,)
            rc = lib().oracle_set_weights(h, _ptr(self._w))
            if rc != 0:
                raise OracleError(rc)
        self.total_weight = int(lib().oracle_total_weight(h))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.oracle_free(h)
            self._h = None

    # --- counts -----------------------------------------------------------
    def count(self, assign) -> int:
        a = np.ascontiguousarray(assign, dtype=np.uint8)
        assert a.shape == (self.n,)
        return int(lib().oracle_count(self._h, _ptr(a)))

    def unsat_mask(self, assign) -> np.ndarray:
        a = np.ascontiguousarray(assign, dtype=np.uint8)
        out = np.zeros(self.m, dtype=np.uint8)
        lib().oracle_unsat_mask(self._h, _ptr(a), _ptr(out))
        return out

    # --- relaxed evaluation ------------------------------------------------
    def loss_grad(self, x, mode: int = UNSAT, want_f: bool = False):
        """x: [n] or [n][R] (float32 values are widened exactly; float64 is used as is).

        Returns (loss[R], grad[n][R] float64, unsat[R] int64[, f[m][R], mu[m][R]])."""
        x = np.asarray(x)
        squeeze = x.ndim == 1
        X = x.reshape(self.n, -1)
        R = X.shape[1]
        loss = np.zeros(R)
        grad = np.zeros((self.n, R))
        unsat = np.zeros(R, dtype=np.int64)
        fs = np.zeros((self.m, R)) if want_f else None
        mus = np.zeros((self.m, R), dtype=np.uint8) if want_f else None
        for r in range(R):
            g = np.zeros(self.n)
            u = C.c_int64()
            f = np.zeros(self.m) if want_f else None
            mu = np.zeros(self.m, dtype=np.uint8) if want_f else None
            if X.dtype == np.float32:
                xr = np.ascontiguousarray(X[:, r])
                loss[r] = lib().oracle_loss_grad_f(self._h, _ptr(xr), mode, _ptr(f), _ptr(mu),
                                                   _ptr(g), C.byref(u))
            else:
                xr = np.ascontiguousarray(X[:, r], dtype=np.float64)
                loss[r] = lib().oracle_loss_grad_d(self._h, _ptr(xr), mode, _ptr(f), _ptr(mu),
                                                   _ptr(g), C.byref(u))
            grad[:, r] = g
            unsat[r] = u.value
            if want_f:
                fs[:, r] = f
                mus[:, r] = mu
        if squeeze:
            grad = grad[:, 0]
            if want_f:
                fs, mus = fs[:, 0], mus[:, 0]
        out = (loss, grad, unsat)
        if want_f:
            out = out + (fs, mus)
        return out

    def loss(self, x, mode: int = UNSAT) -> float:
        return float(self.loss_grad(np.asarray(x), mode)[0][0])

    # --- the loop -------------------------------------------------------------
    def solve(self, steps: int, restarts: int = 1, eval_every: int = 1, seed: int = 0,
              optimizer: int = ADAM, lr: float = 1e-4, beta1: float = 0.9,
              beta2: float = 0.999, eps: float = 1e-8, mode: int = UNSAT, x0=None,
              threads: int = 1, want_x: bool = False) -> dict:
        R = int(restarts)
        rb = np.zeros(R, dtype=np.int64)
        rs = np.zeros(R, dtype=np.int32)
        fl = np.zeros(R)
        ba = np.zeros(self.n, dtype=np.uint8)
        br = C.c_int32()
        x0a = None if x0 is None else np.ascontiguousarray(x0, dtype=np.float32).reshape(self.n, R)
        xo = np.zeros((self.n, R)) if want_x else None
        best = lib().oracle_solve(self._h, int(steps), R, int(eval_every), int(seed) & (2**64 - 1),
                                  int(optimizer), lr, beta1, beta2, eps, int(mode), _ptr(x0a),
                                  int(threads), _ptr(rb), _ptr(rs), _ptr(fl), _ptr(ba),
                                  C.byref(br), _ptr(xo))
        if best < 0:
            raise OracleError(int(best))
        out = dict(best_cost=int(best), best_restart=int(br.value), restart_best=rb,
                   restart_step=rs, final_loss=fl, best_assignment=ba)
        if want_x:
            out["x"] = xo
        return out

    # --- the loop's state (x, moments, step, best so far) ---------------------
    def init_state(self, restarts: int = 1, seed: int = 0, x0=None) -> dict:
        """The state before the first iteration of Algorithm 1: x from x0
        ([n][R] float32) or SplitMix64, zero moments, step 0, best = the total
        weight, best_step = -1, best assignment = round(x).  x, m, v are
        float64 [n][R], best_assignment uint8 [R][n]."""
        R = int(restarts)
        st = dict(x=np.zeros((self.n, R)), m=np.zeros((self.n, R)), v=np.zeros((self.n, R)),
                  step=0, best=np.zeros(R, dtype=np.int64), best_step=np.zeros(R, dtype=np.int32),
                  best_assignment=np.zeros((R, self.n), dtype=np.uint8))
        x0a = None if x0 is None else np.ascontiguousarray(x0, dtype=np.float32).reshape(self.n, R)
        step = C.c_int32()
        lib().oracle_init_state(self._h, R, int(seed) & (2**64 - 1), _ptr(x0a), _ptr(st["x"]), _ptr(st["m"]),
                                _ptr(st["v"]), C.byref(step), _ptr(st["best"]), _ptr(st["best_step"]),
                                _ptr(st["best_assignment"]))
        st["step"] = step.value
        return st

    def run(self, state: dict, steps: int, eval_every: int = 1, optimizer: int = ADAM, lr: float = 1e-4,
            beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8, mode: int = UNSAT,
            threads: int = 1) -> dict:
        """Continue Algorithm 1 from ``state`` for ``steps`` more steps; returns
        a new state (the argument is not changed) with ``final_loss`` [R], the
        loss at its last iterate."""
        st = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in state.items()}
        R = st["x"].shape[1]
        for k, dt in (("x", np.float64), ("m", np.float64), ("v", np.float64)):
            st[k] = np.ascontiguousarray(st[k], dtype=dt).reshape(self.n, R)
        st["best"] = np.ascontiguousarray(st["best"], dtype=np.int64)
        st["best_step"] = np.ascontiguousarray(st["best_step"], dtype=np.int32)
        st["best_assignment"] = np.ascontiguousarray(st["best_assignment"], dtype=np.uint8).reshape(R, self.n)
        fl = np.zeros(R)
        step = C.c_int32(int(st["step"]))
        rc = lib().oracle_run(self._h, int(steps), R, int(eval_every), int(optimizer), lr, beta1, beta2, eps,
                              int(mode), int(threads), _ptr(st["x"]), _ptr(st["m"]), _ptr(st["v"]),
                              C.byref(step), _ptr(st["best"]), _ptr(st["best_step"]),
                              _ptr(st["best_assignment"]), _ptr(fl))
        if rc != 0:
            raise OracleError(rc)
        st["step"] = step.value
        st["final_loss"] = fl
        return st

    def bruteforce(self):
        """(opt, number of optimal assignments, one optimal assignment)."""
        opt, nopt = C.c_int64(), C.c_int64()
        arg = np.zeros(self.n, dtype=np.uint8)
        rc = lib().oracle_bruteforce(self._h, C.byref(opt), C.byref(nopt), _ptr(arg))
        if rc != 0:
            raise OracleError(rc)
        return int(opt.value), int(nopt.value), arg


def adam_step(x, m, v, g, step, lr=1e-4, beta1=0.9, beta2=0.999, eps=1e-8):
    """In-place FP64 Adam step on 1-D float64 arrays."""
    for a in (x, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    g = np.ascontiguousarray(g, dtype=np.float64)
    lib().oracle_adam_step(x.size, _ptr(x), _ptr(m), _ptr(v), _ptr(g), int(step), lr, beta1,
                           beta2, eps)


def sgd_step(x, g, lr):
    assert x.dtype == np.float64 and x.flags.c_contiguous
    g = np.ascontiguousarray(g, dtype=np.float64)
    lib().oracle_sgd_step(x.size, _ptr(x), _ptr(g), lr)


def splitmix64(seed: int, k: int) -> int:
    return int(lib().oracle_splitmix64(seed & (2**64 - 1), k))


def init_x(n: int, R: int, seed: int) -> np.ndarray:
    x = np.zeros((n, R), dtype=np.float32)
    lib().oracle_init_x(n, R, seed & (2**64 - 1), _ptr(x))
    return x


def num_threads() -> int:
    return int(lib().oracle_num_threads())
