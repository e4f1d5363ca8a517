"""CPU oracle for Sparse SAGA / ASAGA (paper: Leblond, Pedregosa &
Lacoste-Julien, "ASAGA: Asynchronous Parallel SAGA", AISTATS 2017).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares
no code with the HIP library (``paper_1606_04809_amd``) and never imports it;
both sides consume the same seeded inputs from ``datagen``.

Two parts:

* the algorithm, step by step, in plain C (``saga_oracle.c``, FP64, one
  thread): the Sparse SAGA update of Section 2 (Eq. SparseSAGA) with the
  projected L2 term of Section 4.2, run serially in the order Algorithm 2
  prescribes, plus the compensated objective and gradient;
* the plain definitions of the optimum the iteration converges to, in numpy:
  the ridge closed form for least squares, damped Newton for small logistic
  problems, and a strong-convexity certificate for large ones.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import time
from dataclasses import dataclass

import numpy as np

LOGISTIC = 0
SQUARED = 1

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_U64 = ctypes.c_uint64
_D = ctypes.c_double
_I = ctypes.c_int

_SIGS = {
    "oracle_splitmix64": (_U64, [_U64, _U64]),
    "oracle_sample": (_I64, [_U64, _U64, _I64]),
    "oracle_sample_stream": (None, [_U64, _U64, _I64, _I64, _P]),
    "oracle_phi": (_D, [_D, _D, _I]),
    "oracle_dphi": (_D, [_D, _D, _I]),
    "oracle_column_counts": (None, [_I64, _I64, _P, _P, _P]),
    "oracle_reweighting": (None, [_I64, _I64, _P, _P]),
    "oracle_smoothness": (_D, [_I64, _P, _P, _I, _D]),
    "oracle_step_size": (_D, [_D, _D, _I64, _P]),
    "oracle_saga_indices": (_I, [_I64, _P, _P, _P, _P, _I, _D, _P, _D, _P, _I64, _P, _P, _P]),
    "oracle_saga_run": (_I, [_I64, _P, _P, _P, _P, _I, _D, _P, _D, _U64, _U64, _I64, _P, _P, _P]),
    "oracle_delayed_saga_run": (_I, [_I64, _I64, _P, _P, _P, _P, _I, _D, _P, _D, _U64, _U64, _I64, _I64, _D, _U64,
                                     _P, _P, _P]),
    "oracle_objective": (_D, [_I64, _I64, _P, _P, _P, _P, _I, _D, _P]),
    "oracle_gradient": (_I, [_I64, _I64, _P, _P, _P, _P, _I, _D, _P, _P]),
    "oracle_memory_average": (_I, [_I64, _I64, _P, _P, _P, _P, _P]),
    "oracle_dense_saga_run": (_I, [_I64, _I64, _P, _P, _P, _P, _I, _D, _D, _U64, _U64, _I64, _P, _P, _P]),
    "oracle_lagged_saga_run": (_I, [_I64, _I64, _P, _P, _P, _P, _I, _D, _D, _U64, _U64, _I64, _P, _P, _P, _P]),
    "oracle_svrg_full_gradient_due": (_I, [_U64, _U64, _I64]),
    "oracle_svrg_snapshot": (None, [_I64, _I64, _P, _P, _P, _P, _I, _P, _P, _P]),
    "oracle_svrg_indices": (_I, [_P, _P, _P, _P, _I, _D, _P, _D, _I64, _P, _I64, _P, _P, _P]),
    "oracle_svrg_run": (_I, [_I64, _I64, _P, _P, _P, _P, _I, _D, _P, _D, _U64, _U64, _I64, _P, _P, _P]),
}


def build(force: bool = True) -> str:
    """Compile the C oracle in place (gcc, no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB_PATH):
        src = os.path.join(_HERE, "saga_oracle.c")
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-shared", "-fPIC", src, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def load(path: str | None = None):
    """The ctypes handle of the oracle library (a custom ``path`` loads
    another build of the same source, e.g. a planted-mistake variant)."""
    global _lib
    if path is not None:
        return _bind(ctypes.CDLL(path))
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=True)
        _lib = _bind(ctypes.CDLL(_LIB_PATH))
    return _lib


def _bind(lib):
    for name, (res, args) in _SIGS.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


def _p(a: np.ndarray):
    return a.ctypes.data


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


# ---------------------------------------------------------------------------
# sample stream
# ---------------------------------------------------------------------------

def splitmix64(seed: int, t: int) -> int:
    return int(load().oracle_splitmix64(seed, t))


def sample_stream(seed: int, t0: int, count: int, n: int) -> np.ndarray:
    out = np.empty(count, dtype=np.int64)
    load().oracle_sample_stream(seed, t0, count, n, _p(out))
    return out


def phi(z: float, b: float, loss: int) -> float:
    return float(load().oracle_phi(z, b, loss))


def dphi(z: float, b: float, loss: int) -> float:
    return float(load().oracle_dphi(z, b, loss))


# ---------------------------------------------------------------------------
# solver state
# ---------------------------------------------------------------------------

@dataclass
class State:
    x: np.ndarray
    alpha: np.ndarray
    abar: np.ndarray
    t: int = 0

    def copy(self) -> "State":
        return State(self.x.copy(), self.alpha.copy(), self.abar.copy(), self.t)


class SparseSaga:
    """Serial FP64 Sparse SAGA on one problem (``datagen.Problem`` or any
    object with n, d, rowptr, colidx, val, b, loss, lam)."""

    def __init__(self, prob, step: float | None = None, seed: int = 0, lib=None):
        self.lib = lib if lib is not None else load()
        self.n, self.d = int(prob.n), int(prob.d)
        self.rowptr = _c(prob.rowptr, np.int64)
        self.colidx = _c(prob.colidx, np.int32)
        self.val = _c(prob.val, np.float64)
        self.b = _c(prob.b, np.float64)
        self.loss = int(prob.loss)
        self.lam = float(prob.lam)
        self.seed = int(seed)
        self.cnt = np.empty(self.d, dtype=np.int64)
        self.lib.oracle_column_counts(self.n, self.d, _p(self.rowptr), _p(self.colidx), _p(self.cnt))
        self.D = np.empty(self.d, dtype=np.float64)
        self.lib.oracle_reweighting(self.n, self.d, _p(self.cnt), _p(self.D))
        self.L = float(self.lib.oracle_smoothness(self.n, _p(self.rowptr), _p(self.val), self.loss, self.lam))
        self.gamma = float(step) if step is not None and step > 0 else \
            float(self.lib.oracle_step_size(self.L, self.lam, self.d, _p(self.D)))
        self.state = State(np.zeros(self.d), np.zeros(self.n), np.zeros(self.d), 0)

    # -- iteration -----------------------------------------------------------
    def run(self, updates: int, state: State | None = None) -> State:
        """Updates t .. t+updates-1 of the seeded stream (in place)."""
        s = self.state if state is None else state
        rc = self.lib.oracle_saga_run(self.n, _p(self.rowptr), _p(self.colidx), _p(self.val), _p(self.b),
                                      self.loss, self.lam, _p(self.D), self.gamma, self.seed, s.t, int(updates),
                                      _p(s.x), _p(s.alpha), _p(s.abar))
        if rc != 0:
            raise RuntimeError(f"oracle_saga_run failed ({rc})")
        s.t += int(updates)
        return s

    def epochs(self, e: float, state: State | None = None) -> State:
        return self.run(int(round(e * self.n)), state)

    def run_indices(self, idx, state: State | None = None) -> State:
        s = self.state if state is None else state
        idx = _c(idx, np.int64)
        rc = self.lib.oracle_saga_indices(self.n, _p(self.rowptr), _p(self.colidx), _p(self.val), _p(self.b),
                                          self.loss, self.lam, _p(self.D), self.gamma, _p(idx), len(idx),
                                          _p(s.x), _p(s.alpha), _p(s.abar))
        if rc != 0:
            raise RuntimeError(f"oracle_saga_indices failed ({rc})")
        return s

    # -- plain definitions ---------------------------------------------------
    def objective(self, x: np.ndarray | None = None) -> float:
        x = self.state.x if x is None else _c(x, np.float64)
        return float(self.lib.oracle_objective(self.n, self.d, _p(self.rowptr), _p(self.colidx), _p(self.val),
                                               _p(self.b), self.loss, self.lam, _p(x)))

    def gradient(self, x: np.ndarray | None = None) -> np.ndarray:
        x = self.state.x if x is None else _c(x, np.float64)
        g = np.empty(self.d)
        rc = self.lib.oracle_gradient(self.n, self.d, _p(self.rowptr), _p(self.colidx), _p(self.val),
                                      _p(self.b), self.loss, self.lam, _p(x), _p(g))
        if rc != 0:
            raise RuntimeError("oracle_gradient failed")
        return g

    def memory_average(self, alpha: np.ndarray | None = None) -> np.ndarray:
        alpha = self.state.alpha if alpha is None else _c(alpha, np.float64)
        out = np.empty(self.d)
        rc = self.lib.oracle_memory_average(self.n, self.d, _p(self.rowptr), _p(self.colidx), _p(self.val),
                                            _p(alpha), _p(out))
        if rc != 0:
            raise RuntimeError("oracle_memory_average failed")
        return out

    def certificate(self, x: np.ndarray | None = None) -> tuple[float, float]:
        """(f(x), f(x) - ||grad f(x)||^2 / (2 lambda)): f is lambda-strongly
        convex (the L2 term of Section 4.1 alone gives mu >= lambda), so the
        second value is a lower bound on f*."""
        f = self.objective(x)
        g = self.gradient(x)
        return f, f - float(g @ g) / (2.0 * self.lam)


class DenseSaga(SparseSaga):
    """Serial FP64 dense SAGA (every coordinate receives abar + lambda x at
    every step), the baseline of the Appendix F comparison.  Same sample
    stream and step rule as Sparse SAGA."""

    def run(self, updates: int, state: State | None = None) -> State:
        s = self.state if state is None else state
        rc = self.lib.oracle_dense_saga_run(self.n, self.d, _p(self.rowptr), _p(self.colidx), _p(self.val), _p(self.b),
                                            self.loss, self.lam, self.gamma, self.seed, s.t, int(updates), _p(s.x),
                                            _p(s.alpha), _p(s.abar))
        if rc != 0:
            raise RuntimeError(f"oracle_dense_saga_run failed ({rc})")
        s.t += int(updates)
        return s


class DelayedSparseSaga(SparseSaga):
    """Sparse SAGA with simulated inconsistent reads (Section 3.3, bounded
    overlap tau and Eq. async): each read lacks, independently with
    probability ``miss``, each coordinate write of each of the last ``tau``
    updates (decided by a SplitMix64 stream from ``delay_seed``); the writes
    are additions to the shared state in update order.  ``miss`` = 0 is
    Sparse SAGA exactly, ``miss`` = 1 reads the state of tau updates earlier.
    The window of missing writes starts empty at each call of ``run``."""

    def __init__(self, prob, tau: int, miss: float, delay_seed: int = 0x5EED, step: float | None = None,
                 seed: int = 0, lib=None):
        super().__init__(prob, step=step, seed=seed, lib=lib)
        self.tau, self.miss, self.delay_seed = int(tau), float(miss), int(delay_seed)

    def run(self, updates: int, state: State | None = None) -> State:
        s = self.state if state is None else state
        rc = self.lib.oracle_delayed_saga_run(self.n, self.d, _p(self.rowptr), _p(self.colidx), _p(self.val),
                                              _p(self.b), self.loss, self.lam, _p(self.D), self.gamma, self.seed,
                                              s.t, int(updates), self.tau, self.miss, self.delay_seed,
                                              _p(s.x), _p(s.alpha), _p(s.abar))
        if rc != 0:
            raise RuntimeError(f"oracle_delayed_saga_run failed ({rc})")
        s.t += int(updates)
        return s


class LaggedSaga(SparseSaga):
    """Serial FP64 lagged-update SAGA (Appendix F): dense SAGA's iterates with
    the dense part of each step deferred to the next read of a coordinate."""

    def __init__(self, prob, step: float | None = None, seed: int = 0, lib=None):
        super().__init__(prob, step=step, seed=seed, lib=lib)
        self.last = np.zeros(self.d, dtype=np.uint64)

    def run(self, updates: int, state: State | None = None) -> State:
        s = self.state if state is None else state
        if s.t != 0 and not np.all(self.last == s.t):
            raise RuntimeError("lagged counters out of step with the state")
        rc = self.lib.oracle_lagged_saga_run(self.n, self.d, _p(self.rowptr), _p(self.colidx), _p(self.val),
                                             _p(self.b), self.loss, self.lam, self.gamma, self.seed, s.t, int(updates),
                                             _p(s.x), _p(s.alpha), _p(s.abar), _p(self.last))
        if rc != 0:
            raise RuntimeError(f"oracle_lagged_saga_run failed ({rc})")
        s.t += int(updates)
        return s


class SparseSvrg(SparseSaga):
    """Serial FP64 sparse SVRG with randomly timed full gradients (the
    Appendix C variant): the memory (alpha_i = phi'(a_i . x~), abar its
    average) is the snapshot's and changes only at snapshots; a snapshot is
    taken at x0 and wherever the U stream fires (probability 1/n per
    iteration)."""

    def __init__(self, prob, step: float | None = None, seed: int = 0, lib=None):
        super().__init__(prob, step=step, seed=seed, lib=lib)
        self.snapshot()

    def snapshot(self, state: State | None = None) -> State:
        s = self.state if state is None else state
        self.lib.oracle_svrg_snapshot(self.n, self.d, _p(self.rowptr), _p(self.colidx), _p(self.val), _p(self.b),
                                      self.loss, _p(s.x), _p(s.alpha), _p(s.abar))
        return s

    def full_gradient_due(self, t: int) -> bool:
        return bool(self.lib.oracle_svrg_full_gradient_due(self.seed, int(t), self.n))

    def run(self, updates: int, state: State | None = None) -> State:
        s = self.state if state is None else state
        rc = self.lib.oracle_svrg_run(self.n, self.d, _p(self.rowptr), _p(self.colidx), _p(self.val), _p(self.b),
                                      self.loss, self.lam, _p(self.D), self.gamma, self.seed, s.t, int(updates),
                                      _p(s.x), _p(s.alpha), _p(s.abar))
        if rc != 0:
            raise RuntimeError(f"oracle_svrg_run failed ({rc})")
        s.t += int(updates)
        return s

    def run_indices(self, idx, state: State | None = None) -> State:
        s = self.state if state is None else state
        idx = _c(idx, np.int64)
        rc = self.lib.oracle_svrg_indices(_p(self.rowptr), _p(self.colidx), _p(self.val), _p(self.b), self.loss,
                                          self.lam, _p(self.D), self.gamma, self.n, _p(idx), len(idx), _p(s.x),
                                          _p(s.alpha), _p(s.abar))
        if rc != 0:
            raise RuntimeError(f"oracle_svrg_indices failed ({rc})")
        return s


# ---------------------------------------------------------------------------
# plain definitions of the optimum
# ---------------------------------------------------------------------------

def ridge_solution(prob) -> np.ndarray:
    """Least squares closed form x* = (A'A/n + lambda I)^-1 A'b/n by Cholesky
    (dense; small d only)."""
    A = prob.dense() if hasattr(prob, "dense") else np.asarray(prob.A)
    n = A.shape[0]
    H = A.T @ A / n + prob.lam * np.eye(A.shape[1])
    r = A.T @ np.asarray(prob.b, dtype=np.float64) / n
    C = np.linalg.cholesky(H)
    return np.linalg.solve(C.T, np.linalg.solve(C, r))


def ridge_solution_csr(prob, rows_per_block: int = 65536) -> np.ndarray:
    """Same closed form, forming A'A/n from blocks of CSR rows without a
    dense A (for tall problems with small d, e.g. 581,000 x 54)."""
    n, d = int(prob.n), int(prob.d)
    H = np.zeros((d, d))
    r = np.zeros(d)
    for r0 in range(0, n, rows_per_block):
        r1 = min(n, r0 + rows_per_block)
        s, e = int(prob.rowptr[r0]), int(prob.rowptr[r1])
        rr = np.repeat(np.arange(r1 - r0), np.diff(prob.rowptr[r0:r1 + 1]))
        Ablk = np.zeros((r1 - r0, d))
        Ablk[rr, prob.colidx[s:e]] = prob.val[s:e]
        H += Ablk.T @ Ablk
        r += Ablk.T @ np.asarray(prob.b[r0:r1], dtype=np.float64)
    H = H / n + prob.lam * np.eye(d)
    C = np.linalg.cholesky(H)
    return np.linalg.solve(C.T, np.linalg.solve(C, r / n))


def logistic_newton(prob, tol: float = 1e-15, max_iter: int = 100) -> np.ndarray:
    """Damped Newton with backtracking on the dense logistic objective
    (1/n) sum log(1+exp(-b_i a_i.x)) + (lambda/2)||x||^2; small d only."""
    A = prob.dense()
    b = np.asarray(prob.b, dtype=np.float64)
    n, d = A.shape
    lam = float(prob.lam)

    def fval(x):
        m = b * (A @ x)
        return float(np.mean(np.logaddexp(0.0, -m)) + 0.5 * lam * x @ x)

    x = np.zeros(d)
    f = fval(x)
    for _ in range(max_iter):
        m = b * (A @ x)
        s = 0.5 * (1.0 + np.tanh(0.5 * m))          # 1/(1+exp(-m)), overflow-free
        g = A.T @ (-b * (1.0 - s)) / n + lam * x
        w = s * (1.0 - s)
        H = (A.T * w) @ A / n + lam * np.eye(d)
        step = np.linalg.solve(H, g)
        dec = float(g @ step)
        if dec / 2.0 <= tol * max(abs(f), 1e-300):
            break
        tstep = 1.0
        while True:
            xn = x - tstep * step
            fn = fval(xn)
            if fn <= f - 0.25 * tstep * dec or tstep < 1e-12:
                break
            tstep *= 0.5
        x, f = xn, fn
    return x


def certified_fstar(prob, tol: float = 1e-11, seed: int = 0, max_epochs: int = 2000,
                    check_every: int = 5, log=None) -> dict:
    """Run the oracle's own Sparse SAGA until the strong-convexity
    certificate ||grad f||^2 / (2 lambda) <= tol * f holds.  Returns the
    bracket [f_lower, f_upper] on f* and the iterate."""
    sv = SparseSaga(prob, seed=seed)
    t0 = time.time()
    ep = 0
    while True:
        sv.epochs(check_every)
        ep += check_every
        f, flo = sv.certificate()
        if log:
            log(f"epoch {ep}: f={f:.17g} gap={f - flo:.3e} ({time.time() - t0:.1f}s)")
        if f - flo <= tol * abs(f) or ep >= max_epochs:
            break
    return {"f_upper": f, "f_lower": flo, "epochs": ep, "x": sv.state.x.copy(), "gamma": sv.gamma, "L": sv.L,
            "converged": f - flo <= tol * abs(f)}
