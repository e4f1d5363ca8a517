"""Python binding of the gfx950 Sparse SAGA / ASAGA library (libasaga.so).

Argument marshalling only: every step of the method runs in the HIP kernels
behind the C ABI declared in ``include/asaga.h``.  The functions below carry
the C names; ``Solver`` bundles them for one context.  Inputs may be numpy
arrays (host memory, copied by the library) or torch CUDA tensors (device
memory, borrowed); torch is used for nothing else than device memory and
streams.

If the library has not been built this module raises ImportError: there is
no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libasaga.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build the HIP library first "
                      "(python paper_1606_04809_amd/build.py, or __graft_entry__.build())")

# One HIP runtime per process: torch ships its own libamdhip64 (same SONAME
# as the system one).  Loading torch first lets the dynamic loader resolve
# this library's HIP dependency to the runtime torch already mapped, so that
# device pointers and streams are shared instead of split across two runtimes.
try:
    import torch  # noqa: F401
except ImportError:  # the library itself does not need torch
    pass

_lib = ctypes.CDLL(LIB_PATH)

# ---- constants (asaga.h) ----------------------------------------------------
ASAGA_OK = 0
ASAGA_E_ARG = -1
ASAGA_E_CSR = -2
ASAGA_E_OOM = -3
ASAGA_E_HIP = -4
ASAGA_E_DIVERGED = -5
ASAGA_E_STATE = -6
ASAGA_LOSS_LOGISTIC = 0
ASAGA_LOSS_SQUARED = 1
ASAGA_VAL_F64 = 0
ASAGA_VAL_F32 = 1
ASAGA_VAL_BF16 = 2
ASAGA_MEM_HOST = 0
ASAGA_MEM_DEVICE = 1
ASAGA_MODE_SERIAL = 0
ASAGA_MODE_ASYNC = 1
ASAGA_PREC_F64 = 0
ASAGA_PREC_MIXED = 1
ASAGA_PREC_F32 = 2
ASAGA_METHOD_SAGA = 0
ASAGA_METHOD_SVRG = 1
ASAGA_NOALLOC_MAX_ROWS = 4194304

ERROR_NAMES = {0: "ASAGA_OK", -1: "ASAGA_E_ARG", -2: "ASAGA_E_CSR", -3: "ASAGA_E_OOM", -4: "ASAGA_E_HIP",
               -5: "ASAGA_E_DIVERGED", -6: "ASAGA_E_STATE"}


class asaga_problem(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("d", ctypes.c_int64), ("rowptr", ctypes.c_void_p),
                ("colidx", ctypes.c_void_p), ("val", ctypes.c_void_p), ("b", ctypes.c_void_p),
                ("lam", ctypes.c_double), ("val_dtype", ctypes.c_int32), ("loss", ctypes.c_int32),
                ("mem", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class asaga_opts(ctypes.Structure):
    _fields_ = [("step", ctypes.c_double), ("seed", ctypes.c_uint64), ("mode", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("waves", ctypes.c_int32), ("lanes_per_sample", ctypes.c_int32),
                ("racy", ctypes.c_int32), ("hot_columns", ctypes.c_int32), ("flush_every", ctypes.c_int32),
                ("threads_per_block", ctypes.c_int32), ("hot_tier_columns", ctypes.c_int32),
                ("hot_tier_every", ctypes.c_int32), ("plain_launch", ctypes.c_int32), ("method", ctypes.c_int32),
                ("stream", ctypes.c_void_p), ("hot_reload_from", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class asaga_batch(ctypes.Structure):
    _fields_ = [("n_inst", ctypes.c_int32), ("reserved", ctypes.c_int32), ("row_fold", ctypes.c_void_p),
                ("inst_fold", ctypes.c_void_p), ("inst_lambda", ctypes.c_void_p)]


class asaga_tune_report(ctypes.Structure):
    _fields_ = [("candidates", ctypes.c_int32), ("waves", ctypes.c_int32), ("hot_columns", ctypes.c_int32),
                ("hot_tier_columns", ctypes.c_int32), ("gamma", ctypes.c_double), ("ms_per_epoch", ctypes.c_double),
                ("est_epochs", ctypes.c_double), ("est_seconds", ctypes.c_double),
                ("step_groups", ctypes.c_double), ("step_cap", ctypes.c_double),
                ("widen_gamma", ctypes.c_double), ("threads_per_block", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class asaga_overlap_report(ctypes.Structure):
    _fields_ = [("logged", ctypes.c_int64), ("every", ctypes.c_int64), ("tau_mean", ctypes.c_double),
                ("tau_p50", ctypes.c_double), ("tau_p99", ctypes.c_double), ("tau_max", ctypes.c_double),
                ("latency_mean_us", ctypes.c_double), ("latency_p99_us", ctypes.c_double),
                ("updates_per_s", ctypes.c_double), ("little", ctypes.c_double)]


class asaga_instance(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int64), ("t", ctypes.c_int64), ("lam", ctypes.c_double), ("gamma", ctypes.c_double),
                ("L", ctypes.c_double), ("fold", ctypes.c_int32), ("active", ctypes.c_int32)]


class asaga_info(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("d", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("delta_r", ctypes.c_int64), ("t", ctypes.c_int64), ("L", ctypes.c_double),
                ("gamma", ctypes.c_double), ("lam", ctypes.c_double), ("waves", ctypes.c_int32),
                ("lanes_per_sample", ctypes.c_int32), ("n_inst", ctypes.c_int32), ("hot_columns", ctypes.c_int32),
                ("flush_every", ctypes.c_int32), ("threads_per_block", ctypes.c_int32),
                ("hot_tier_columns", ctypes.c_int32), ("hot_tier_every", ctypes.c_int32),
                ("hot_reload_from", ctypes.c_int32)]


_P = ctypes.c_void_p
_CTX = ctypes.c_void_p
_SIGS = {
    "asaga_init": (ctypes.c_int, [ctypes.POINTER(_CTX), ctypes.POINTER(asaga_problem), ctypes.POINTER(asaga_opts)]),
    "asaga_init_batched": (ctypes.c_int, [ctypes.POINTER(_CTX), ctypes.POINTER(asaga_problem),
                                          ctypes.POINTER(asaga_opts), ctypes.POINTER(asaga_batch)]),
    "asaga_epochs": (ctypes.c_int, [_CTX, ctypes.c_int64]),
    "asaga_set_active": (ctypes.c_int, [_CTX, _P]),
    "asaga_set_stop": (ctypes.c_int, [_CTX, _P]),
    "asaga_stop_report": (ctypes.c_int, [_CTX, _P, _P]),
    "asaga_updates": (ctypes.c_int, [_CTX, ctypes.c_int64]),
    "asaga_objective": (ctypes.c_int, [_CTX, ctypes.c_int32, _P, ctypes.POINTER(ctypes.c_double)]),
    "asaga_objective_noalloc": (ctypes.c_int, [ctypes.POINTER(asaga_problem), _P, _P, _P]),
    "asaga_full_grad": (ctypes.c_int, [_CTX, ctypes.c_int32, _P, _P]),
    "asaga_get_x": (ctypes.c_int, [_CTX, ctypes.c_int32, _P]),
    "asaga_get_state": (ctypes.c_int, [_CTX, ctypes.c_int32, _P, _P, _P, ctypes.POINTER(ctypes.c_int64)]),
    "asaga_set_state": (ctypes.c_int, [_CTX, ctypes.c_int32, _P, _P, _P, ctypes.POINTER(ctypes.c_int64)]),
    "asaga_reanchor": (ctypes.c_int, [_CTX]),
    "asaga_widen": (ctypes.c_int, [_CTX]),
    "asaga_autotune": (ctypes.c_int, [_CTX, ctypes.c_double, ctypes.c_int32, ctypes.POINTER(asaga_tune_report)]),
    "asaga_overlap": (ctypes.c_int, [_CTX, ctypes.c_int64, ctypes.POINTER(asaga_overlap_report)]),
    "asaga_overlap_estimate": (ctypes.c_int, [_P, ctypes.c_int64, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                              ctypes.POINTER(asaga_overlap_report)]),
    "asaga_info_get": (ctypes.c_int, [_CTX, ctypes.POINTER(asaga_info)]),
    "asaga_instance_get": (ctypes.c_int, [_CTX, ctypes.c_int32, ctypes.POINTER(asaga_instance)]),
    "asaga_sync": (ctypes.c_int, [_CTX]),
    "asaga_sample_stream": (ctypes.c_int, [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int64, ctypes.c_int64, _P]),
    "asaga_request_ceiling": (ctypes.c_int, [ctypes.c_int64, ctypes.POINTER(ctypes.c_double),
                                             ctypes.POINTER(ctypes.c_double)]),
    "asaga_last_error": (ctypes.c_char_p, [_CTX]),
    "asaga_free": (None, [_CTX]),
}
for _name, (_res, _args) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args

EXPORTED = tuple(_SIGS)


def hip_runtimes_loaded() -> list[str]:
    """Paths of the libamdhip64 copies mapped into this process (one is
    expected)."""
    paths = set()
    with open("/proc/self/maps") as fh:
        for line in fh:
            if "libamdhip64" in line:
                paths.add(line.split()[-1])
    return sorted(paths)


class AsagaError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


def _check(rc: int, ctx=None):
    if rc != ASAGA_OK:
        raise AsagaError(rc, asaga_last_error(ctx))
    return rc


# ---- the C functions, same names ---------------------------------------------
def asaga_init(prob: asaga_problem, opts: asaga_opts):
    ctx = _CTX()
    _check(_lib.asaga_init(ctypes.byref(ctx), ctypes.byref(prob), ctypes.byref(opts)))
    return ctx


def asaga_init_batched(prob: asaga_problem, opts: asaga_opts, batch: asaga_batch):
    ctx = _CTX()
    _check(_lib.asaga_init_batched(ctypes.byref(ctx), ctypes.byref(prob), ctypes.byref(opts), ctypes.byref(batch)))
    return ctx


def asaga_epochs(ctx, n_epochs: int):
    return _check(_lib.asaga_epochs(ctx, int(n_epochs)), ctx)


def asaga_set_active(ctx, active):
    a = np.ascontiguousarray(active, dtype=np.uint8)
    return _check(_lib.asaga_set_active(ctx, a.ctypes.data), ctx)


def asaga_set_stop(ctx, thresholds):
    if thresholds is None:
        return _check(_lib.asaga_set_stop(ctx, None), ctx)
    t = np.ascontiguousarray(thresholds, dtype=np.float64)
    return _check(_lib.asaga_set_stop(ctx, t.ctypes.data), ctx)


def asaga_stop_report(ctx, n_inst: int):
    proxy = np.empty(n_inst, dtype=np.float64)
    epochs = np.empty(n_inst, dtype=np.int64)
    _check(_lib.asaga_stop_report(ctx, proxy.ctypes.data, epochs.ctypes.data), ctx)
    return proxy, epochs


def asaga_updates(ctx, count: int):
    return _check(_lib.asaga_updates(ctx, int(count)), ctx)


def _host_f64(x, size):
    if x is None:
        return None, None
    a = np.ascontiguousarray(x, dtype=np.float64)
    if a.shape != (size,):
        raise ValueError(f"expected a vector of length {size}")
    return a, a.ctypes.data


def asaga_objective(ctx, inst: int, d: int, x=None) -> float:
    keep, px = _host_f64(x, d)
    f = ctypes.c_double()
    _check(_lib.asaga_objective(ctx, int(inst), px, ctypes.byref(f)), ctx)
    return f.value


def asaga_objective_noalloc(prob: asaga_problem, x_dev: int, f_dev: int, stream=None):
    """Enqueue f(x) of a device-resident problem into the device double at
    f_dev (x_dev: device double[d]); allocates nothing.  ``stream``: a
    torch.cuda.Stream or a raw hipStream_t integer (None: null stream)."""
    if stream is not None and not isinstance(stream, int):
        stream = stream.cuda_stream
    return _check(_lib.asaga_objective_noalloc(ctypes.byref(prob), x_dev, f_dev, stream))


def asaga_full_grad(ctx, inst: int, d: int, x=None) -> np.ndarray:
    keep, px = _host_f64(x, d)
    g = np.empty(d)
    _check(_lib.asaga_full_grad(ctx, int(inst), px, g.ctypes.data), ctx)
    return g


def asaga_get_x(ctx, inst: int, d: int) -> np.ndarray:
    x = np.empty(d)
    _check(_lib.asaga_get_x(ctx, int(inst), x.ctypes.data), ctx)
    return x


def asaga_get_state(ctx, inst: int, d: int):
    m = asaga_instance_get(ctx, inst).m
    x, alpha, abar = np.empty(d), np.empty(m), np.empty(d)
    t = ctypes.c_int64()
    _check(_lib.asaga_get_state(ctx, int(inst), x.ctypes.data, alpha.ctypes.data, abar.ctypes.data, ctypes.byref(t)),
           ctx)
    return x, alpha, abar, int(t.value)


def asaga_set_state(ctx, inst: int, d: int, x=None, alpha=None, abar=None, t=None):
    m = asaga_instance_get(ctx, inst).m
    kx, px = _host_f64(x, d)
    ka, pa = _host_f64(alpha, m)
    kb, pb = _host_f64(abar, d)
    tt = ctypes.c_int64(int(t)) if t is not None else None
    _check(_lib.asaga_set_state(ctx, int(inst), px, pa, pb, ctypes.byref(tt) if tt is not None else None), ctx)


def asaga_reanchor(ctx):
    return _check(_lib.asaga_reanchor(ctx), ctx)


def asaga_widen(ctx):
    return _check(_lib.asaga_widen(ctx), ctx)


def asaga_autotune(ctx, target: float = 1e-9, probe_epochs: int = 9) -> asaga_tune_report:
    rep = asaga_tune_report()
    _check(_lib.asaga_autotune(ctx, float(target), int(probe_epochs), ctypes.byref(rep)), ctx)
    return rep


def asaga_overlap(ctx, n_epochs: int = 1) -> asaga_overlap_report:
    rep = asaga_overlap_report()
    _check(_lib.asaga_overlap(ctx, int(n_epochs), ctypes.byref(rep)), ctx)
    return rep


def asaga_overlap_estimate(log, every: int, clock_hz: float, updates_per_s: float = 0.0) -> asaga_overlap_report:
    a = np.ascontiguousarray(log, dtype=np.int64).reshape(-1, 2)
    rep = asaga_overlap_report()
    _check(_lib.asaga_overlap_estimate(a.ctypes.data, len(a), int(every), float(clock_hz), float(updates_per_s),
                                       ctypes.byref(rep)))
    return rep


def asaga_instance_get(ctx, inst: int) -> asaga_instance:
    out = asaga_instance()
    _check(_lib.asaga_instance_get(ctx, int(inst), ctypes.byref(out)), ctx)
    return out


def asaga_info_get(ctx) -> asaga_info:
    info = asaga_info()
    _check(_lib.asaga_info_get(ctx, ctypes.byref(info)), ctx)
    return info


def asaga_sync(ctx):
    return _check(_lib.asaga_sync(ctx), ctx)


def asaga_request_ceiling(columns: int) -> tuple[float, float]:
    """(atomic-only, read + atomic) memory-side requests per second of the
    device, measured over a state of `columns` columns."""
    a, m = ctypes.c_double(0.0), ctypes.c_double(0.0)
    _check(_lib.asaga_request_ceiling(int(columns), ctypes.byref(a), ctypes.byref(m)))
    return a.value, m.value


def asaga_sample_stream(seed: int, t0: int, count: int, n: int) -> np.ndarray:
    out = np.empty(count, dtype=np.int64)
    _check(_lib.asaga_sample_stream(int(seed), int(t0), int(count), int(n), out.ctypes.data))
    return out


def asaga_last_error(ctx=None) -> str:
    s = _lib.asaga_last_error(ctx)
    return s.decode() if s else ""


def asaga_free(ctx):
    _lib.asaga_free(ctx)


# ---- one context -------------------------------------------------------------
def _is_torch_cuda(a) -> bool:
    return type(a).__module__.startswith("torch") and getattr(a, "is_cuda", False)


class Solver:
    """One library context over a CSR problem.

    ``rowptr`` int64[n+1], ``colidx`` int32[nnz], ``val`` float64/float32
    or bfloat16 bit patterns (uint16, with ``val_dtype=ASAGA_VAL_BF16``),
    ``b`` float64[n].  All four are numpy arrays (copied to the device) or
    all four are torch CUDA tensors (borrowed; this object keeps them
    alive).  ``stream`` is a torch.cuda.Stream or a raw hipStream_t integer.
    """

    def __init__(self, n, d, rowptr, colidx, val, b, lam, loss=ASAGA_LOSS_LOGISTIC, val_dtype=None,
                 mode=ASAGA_MODE_SERIAL, precision=ASAGA_PREC_F64, step=0.0, seed=0, waves=0,
                 lanes_per_sample=0, racy=0, hot_columns=0, flush_every=0, threads_per_block=0,
                 hot_tier_columns=0, hot_tier_every=0, plain_launch=0, method=ASAGA_METHOD_SAGA, stream=None,
                 batch=None, hot_reload_from=0):
        self.n, self.d = int(n), int(d)
        arrays = (rowptr, colidx, val, b)
        on_dev = [_is_torch_cuda(a) for a in arrays]
        if any(on_dev) and not all(on_dev):
            raise ValueError("problem arrays must all be numpy arrays or all be torch CUDA tensors")
        if all(on_dev):
            mem = ASAGA_MEM_DEVICE
            self._keep = arrays
            ptrs = [a.data_ptr() for a in arrays]
            if val_dtype is None:
                val_dtype = {8: ASAGA_VAL_F64, 4: ASAGA_VAL_F32, 2: ASAGA_VAL_BF16}[val.element_size()]
        else:
            mem = ASAGA_MEM_HOST
            rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
            colidx = np.ascontiguousarray(colidx, dtype=np.int32)
            if val_dtype is None:
                val_dtype = {np.dtype(np.float64): ASAGA_VAL_F64, np.dtype(np.float32): ASAGA_VAL_F32,
                             np.dtype(np.uint16): ASAGA_VAL_BF16}[np.asarray(val).dtype]
            vdt = {ASAGA_VAL_F64: np.float64, ASAGA_VAL_F32: np.float32, ASAGA_VAL_BF16: np.uint16}[val_dtype]
            val = np.ascontiguousarray(val, dtype=vdt)
            b = np.ascontiguousarray(b, dtype=np.float64)
            self._keep = (rowptr, colidx, val, b)
            ptrs = [a.ctypes.data for a in self._keep]
        self.prob = asaga_problem(self.n, self.d, *ptrs, float(lam), int(val_dtype), int(loss), mem, 0)
        if stream is not None and not isinstance(stream, int):
            stream = stream.cuda_stream
        self.opts = asaga_opts(float(step), int(seed), int(mode), int(precision), int(waves), int(lanes_per_sample),
                               int(racy), int(hot_columns), int(flush_every), int(threads_per_block),
                               int(hot_tier_columns), int(hot_tier_every), int(plain_launch), int(method), stream,
                               int(hot_reload_from), 0)
        if batch is None:
            self.ctx = asaga_init(self.prob, self.opts)
            self.n_inst = 1
        else:
            row_fold, inst_fold, inst_lambda = batch
            self._bkeep = (None if row_fold is None else np.ascontiguousarray(row_fold, dtype=np.int8),
                           np.ascontiguousarray(inst_fold, dtype=np.int32),
                           np.ascontiguousarray(inst_lambda, dtype=np.float64))
            rf, inf_, il = self._bkeep
            bt = asaga_batch(len(inf_), 0, None if rf is None else rf.ctypes.data, inf_.ctypes.data, il.ctypes.data)
            self.ctx = asaga_init_batched(self.prob, self.opts, bt)
            self.n_inst = len(inf_)

    # marshalling wrappers
    def epochs(self, e: int):
        asaga_epochs(self.ctx, e)

    def updates(self, count: int):
        asaga_updates(self.ctx, count)

    def set_active(self, active):
        if len(active) != self.n_inst:
            raise ValueError(f"expected {self.n_inst} flags")
        asaga_set_active(self.ctx, active)

    def set_stop(self, thresholds):
        """Arm the in-graph stop test with one threshold per instance, or
        disarm it (None)."""
        if thresholds is not None and len(thresholds) != self.n_inst:
            raise ValueError(f"expected {self.n_inst} thresholds")
        asaga_set_stop(self.ctx, thresholds)

    def stop_report(self):
        """(proxy, epochs): the stop test's last proxy and the epochs each
        instance ran in the last call with it armed."""
        return asaga_stop_report(self.ctx, self.n_inst)

    def objective(self, inst: int = 0, x=None) -> float:
        return asaga_objective(self.ctx, inst, self.d, x)

    def full_grad(self, inst: int = 0, x=None) -> np.ndarray:
        return asaga_full_grad(self.ctx, inst, self.d, x)

    def get_x(self, inst: int = 0) -> np.ndarray:
        return asaga_get_x(self.ctx, inst, self.d)

    def get_state(self, inst: int = 0):
        """(x, alpha, abar, t) of an instance; alpha has the instance's own
        length (its training rows)."""
        return asaga_get_state(self.ctx, inst, self.d)

    def set_state(self, inst: int = 0, **kw):
        asaga_set_state(self.ctx, inst, self.d, **kw)

    def instance(self, inst: int = 0) -> asaga_instance:
        return asaga_instance_get(self.ctx, inst)

    def reanchor(self):
        asaga_reanchor(self.ctx)

    def widen(self):
        asaga_widen(self.ctx)

    def autotune(self, target: float = 1e-9, probe_epochs: int = 9) -> asaga_tune_report:
        return asaga_autotune(self.ctx, target, probe_epochs)

    def overlap(self, n_epochs: int = 1) -> asaga_overlap_report:
        return asaga_overlap(self.ctx, n_epochs)

    def info(self) -> asaga_info:
        return asaga_info_get(self.ctx)

    def sync(self):
        asaga_sync(self.ctx)

    def close(self):
        if getattr(self, "ctx", None):
            asaga_free(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def from_problem(p, **kw) -> Solver:
    """Solver over a ``datagen.Problem``-like object (n, d, rowptr, colidx,
    val, b, loss, lam; optional val_bf16).  ``bf16=True`` passes the stored
    bfloat16 values instead of the float64 ones."""
    bf16 = kw.pop("bf16", False)
    val = p.val_bf16 if bf16 else p.val
    vdt = ASAGA_VAL_BF16 if bf16 else None
    return Solver(p.n, p.d, p.rowptr, p.colidx, val, p.b, p.lam, loss=p.loss, val_dtype=vdt, **kw)
