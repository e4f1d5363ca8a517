"""Seeded synthetic inputs for the Sparse SAGA / ASAGA workloads.

This module only builds problem instances (CSR matrices, labels, fold
assignments, lambda grids).  It holds none of the optimisation method's
arithmetic, and it is the one piece of code shared by the CPU oracle and the
HIP path: both consume the arrays it returns.

The paper's datasets (RCV1, URL, Covtype; Section 4.1 and Appendix G) are not
available, so each generator stands in for one of them with the same shape
(n, d, support sizes) and a stated value distribution:

* ``config1``  tiny logistic instance (2,000 x 500, 25 uniform columns/row).
* ``config2``  RCV1-like: 700,000 x 47,000, Poisson(75) distinct Zipf(1.1)
  columns per row, TF-IDF-like values (lognormal(0,1) term weight times the
  smooth inverse document frequency ln((1+n)/(1+df_v)) + 1 of the column),
  rows L2-normalised, planted labels with 10% flips.
* ``config3``  Covtype-like least squares: 581,000 x 54, ten standardised
  Gaussian columns plus one-hot blocks of 4 and 40 columns (12 nnz/row),
  targets a.w* + N(0, 0.1^2).
* ``config4``  URL-like: 2,400,000 x 3,200,000, Poisson(115) distinct
  Zipf(1.2) columns, binary values row-normalised and stored as bfloat16,
  planted labels with 5% flips.
* ``folds5`` / ``lambda_grid5``  the cross-validation folds and regularisation
  path laid over the config-2 matrix for batched solves; ``config5`` puts
  them together over the bfloat16-stored config-2 matrix (160 instances).

Every random draw comes from ``numpy.random.default_rng`` seeded by
``SeedSequence([seed, tag])`` with one tag per independent sub-stream, plus a
small C sampler (``zipfrows.c``) for the per-row distinct column supports.
"""
from __future__ import annotations

import ctypes
import hashlib
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

LOGISTIC = 0
SQUARED = 1

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libdatagen.so")
_lib = None

# independent sub-stream tags
_T_SUPPORT, _T_COUNTS, _T_VALUES, _T_WSTAR, _T_FLIPS, _T_NOISE, _T_FOLDS, _T_PERM, _T_CATS = range(1, 10)


def build(force: bool = True) -> str:
    """Compile the C column sampler in place (gcc, OpenMP)."""
    if force or not os.path.exists(_LIB_PATH):
        src = os.path.join(_HERE, "zipfrows.c")
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", src, "-o", tmp])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=True)
        lib = ctypes.CDLL(_LIB_PATH)
        lib.datagen_distinct_rows.restype = ctypes.c_int
        lib.datagen_distinct_rows.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64,
                                              ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                              ctypes.c_void_p]
        _lib = lib
    return _lib


@dataclass
class Problem:
    """A CSR problem instance.  ``val`` is always float64 (for bfloat16
    instances it holds the exactly widened stored values); ``val_bf16`` holds
    the raw bfloat16 bit patterns when the instance is stored in bfloat16."""
    name: str
    n: int
    d: int
    rowptr: np.ndarray        # int64 [n+1]
    colidx: np.ndarray        # int32 [nnz], strictly increasing within a row
    val: np.ndarray           # float64 [nnz]
    b: np.ndarray             # float64 [n]
    loss: int                 # LOGISTIC or SQUARED
    lam: float
    val_bf16: np.ndarray | None = None
    meta: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    def digest(self) -> str:
        """sha256 over the arrays, to check that a regenerated instance is
        the one a stored value was computed on."""
        h = hashlib.sha256()
        for a in (self.rowptr, self.colidx, self.val, self.b):
            h.update(np.ascontiguousarray(a).tobytes())
        h.update(repr((self.n, self.d, self.loss, float(self.lam))).encode())
        return h.hexdigest()

    def dense(self) -> np.ndarray:
        A = np.zeros((self.n, self.d))
        rows = np.repeat(np.arange(self.n), np.diff(self.rowptr))
        A[rows, self.colidx] = self.val
        return A


def _rng(seed: int, tag: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([int(seed), int(tag)]))


def _distinct_supports(seed: int, n: int, d: int, counts: np.ndarray, cdf: np.ndarray,
                       perm: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    counts = np.minimum(np.asarray(counts, dtype=np.int64), d)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    colidx = np.empty(int(rowptr[-1]), dtype=np.int32)
    row_seed = _rng(seed, _T_SUPPORT).integers(0, 2**63, size=n, dtype=np.int64).astype(np.uint64)
    cdf = np.ascontiguousarray(cdf, dtype=np.float64)
    perm = np.ascontiguousarray(perm, dtype=np.int32)
    rc = _load().datagen_distinct_rows(row_seed.ctypes.data, n, d, cdf.ctypes.data, perm.ctypes.data,
                                       rowptr.ctypes.data, colidx.ctypes.data)
    if rc != 0:
        raise RuntimeError(f"datagen_distinct_rows failed ({rc})")
    return rowptr, colidx


def _zipf_cdf(d: int, s: float) -> np.ndarray:
    w = np.arange(1, d + 1, dtype=np.float64) ** (-s)
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    cdf[-1] = 1.0
    return cdf


def _row_normalise(rowptr: np.ndarray, val: np.ndarray) -> np.ndarray:
    sq = np.add.reduceat(val * val, rowptr[:-1])
    return val / np.repeat(np.sqrt(sq), np.diff(rowptr))


def _row_dot(rowptr, colidx, val, w):
    return np.add.reduceat(val * w[colidx], rowptr[:-1])


def _planted_labels(seed, rowptr, colidx, val, d, flip):
    wstar = _rng(seed, _T_WSTAR).standard_normal(d)
    z = _row_dot(rowptr, colidx, val, wstar)
    b = np.where(z >= 0.0, 1.0, -1.0)
    flips = _rng(seed, _T_FLIPS).random(len(b)) < flip
    b[flips] = -b[flips]
    return b


def config1(seed: int = 0, n: int = 2000, d: int = 500, k: int = 25) -> Problem:
    """Tiny logistic instance: k distinct uniform columns per row, N(0,1)
    values, rows L2-normalised, labels sign(a.w*) with 5% flips, lambda=1/n."""
    counts = np.full(n, k, dtype=np.int64)
    cdf = np.arange(1, d + 1, dtype=np.float64) / d
    rowptr, colidx = _distinct_supports(seed, n, d, counts, cdf, np.arange(d, dtype=np.int32))
    val = _row_normalise(rowptr, _rng(seed, _T_VALUES).standard_normal(len(colidx)))
    b = _planted_labels(seed, rowptr, colidx, val, d, 0.05)
    return Problem("config1", n, d, rowptr, colidx, val, b, LOGISTIC, 1.0 / n)


def config2(seed: int = 0, n: int = 700_000, d: int = 47_000, mean_nnz: float = 75.0,
            zipf_s: float = 1.1, idf: bool = True) -> Problem:
    """RCV1-like logistic instance (see module docstring).  Frequent columns
    get small weights, as term weighting does in text data.  idf=False
    gives the other reading of the values: lognormal(0, 1) alone, then
    row-normalised (the same supports)."""
    counts = np.maximum(1, _rng(seed, _T_COUNTS).poisson(mean_nnz, size=n))
    perm = _rng(seed, _T_PERM).permutation(d).astype(np.int32)
    rowptr, colidx = _distinct_supports(seed, n, d, counts, _zipf_cdf(d, zipf_s), perm)
    tf = _rng(seed, _T_VALUES).lognormal(0.0, 1.0, size=len(colidx))
    if idf:
        df = np.bincount(colidx, minlength=d)
        w = np.log((1.0 + n) / (1.0 + df)) + 1.0
        val = _row_normalise(rowptr, tf * w[colidx])
    else:
        val = _row_normalise(rowptr, tf)
    b = _planted_labels(seed, rowptr, colidx, val, d, 0.10)
    return Problem("config2", n, d, rowptr, colidx, val, b, LOGISTIC, 1.0 / n,
                   meta={"zipf_s": zipf_s, "mean_nnz": mean_nnz,
                         "values": "lognormal tf x smooth idf" if idf else "lognormal"})


def config3(seed: int = 0, n: int = 581_000, lam: float = 1e-4) -> Problem:
    """Covtype-like least-squares instance, d = 54, 12 nnz per row."""
    d = 54
    X = _rng(seed, _T_VALUES).standard_normal((n, 10))
    X = (X - X.mean(axis=0)) / X.std(axis=0)
    cats = _rng(seed, _T_CATS)
    c4 = cats.integers(0, 4, size=n)
    c40 = cats.integers(0, 40, size=n)
    colidx = np.empty((n, 12), dtype=np.int32)
    colidx[:, :10] = np.arange(10, dtype=np.int32)
    colidx[:, 10] = 10 + c4
    colidx[:, 11] = 14 + c40
    val = np.ones((n, 12))
    val[:, :10] = X
    rowptr = np.arange(0, 12 * n + 1, 12, dtype=np.int64)
    colidx = colidx.reshape(-1)
    val = val.reshape(-1)
    wstar = _rng(seed, _T_WSTAR).standard_normal(d)
    b = _row_dot(rowptr, colidx, val, wstar) + 0.1 * _rng(seed, _T_NOISE).standard_normal(n)
    return Problem("config3", n, d, rowptr, colidx, val, b, SQUARED, lam)


def bf16_round(x: np.ndarray) -> np.ndarray:
    """Round float64 values to bfloat16 (round to nearest, ties to even, via
    float32); returns the uint16 bit patterns."""
    f = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32)
    lsb = (f >> 16) & 1
    return ((f + np.uint32(0x7FFF) + lsb) >> 16).astype(np.uint16)


def bf16_widen(bits: np.ndarray) -> np.ndarray:
    return (bits.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def config4(seed: int = 0, n: int = 2_400_000, d: int = 3_200_000, mean_nnz: float = 115.0,
            zipf_s: float = 1.2) -> Problem:
    """URL-like logistic instance, values 1/sqrt(nnz_i) stored as bfloat16;
    the bfloat16-quantised matrix is the instance (``val`` is its exact
    float64 widening)."""
    counts = np.maximum(1, _rng(seed, _T_COUNTS).poisson(mean_nnz, size=n))
    perm = _rng(seed, _T_PERM).permutation(d).astype(np.int32)
    rowptr, colidx = _distinct_supports(seed, n, d, counts, _zipf_cdf(d, zipf_s), perm)
    k = np.diff(rowptr)
    bits = bf16_round(np.repeat(1.0 / np.sqrt(k.astype(np.float64)), k))
    val = bf16_widen(bits)
    b = _planted_labels(seed, rowptr, colidx, val, d, 0.05)
    return Problem("config4", n, d, rowptr, colidx, val, b, LOGISTIC, 1.0 / n, val_bf16=bits,
                   meta={"zipf_s": zipf_s, "mean_nnz": mean_nnz})


FOLD_SIZES_700K = (128_000, 134_000, 140_000, 146_000, 152_000)


def folds5(n: int, seed: int = 0) -> np.ndarray:
    """Five uneven cross-validation folds over n rows (sizes proportional to
    128k, 134k, 140k, 146k, 152k out of 700k), assigned through a seeded
    permutation.  Returns row_fold int8[n]."""
    sizes = np.floor(np.array(FOLD_SIZES_700K, dtype=np.float64) * n / 700_000).astype(np.int64)
    sizes[-1] = n - sizes[:-1].sum()
    perm = _rng(seed, _T_FOLDS).permutation(n)
    row_fold = np.empty(n, dtype=np.int8)
    start = 0
    for f, s in enumerate(sizes):
        row_fold[perm[start:start + s]] = f
        start += s
    return row_fold


def lambda_grid5(count: int = 32, lo_exp: float = -8.0, hi_exp: float = -2.0) -> np.ndarray:
    """Log-spaced regularisation path, 10^(lo + (hi-lo) k/(count-1))."""
    k = np.arange(count, dtype=np.float64)
    return 10.0 ** (lo_exp + (hi_exp - lo_exp) * k / max(count - 1, 1))


def subproblem(p: Problem, rows: np.ndarray, lam: float | None = None, name: str | None = None) -> Problem:
    """The instance restricted to the given rows (in the given order)."""
    rows = np.asarray(rows, dtype=np.int64)
    starts = p.rowptr[rows]
    k = p.rowptr[rows + 1] - starts
    rowptr = np.zeros(len(rows) + 1, dtype=np.int64)
    np.cumsum(k, out=rowptr[1:])
    gather = np.repeat(starts - rowptr[:-1], k) + np.arange(int(rowptr[-1]))
    bits = p.val_bf16[gather] if p.val_bf16 is not None else None
    return Problem(name or p.name + "_sub", len(rows), p.d, rowptr, p.colidx[gather], p.val[gather],
                   p.b[rows], p.loss, p.lam if lam is None else lam, val_bf16=bits, meta=dict(p.meta))


@dataclass
class Batch:
    """Many solves over one shared matrix: instance k trains on the rows
    whose fold differs from ``inst_fold[k]`` (all rows if it is -1), with
    regularisation ``inst_lambda[k]``."""
    problem: Problem
    row_fold: np.ndarray      # int8 [n]
    inst_fold: np.ndarray     # int32 [n_inst]
    inst_lambda: np.ndarray   # float64 [n_inst]

    @property
    def n_inst(self) -> int:
        return len(self.inst_fold)

    def rows(self, k: int) -> np.ndarray:
        f = int(self.inst_fold[k])
        return np.arange(self.problem.n) if f < 0 else np.nonzero(self.row_fold != f)[0]

    def instance(self, k: int) -> Problem:
        """Instance k as a problem of its own (its training rows in matrix order)."""
        return subproblem(self.problem, self.rows(k), lam=float(self.inst_lambda[k]),
                          name=f"{self.problem.name}[{k}]")


def config5(seed: int = 0, n: int = 700_000, d: int = 47_000, n_lambda: int = 32, **kw) -> Batch:
    """The config-2 matrix with its values stored as bfloat16 (the quantised
    matrix is the instance, ``val`` its exact float64 widening; labels are
    config 2's), five uneven folds and a 32-value lambda path over
    1e-8..1e-2: 160 instances, lambda-major (instance k = lambda index k // 5,
    fold k % 5)."""
    p = config2(seed=seed, n=n, d=d, **kw)
    bits = bf16_round(p.val)
    q = Problem("config5", p.n, p.d, p.rowptr, p.colidx, bf16_widen(bits), p.b, p.loss, p.lam, val_bf16=bits,
                meta=dict(p.meta))
    lams = lambda_grid5(n_lambda)
    inst_fold = np.tile(np.arange(5, dtype=np.int32), n_lambda)
    inst_lambda = np.repeat(lams, 5)
    return Batch(q, folds5(p.n, seed), inst_fold, inst_lambda)


def by_name(name: str, **kw) -> Problem:
    return {"config1": config1, "config2": config2, "config3": config3, "config4": config4}[name](**kw)
