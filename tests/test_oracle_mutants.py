"""Planted mistakes in the oracle (CPU only): each plausible slip -- a
dropped term, a wrong sign, an inverted ratio, a wrong index -- is compiled
into a copy of the oracle, and at least one pin of the kind that
test_oracle_pins.py uses must reject that copy."""
import os
import subprocess

import numpy as np
import pytest

import oracle
from conftest import ROOT, rel_err
from test_oracle_pins import csr_problem, random_sparse, scipy_csr

SRC = os.path.join(ROOT, "oracle", "saga_oracle.c")

MUTANTS = {
    "dropped lambda term": ("D[v] * (ab + lambda * xo)", "D[v] * (ab)"),
    "dropped abar term": ("D[v] * (ab + lambda * xo)", "D[v] * (lambda * xo)"),
    "abar update sign": ("abar[v] = ab + delta * val[k] / (double)n;", "abar[v] = ab - delta * val[k] / (double)n;"),
    "abar not divided by n": ("abar[v] = ab + delta * val[k] / (double)n;", "abar[v] = ab + delta * val[k];"),
    "memory not updated": ("alpha[i] = alpha[i] + delta;", "alpha[i] = alpha[i];"),
    "memory stores delta": ("alpha[i] = alpha[i] + delta;", "alpha[i] = delta;"),
    "inverted reweighting": ("(double)n / (double)cnt[v]", "(double)cnt[v] / (double)n"),
    "logistic derivative sign": ("return -b / (1.0 + exp(m));", "return b / (1.0 + exp(m));"),
    "logistic branch swapped": ("return -b * e / (1.0 + e);", "return -b / (1.0 + e);"),
    "wrong dot index": ("z += val[k] * x[colidx[k]];", "z += val[k] * x[k % 2];"),
    "step misses gamma on delta": ("gamma * (delta * val[k] +", "(delta * val[k] +"),
    "squared loss derivative": ("if (loss == ORACLE_SQUARED) return z - b;", "if (loss == ORACLE_SQUARED) return b - z;"),
}


def build_mutant(tmp_path, name, old, new):
    src = open(SRC).read()
    assert src.count(old) >= 1, name
    mutated = src.replace(old, new)
    c = tmp_path / "m.c"
    c.write_text(mutated)
    so = tmp_path / "libm.so"
    subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-shared", "-fPIC", str(c), "-o", str(so), "-lm"])
    return oracle.load(str(so))


def pins_pass(lib) -> bool:
    """A compact run of the pins; False as soon as one fails."""
    try:
        rng = np.random.default_rng(42)
        # ridge closed form, sparse support
        p = random_sparse(rng, 60, 10, 0.35, oracle.SQUARED, 0.2)
        sv = oracle.SparseSaga(p, lib=lib)
        sv.epochs(600)
        Ad = p.dense()
        xstar = np.linalg.solve(Ad.T @ Ad / p.n + 0.2 * np.eye(p.d), Ad.T @ p.b / p.n)
        if not rel_err(sv.state.x, xstar) < 1e-10:
            return False
        # running-average invariant, logistic
        q = random_sparse(rng, 50, 20, 0.3, oracle.LOGISTIC, 0.02)
        sq = oracle.SparseSaga(q, seed=3, lib=lib)
        sq.epochs(2)
        rec = scipy_csr(q).T @ sq.state.alpha / q.n
        if not np.max(np.abs(sq.state.abar - rec)) <= 1e-12 * max(1.0, np.max(np.abs(rec))):
            return False
        # unbiasedness against the dense gradient, logistic
        r = random_sparse(rng, 25, 9, 0.3, oracle.LOGISTIC, 0.07)
        sr = oracle.SparseSaga(r, lib=lib)
        Ar = r.dense()
        x = rng.standard_normal(r.d) * 0.5
        al = rng.standard_normal(r.n) * 0.3
        ab = Ar.T @ al / r.n
        dirs = []
        for i in range(r.n):
            s = oracle.State(x.copy(), al.copy(), ab.copy())
            sr.run_indices([i], s)
            dirs.append((x - s.x) / sr.gamma)
        zz = Ar @ x
        grad = Ar.T @ (-r.b / (1 + np.exp(r.b * zz))) / r.n + r.lam * x
        if not rel_err(np.mean(dirs, axis=0), grad) < 1e-13:
            return False
        # n = 1 gradient descent, logistic, and the derivative by differences
        a = np.array([0.4, 0.0, -1.2, 0.7])
        one = csr_problem(a[None, :], [-1.0], 0.3, oracle.LOGISTIC)
        so = oracle.SparseSaga(one, step=0.4, lib=lib)
        xx = np.zeros(4)
        on = (a != 0).astype(float)
        for _ in range(10):
            so.run_indices([0])
            zz = a @ xx
            xx = xx - 0.4 * ((1.0 / (1 + np.exp(-zz))) * a + 0.3 * on * xx)
        if not rel_err(so.state.x, xx) < 1e-14:
            return False
        h = 1e-5
        for loss, b in ((oracle.LOGISTIC, 1.0), (oracle.LOGISTIC, -1.0), (oracle.SQUARED, 0.3)):
            for z in (-3.0, 0.0, 2.0):
                fd = (lib.oracle_phi(z + h, b, loss) - lib.oracle_phi(z - h, b, loss)) / (2 * h)
                if abs(fd - lib.oracle_dphi(z, b, loss)) > 1e-8 * max(1.0, abs(fd)):
                    return False
        return True
    except (RuntimeError, FloatingPointError, np.linalg.LinAlgError):
        return False


def test_unmutated_oracle_passes(tmp_path):
    lib = build_mutant(tmp_path, "identity", "#include <math.h>", "#include <math.h>")
    assert pins_pass(lib)


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(tmp_path, name):
    old, new = MUTANTS[name]
    with np.errstate(all="ignore"):
        assert not pins_pass(build_mutant(tmp_path, name, old, new)), name


# Planted mistakes in the sparse SVRG path, against its own pins.
SVRG_MUTANTS = {
    "svrg snapshot sign": ("alpha[i] = oracle_dphi(z, b[i], loss);", "alpha[i] = -oracle_dphi(z, b[i], loss);"),
    "svrg snapshot average not divided": ("abar[v] /= (double)n;", "abar[v] /= 1.0;"),
    "svrg step drops lambda": ("D[v] * (abar[v] + lambda * xo)", "D[v] * (abar[v])"),
    "svrg step drops the snapshot gradient": ("D[v] * (abar[v] + lambda * xo)", "D[v] * (lambda * xo)"),
    "svrg full gradient never due": ("return oracle_sample(seed ^ ORACLE_SVRG_TAG, t, n) == 0;", "return 0;"),
    "svrg full gradient always due": ("return oracle_sample(seed ^ ORACLE_SVRG_TAG, t, n) == 0;", "return 1;"),
}


def svrg_pins_pass(lib) -> bool:
    """A compact run of the SVRG pins; False as soon as one fails."""
    try:
        rng = np.random.default_rng(7)
        n, T = 500, 200_000
        due = sum(lib.oracle_svrg_full_gradient_due(3, t, n) for t in range(T))
        if abs(due - T / n) > 5 * np.sqrt(T / n):
            return False
        p = random_sparse(rng, 30, 10, 0.35, oracle.LOGISTIC, 0.05)
        sv = oracle.SparseSvrg(p, lib=lib)
        A = p.dense()
        xt = rng.standard_normal(p.d) * 0.5
        snap = oracle.State(xt.copy(), np.zeros(p.n), np.zeros(p.d))
        sv.snapshot(snap)
        zt = A @ xt
        alpha = -p.b * np.exp(-np.logaddexp(0.0, p.b * zt))
        if not (rel_err(snap.alpha, alpha) < 1e-13 and rel_err(snap.abar, A.T @ alpha / p.n) < 1e-13):
            return False
        x = rng.standard_normal(p.d) * 0.5
        dirs = []
        for i in range(p.n):
            s = oracle.State(x.copy(), snap.alpha.copy(), snap.abar.copy())
            sv.run_indices([i], s)
            dirs.append((x - s.x) / sv.gamma)
        z = A @ x
        grad = A.T @ (-p.b * np.exp(-np.logaddexp(0.0, p.b * z))) / p.n + p.lam * x
        if not rel_err(np.mean(dirs, axis=0), grad) < 1e-13:
            return False
        q = random_sparse(rng, 60, 10, 0.35, oracle.SQUARED, 0.2)
        sq = oracle.SparseSvrg(q, seed=4, lib=lib)
        sq.epochs(400)
        Aq = q.dense()
        xstar = np.linalg.solve(Aq.T @ Aq / q.n + 0.2 * np.eye(q.d), Aq.T @ q.b / q.n)
        return bool(rel_err(sq.state.x, xstar) < 1e-10)
    except (RuntimeError, FloatingPointError, np.linalg.LinAlgError):
        return False


def test_unmutated_oracle_passes_svrg_pins(tmp_path):
    lib = build_mutant(tmp_path, "identity", "#include <math.h>", "#include <math.h>")
    assert svrg_pins_pass(lib)


@pytest.mark.parametrize("name", sorted(SVRG_MUTANTS))
def test_svrg_mutant_is_caught(tmp_path, name):
    old, new = SVRG_MUTANTS[name]
    with np.errstate(all="ignore"):
        assert not svrg_pins_pass(build_mutant(tmp_path, name, old, new)), name


# Planted mistakes in the dense and lagged SAGA paths.
DENSE_LAGGED_MUTANTS = {
    "dense drops lambda": ("x[v] = x[v] - gamma * (abar[v] + lambda * x[v]);", "x[v] = x[v] - gamma * (abar[v]);"),
    "dense drops abar": ("x[v] = x[v] - gamma * (abar[v] + lambda * x[v]);", "x[v] = x[v] - gamma * (lambda * x[v]);"),
    "lagged catch-up sign": ("x[v] = q * x[v] + expm1(lq) * abar[v] / lambda;",
                             "x[v] = q * x[v] - expm1(lq) * abar[v] / lambda;"),
    "lagged forgets the decay": ("x[v] = q * x[v] + expm1(lq) * abar[v] / lambda;",
                                 "x[v] = x[v] + expm1(lq) * abar[v] / lambda;"),
    "lagged counter not advanced": ("            last[v] = t + 1;\n", "            last[v] = t;\n"),
}


def dense_lagged_pins_pass(lib) -> bool:
    try:
        rng = np.random.default_rng(9)
        p = random_sparse(rng, 60, 10, 0.35, oracle.SQUARED, 0.2)
        sv = oracle.DenseSaga(p, seed=2, lib=lib)
        sv.epochs(600)
        A = p.dense()
        xstar = np.linalg.solve(A.T @ A / p.n + 0.2 * np.eye(p.d), A.T @ p.b / p.n)
        if not rel_err(sv.state.x, xstar) < 1e-10:
            return False
        q = random_sparse(rng, 80, 30, 0.1, oracle.LOGISTIC, 0.01)
        dense = oracle.DenseSaga(q, seed=5, lib=lib)
        lag = oracle.LaggedSaga(q, seed=5, lib=lib)
        for _ in range(3):
            dense.epochs(1)
            lag.epochs(1)
            if not rel_err(lag.state.x, dense.state.x) < 1e-12:
                return False
        return True
    except (RuntimeError, FloatingPointError, np.linalg.LinAlgError):
        return False


def test_unmutated_oracle_passes_dense_lagged_pins(tmp_path):
    lib = build_mutant(tmp_path, "identity", "#include <math.h>", "#include <math.h>")
    assert dense_lagged_pins_pass(lib)


@pytest.mark.parametrize("name", sorted(DENSE_LAGGED_MUTANTS))
def test_dense_lagged_mutant_is_caught(tmp_path, name):
    old, new = DENSE_LAGGED_MUTANTS[name]
    with np.errstate(all="ignore"):
        assert not dense_lagged_pins_pass(build_mutant(tmp_path, name, old, new)), name


DELAYED_MUTANTS = {
    "delayed read adds the missing writes": ("xh[k - rs] = x[v] - miss_x[v];", "xh[k - rs] = x[v] + miss_x[v];"),
    "delayed window one update short": ("int64_t first = s - tau > 0 ? s - tau : 0;",
                                        "int64_t first = s - tau + 1 > 0 ? s - tau + 1 : 0;"),
    "delayed memory read current": ("(alpha[i] - miss_alpha)", "(alpha[i])"),
    "delayed abar read current": ("abh[k - rs] = abar[v] - miss_ab[v];", "abh[k - rs] = abar[v];"),
    "delayed scratch not cleared": ("                miss_x[colidx[k]] = 0.0;\n", ""),
    "delayed write uses the current x": ("D[v] * (abh[k - rs] + lambda * xh[k - rs])",
                                         "D[v] * (abh[k - rs] + lambda * x[v])"),
}


def delayed_pins_pass(lib) -> bool:
    from test_oracle_pins import delayed_full_miss_brute_force
    try:
        rng = np.random.default_rng(31)
        for loss in (oracle.LOGISTIC, oracle.SQUARED):
            p = random_sparse(rng, 20, 9, 0.4, loss, 0.05)
            for tau in (1, 3, 11):
                sv = oracle.DelayedSparseSaga(p, tau=tau, miss=1.0, seed=2, lib=lib)
                sv.run(240)
                x, alpha, abar = delayed_full_miss_brute_force(p, sv, 240, tau)
                if not (rel_err(sv.state.x, x) < 1e-12 and rel_err(sv.state.alpha, alpha) < 1e-12
                        and rel_err(sv.state.abar, abar) < 1e-12):
                    return False
        return True
    except (RuntimeError, FloatingPointError):
        return False


def test_delayed_pins_pass_on_the_oracle():
    assert delayed_pins_pass(oracle.load())


@pytest.mark.parametrize("name", sorted(DELAYED_MUTANTS))
def test_delayed_mutant_is_caught(tmp_path, name):
    old, new = DELAYED_MUTANTS[name]
    with np.errstate(all="ignore"):
        assert not delayed_pins_pass(build_mutant(tmp_path, name, old, new)), name
