"""Pins of the CPU oracle to facts outside itself: published generator
outputs, calculus, closed forms, identities proved in the paper, special
cases that reduce to textbook methods.  CPU only."""
import numpy as np
import pytest
import scipy.sparse as sp

import datagen
import oracle
from conftest import rel_err


def csr_problem(A, b, lam, loss, mask=None, name="tiny"):
    """Problem from a dense matrix; `mask` marks the stored entries (the
    structural support), default: the nonzeros."""
    A = np.asarray(A, dtype=np.float64)
    mask = (A != 0) if mask is None else np.asarray(mask, dtype=bool)
    n, d = A.shape
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(mask.sum(axis=1), out=rowptr[1:])
    rr, cc = np.nonzero(mask)
    return datagen.Problem(name, n, d, rowptr, cc.astype(np.int32), A[rr, cc].copy(), np.asarray(b, float), loss, lam)


def random_sparse(rng, n, d, density, loss, lam):
    while True:
        mask = rng.random((n, d)) < density
        if mask.sum(axis=1).min() > 0:
            break
    A = rng.standard_normal((n, d)) * mask
    if loss == oracle.LOGISTIC:
        b = np.where(rng.random(n) < 0.5, 1.0, -1.0)
    else:
        b = rng.standard_normal(n)
    return csr_problem(A, b, lam, loss, mask)


def scipy_csr(p):
    return sp.csr_matrix((p.val, p.colidx, p.rowptr), shape=(p.n, p.d))


# ---------------------------------------------------------------------------
# sample stream
# ---------------------------------------------------------------------------

def test_splitmix64_published_vector():
    # SplitMix64 started from state 1234567: the first five outputs of the
    # reference implementation of Steele, Lea & Flood's generator.
    want = [6457827717110365317, 3203168211198807973, 9817491932198370423, 4593380528125082431,
            16408922859458223821]
    assert [oracle.splitmix64(1234567, t) for t in range(5)] == want


def test_sample_index_is_high_bits_for_powers_of_two():
    for k in (1, 5, 17, 31):
        idx = oracle.sample_stream(7, 100, 1000, 1 << k)
        raw = np.array([oracle.splitmix64(7, 100 + t) for t in range(1000)], dtype=np.uint64)
        assert np.array_equal(idx.astype(np.uint64), raw >> np.uint64(64 - k))


def test_sample_stream_uniform():
    n = 1000
    idx = oracle.sample_stream(0, 0, 1_000_000, n)
    assert idx.min() >= 0 and idx.max() < n
    counts = np.bincount(idx, minlength=n)
    chi2 = float(((counts - 1000.0) ** 2 / 1000.0).sum())
    # 999 degrees of freedom: mean 999, sd ~44.7; 6 sd either side
    assert 999 - 6 * 44.7 < chi2 < 999 + 6 * 44.7


# ---------------------------------------------------------------------------
# losses: calculus and special values
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("loss", [oracle.LOGISTIC, oracle.SQUARED])
def test_dphi_is_derivative_of_phi(loss):
    h = 1e-5
    for b in (-1.0, 1.0) if loss == oracle.LOGISTIC else (-0.7, 0.0, 2.5):
        for z in (-30.0, -3.0, -0.4, 0.0, 0.25, 2.0, 17.0):
            fd = (oracle.phi(z + h, b, loss) - oracle.phi(z - h, b, loss)) / (2 * h)
            assert abs(fd - oracle.dphi(z, b, loss)) <= 1e-8 * max(1.0, abs(fd))


def test_logistic_special_values():
    L = oracle.LOGISTIC
    assert oracle.phi(0.0, 1.0, L) == pytest.approx(np.log(2.0), rel=1e-16)
    assert oracle.dphi(0.0, 1.0, L) == -0.5 and oracle.dphi(0.0, -1.0, L) == 0.5
    # no overflow far out; asymptotes log(1+e^-m) -> -m and -> e^-m
    assert oracle.phi(-800.0, 1.0, L) == pytest.approx(800.0, rel=1e-15)
    assert oracle.phi(800.0, 1.0, L) == 0.0
    assert oracle.phi(40.0, 1.0, L) == pytest.approx(np.exp(-40.0), rel=1e-15)
    assert oracle.dphi(-800.0, 1.0, L) == -1.0 and oracle.dphi(800.0, -1.0, L) == 1.0
    # phi(z; b) = phi(-z; -b)
    for z in (-2.0, 0.3, 5.0):
        assert oracle.phi(z, 1.0, L) == oracle.phi(-z, -1.0, L)


def test_objective_at_zero_and_gradient_by_differences():
    rng = np.random.default_rng(1)
    for loss in (oracle.LOGISTIC, oracle.SQUARED):
        p = random_sparse(rng, 30, 8, 0.4, loss, 0.05)
        sv = oracle.SparseSaga(p)
        f0 = sv.objective(np.zeros(p.d))
        want = np.log(2.0) if loss == oracle.LOGISTIC else 0.5 * np.mean(p.b ** 2)
        assert f0 == pytest.approx(want, rel=1e-15)
        x = rng.standard_normal(p.d) * 0.3
        g = sv.gradient(x)
        h = 1e-6
        fd = np.array([(sv.objective(x + h * e) - sv.objective(x - h * e)) / (2 * h) for e in np.eye(p.d)])
        assert rel_err(g, fd) < 1e-7


# ---------------------------------------------------------------------------
# T1: dense least squares converges to the ridge closed form
# ---------------------------------------------------------------------------

def test_ridge_closed_form_dense():
    # every row dense: p_v = 1, D = I, Sparse SAGA is SAGA (Section 2)
    rng = np.random.default_rng(2)
    n, d = 40, 6
    A = rng.standard_normal((n, d))
    b = rng.standard_normal(n)
    p = csr_problem(A, b, 0.1, oracle.SQUARED, mask=np.ones((n, d), bool))
    sv = oracle.SparseSaga(p)
    assert np.all(sv.D == 1.0)
    sv.epochs(400)
    xstar = np.linalg.solve(A.T @ A / n + 0.1 * np.eye(d), A.T @ b / n)
    assert rel_err(sv.state.x, xstar) < 1e-10


def test_ridge_closed_form_sparse_support():
    # with a sparse support D != I; the fixed point still solves the ridge
    # normal equations (D_i reweighting leaves the optimum unchanged)
    rng = np.random.default_rng(3)
    p = random_sparse(rng, 60, 10, 0.35, oracle.SQUARED, 0.2)
    sv = oracle.SparseSaga(p)
    assert not np.all(sv.D == 1.0)
    sv.epochs(600)
    A = p.dense()
    xstar = np.linalg.solve(A.T @ A / p.n + 0.2 * np.eye(p.d), A.T @ p.b / p.n)
    assert rel_err(sv.state.x, xstar) < 1e-10
    assert rel_err(oracle.ridge_solution(p), xstar) < 1e-12
    assert rel_err(oracle.ridge_solution_csr(p, rows_per_block=7), xstar) < 1e-12


# ---------------------------------------------------------------------------
# T2: abar = (1/n) sum_i alpha_i a_i after any number of updates
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("loss", [oracle.LOGISTIC, oracle.SQUARED])
def test_running_average_invariant(loss):
    rng = np.random.default_rng(4)
    p = random_sparse(rng, 50, 20, 0.3, loss, 0.02)
    sv = oracle.SparseSaga(p, seed=11)
    M = scipy_csr(p)
    for _ in range(5):
        sv.epochs(1.3)
        recomputed = M.T @ sv.state.alpha / p.n
        assert np.max(np.abs(sv.state.abar - recomputed)) <= 1e-12 * max(1.0, np.max(np.abs(recomputed)))
        assert np.max(np.abs(sv.memory_average() - recomputed)) <= 1e-15 * max(1.0, np.max(np.abs(recomputed)))


# ---------------------------------------------------------------------------
# T3: the sparse update is unbiased (Appendix B): averaging the update
# direction over all i gives dense SAGA's average, which is grad f
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("loss", [oracle.LOGISTIC, oracle.SQUARED])
def test_expected_update_equals_gradient(loss):
    rng = np.random.default_rng(5)
    p = random_sparse(rng, 25, 9, 0.3, loss, 0.07)
    sv = oracle.SparseSaga(p)
    A = p.dense()
    x = rng.standard_normal(p.d) * 0.5
    alpha = rng.standard_normal(p.n) * 0.3
    abar = A.T @ alpha / p.n                       # a consistent memory state
    dirs = []
    for i in range(p.n):
        s = oracle.State(x.copy(), alpha.copy(), abar.copy())
        sv.run_indices([i], s)
        dirs.append((x - s.x) / sv.gamma)
    mean_sparse = np.mean(dirs, axis=0)
    z = A @ x
    if loss == oracle.LOGISTIC:
        dphi = -p.b / (1.0 + np.exp(p.b * z))
    else:
        dphi = z - p.b
    # dense SAGA direction (Eq. SAGAupdate) with the L2 term: f'_i - alpha_i + abar + lambda x
    dense = np.mean([(dphi[i] - alpha[i]) * A[i] + abar + p.lam * x for i in range(p.n)], axis=0)
    grad = A.T @ dphi / p.n + p.lam * x
    assert rel_err(mean_sparse, dense) < 1e-13
    assert rel_err(mean_sparse, grad) < 1e-13
    assert rel_err(sv.gradient(x), grad) < 1e-14


# ---------------------------------------------------------------------------
# T4: variance identity of Appendix B:
#   E||alpha_i - D_i abar - c_i||^2 = E||alpha_i - c_i||^2 - abar' D abar
# for vectors alpha_i, c_i supported on S_i with E c_i = 0
# ---------------------------------------------------------------------------

def test_variance_identity_pins_reweighting():
    rng = np.random.default_rng(6)
    p = random_sparse(rng, 30, 8, 0.3, oracle.LOGISTIC, 0.1)
    sv = oracle.SparseSaga(p)
    A = p.dense()
    mask = A != 0
    s_alpha = rng.standard_normal(p.n)
    alpha_vec = s_alpha[:, None] * A
    # c_i = s_i a_i with A's = 0 (s in the null space of A')
    U, S, Vt = np.linalg.svd(A.T)
    s_c = Vt[-1] * 3.0
    c_vec = s_c[:, None] * A
    assert np.max(np.abs(c_vec.sum(axis=0))) < 1e-12
    abar = alpha_vec.mean(axis=0)
    lhs = np.mean([np.sum((alpha_vec[i] - mask[i] * sv.D * abar - c_vec[i]) ** 2) for i in range(p.n)])
    rhs = np.mean([np.sum((alpha_vec[i] - c_vec[i]) ** 2) for i in range(p.n)]) - abar @ (sv.D * abar)
    assert lhs == pytest.approx(rhs, rel=1e-12)
    # and E D_i abar = abar
    assert rel_err(np.mean(mask * sv.D * abar, axis=0), abar) < 1e-14


# ---------------------------------------------------------------------------
# T5: Remark 1 -- the smallest D with (1/n) sum ||x||_{S_i}^2 <= D ||x||^2
# is Delta_r / n, Delta_r = max column count
# ---------------------------------------------------------------------------

def test_remark1_sparsity_constant():
    rng = np.random.default_rng(7)
    p = random_sparse(rng, 40, 15, 0.25, oracle.LOGISTIC, 0.1)
    sv = oracle.SparseSaga(p)
    mask = p.dense() != 0
    M = sum(np.diag(mask[i].astype(float)) for i in range(p.n)) / p.n   # (1/n) sum_i P_{S_i}
    lam_max = np.linalg.eigvalsh(M).max()
    assert lam_max == pytest.approx(sv.cnt.max() / p.n, rel=1e-14)
    assert np.array_equal(sv.cnt, mask.sum(axis=0))
    assert np.allclose(sv.D, np.where(sv.cnt > 0, p.n / np.maximum(sv.cnt, 1), 0.0), rtol=0, atol=0)


# ---------------------------------------------------------------------------
# T6: n = 1 -- Sparse SAGA is gradient descent on the row's support
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("loss", [oracle.LOGISTIC, oracle.SQUARED])
def test_single_sample_is_gradient_descent(loss):
    rng = np.random.default_rng(8)
    d = 7
    a = np.zeros(d)
    supp = np.array([0, 2, 3, 6])
    a[supp] = rng.standard_normal(len(supp))
    b = 1.0 if loss == oracle.LOGISTIC else 0.8
    p = csr_problem(a[None, :], [b], 0.3, loss)
    sv = oracle.SparseSaga(p, step=0.4)
    x = np.zeros(d)
    on = np.zeros(d)
    on[supp] = 1.0
    for _ in range(25):
        sv.run_indices([0])
        z = a @ x
        g = (-b / (1 + np.exp(b * z))) if loss == oracle.LOGISTIC else z - b
        x = x - 0.4 * (g * a + 0.3 * on * x)        # gradient step of f restricted to S
        assert rel_err(sv.state.x, x) < 1e-14
    assert np.all(sv.state.x[on == 0] == 0.0)


# ---------------------------------------------------------------------------
# T7: Theorem 1 envelope, seed-averaged
# ---------------------------------------------------------------------------

def test_theorem1_envelope():
    rng = np.random.default_rng(9)
    p = random_sparse(rng, 20, 6, 0.5, oracle.LOGISTIC, 0.05)
    xstar = oracle.logistic_newton(p)
    sv0 = oracle.SparseSaga(p)
    L = sv0.L
    a_ = 1.0
    gamma = a_ / (5 * L)
    mu = p.lam
    rho = 0.2 * min(1.0 / p.n, a_ * mu / L)
    A = p.dense()
    z = A @ xstar
    gi = -p.b / (1 + np.exp(p.b * z))
    fi_star = gi[:, None] * A + p.lam * xstar        # f'_i(x*), alpha_i^0 = 0
    C0 = xstar @ xstar + np.sum(fi_star ** 2) / (5 * L ** 2)
    checkpoints = [p.n * k for k in (1, 5, 20, 60)]
    errs = np.zeros(len(checkpoints))
    seeds = 16
    for seed in range(seeds):
        sv = oracle.SparseSaga(p, step=gamma, seed=seed)
        done = 0
        for c, t in enumerate(checkpoints):
            sv.run(t - done)
            done = t
            errs[c] += np.sum((sv.state.x - xstar) ** 2) / seeds
    for c, t in enumerate(checkpoints):
        assert errs[c] <= (1 - rho) ** t * C0


# ---------------------------------------------------------------------------
# T8: the f* values the GPU results are compared with
# ---------------------------------------------------------------------------

def test_config1_newton_and_oracle_agree():
    p = datagen.config1()
    sv = oracle.SparseSaga(p)
    x = oracle.logistic_newton(p)
    assert np.linalg.norm(sv.gradient(x)) < 1e-14
    fstar = sv.objective(x)
    sv.epochs(50)
    assert abs(sv.objective() - fstar) <= 1e-13 * fstar
    f, flo = sv.certificate()
    assert flo <= fstar + 1e-15 and f >= fstar - 1e-15


def test_config3_closed_form_is_stationary():
    p = datagen.config3(n=20_000)
    sv = oracle.SparseSaga(p)
    x = oracle.ridge_solution_csr(p)
    assert np.linalg.norm(sv.gradient(x)) < 1e-13


def test_certificate_brackets_fstar():
    rng = np.random.default_rng(10)
    p = random_sparse(rng, 200, 30, 0.2, oracle.LOGISTIC, 1e-2)
    fstar = oracle.SparseSaga(p).objective(oracle.logistic_newton(p))
    r = oracle.certified_fstar(p, tol=1e-12, check_every=10)
    assert r["converged"]
    assert r["f_lower"] <= fstar + 1e-15 <= r["f_upper"] + 2e-15


def test_golden_fstar_small_configs(golden):
    p1 = datagen.config1()
    assert golden["config1"]["digest"] == p1.digest()
    sv = oracle.SparseSaga(p1)
    assert sv.objective(oracle.logistic_newton(p1)) == pytest.approx(golden["config1"]["f_star"], rel=1e-14)


def test_step_size_rule():
    p = datagen.config1()
    sv = oracle.SparseSaga(p)
    rows = np.add.reduceat(p.val ** 2, p.rowptr[:-1])
    # config 1's rows are L2-normalised, so the logistic smoothness constant
    # is the value the paper's Section 4.1 table gives for the unit-norm RCV1
    # rows, 0.25, plus the regulariser's lambda
    assert rows.max() == pytest.approx(1.0, rel=1e-12)
    assert sv.L == pytest.approx(0.25 + p.lam, rel=1e-12)
    # 0.25 is the largest curvature of the logistic loss, phi''(0), here
    # measured by central differences of the oracle's own phi'
    h = 1e-5
    curv = [(oracle.dphi(z + h, b, oracle.LOGISTIC) - oracle.dphi(z - h, b, oracle.LOGISTIC)) / (2 * h)
            for z in np.linspace(-3, 3, 61) for b in (-1.0, 1.0)]
    assert max(curv) == pytest.approx(0.25, rel=1e-8)
    # squared loss: curvature 1, so L = max ||a_i||^2 + lambda
    q = datagen.config3(n=3000)
    assert oracle.SparseSaga(q).L == pytest.approx(np.add.reduceat(q.val ** 2, q.rowptr[:-1]).max() + q.lam,
                                                   rel=1e-14)
    assert sv.gamma == pytest.approx(min(1 / (3 * sv.L), 1 / (p.lam * sv.D.max())), rel=1e-15)
    # the cap binds when lambda * max D is large
    q = datagen.config1(n=200, d=50, k=3)
    q.lam = 0.5
    sq = oracle.SparseSaga(q)
    assert sq.gamma == pytest.approx(1 / (0.5 * sq.D.max()), rel=1e-15)


# ---------------------------------------------------------------------------
# sparse SVRG with randomly timed full gradients (Appendix C)
# ---------------------------------------------------------------------------

def dense_dphi(z, b, loss):
    if loss == oracle.SQUARED:
        return z - b
    return -b * np.exp(-np.logaddexp(0.0, b * z))        # -b / (1 + exp(b z)), stably


def test_svrg_full_gradient_rate_is_one_over_n():
    sv_lib = oracle.load()
    n, T = 1000, 400_000
    due = np.array([sv_lib.oracle_svrg_full_gradient_due(7, t, n) for t in range(T)])
    expected = T / n
    assert abs(due.sum() - expected) < 5 * np.sqrt(expected)
    # a stream of its own: not the sample stream's index 0
    idx = oracle.sample_stream(7, 0, T, n)
    assert abs(np.sum(due & (idx == 0)) - T / n ** 2) < 5 * np.sqrt(T / n ** 2) + 1


@pytest.mark.parametrize("loss", [oracle.LOGISTIC, oracle.SQUARED])
def test_svrg_snapshot_is_dense_phi_prime_and_its_average(loss):
    rng = np.random.default_rng(11)
    p = random_sparse(rng, 40, 15, 0.3, loss, 0.05)
    sv = oracle.SparseSvrg(p)
    A = p.dense()
    x = rng.standard_normal(p.d)
    s = oracle.State(x.copy(), np.zeros(p.n), np.zeros(p.d))
    sv.snapshot(s)
    alpha = dense_dphi(A @ x, p.b, loss)
    assert rel_err(s.alpha, alpha) < 1e-13
    assert rel_err(s.abar, A.T @ alpha / p.n) < 1e-13
    assert np.array_equal(s.x, x)


def test_svrg_inner_steps_leave_the_memory_alone():
    rng = np.random.default_rng(12)
    p = random_sparse(rng, 30, 12, 0.3, oracle.LOGISTIC, 0.05)
    sv = oracle.SparseSvrg(p)
    sv.run_indices(rng.integers(0, p.n, size=50))
    s0 = sv.state.copy()
    sv.run_indices(rng.integers(0, p.n, size=50))
    assert np.array_equal(sv.state.alpha, s0.alpha) and np.array_equal(sv.state.abar, s0.abar)
    assert not np.array_equal(sv.state.x, s0.x)


@pytest.mark.parametrize("loss", [oracle.LOGISTIC, oracle.SQUARED])
def test_svrg_expected_step_is_the_gradient(loss):
    # memory from a snapshot at x~, iterate at another x: averaged over all i,
    # the sparse SVRG direction is grad f(x) (Appendix B's unbiasedness, the
    # D_i reweighting of the snapshot's full gradient and of the L2 term)
    rng = np.random.default_rng(13)
    p = random_sparse(rng, 25, 9, 0.35, loss, 0.07)
    sv = oracle.SparseSvrg(p)
    A = p.dense()
    xt = rng.standard_normal(p.d) * 0.5
    snap = oracle.State(xt.copy(), np.zeros(p.n), np.zeros(p.d))
    sv.snapshot(snap)
    x = rng.standard_normal(p.d) * 0.5
    dirs = []
    for i in range(p.n):
        s = oracle.State(x.copy(), snap.alpha.copy(), snap.abar.copy())
        sv.run_indices([i], s)
        dirs.append((x - s.x) / sv.gamma)
    grad = A.T @ dense_dphi(A @ x, p.b, loss) / p.n + p.lam * x
    assert rel_err(np.mean(dirs, axis=0), grad) < 1e-13


def test_svrg_step_at_the_snapshot_is_the_reweighted_full_gradient():
    rng = np.random.default_rng(14)
    p = random_sparse(rng, 20, 8, 0.4, oracle.LOGISTIC, 0.03)
    sv = oracle.SparseSvrg(p)
    A = p.dense()
    x = rng.standard_normal(p.d)
    snap = oracle.State(x.copy(), np.zeros(p.n), np.zeros(p.d))
    sv.snapshot(snap)
    full = A.T @ dense_dphi(A @ x, p.b, oracle.LOGISTIC) / p.n + p.lam * x
    cnt = (A != 0).sum(axis=0)
    D = np.where(cnt > 0, p.n / np.maximum(cnt, 1), 0.0)
    for i in (0, 7, 19):
        s = oracle.State(x.copy(), snap.alpha.copy(), snap.abar.copy())
        sv.run_indices([i], s)
        on = (A[i] != 0).astype(float)
        assert rel_err((x - s.x) / sv.gamma, on * D * full) < 1e-13


def test_svrg_converges_to_the_ridge_closed_form():
    rng = np.random.default_rng(15)
    p = random_sparse(rng, 60, 10, 0.35, oracle.SQUARED, 0.2)
    sv = oracle.SparseSvrg(p, seed=4)
    sv.epochs(400)
    A = p.dense()
    xstar = np.linalg.solve(A.T @ A / p.n + 0.2 * np.eye(p.d), A.T @ p.b / p.n)
    assert rel_err(sv.state.x, xstar) < 1e-10


# ---------------------------------------------------------------------------
# dense and lagged SAGA (Appendix F comparison)
# ---------------------------------------------------------------------------

def test_dense_saga_converges_to_the_ridge_closed_form():
    rng = np.random.default_rng(21)
    p = random_sparse(rng, 60, 10, 0.35, oracle.SQUARED, 0.2)
    sv = oracle.DenseSaga(p, seed=2)
    sv.epochs(600)
    A = p.dense()
    xstar = np.linalg.solve(A.T @ A / p.n + 0.2 * np.eye(p.d), A.T @ p.b / p.n)
    assert rel_err(sv.state.x, xstar) < 1e-10


def test_dense_saga_single_sample_is_gradient_descent():
    a = np.array([0.4, 0.0, -1.2, 0.7])
    one = csr_problem(a[None, :], [-1.0], 0.3, oracle.LOGISTIC)
    sv = oracle.DenseSaga(one, step=0.4)
    x = np.zeros(4)
    sv.epochs(1)        # the first step's memory is zero: x1 = x0 - gamma (phi' a + lambda x0)
    x = x - 0.4 * ((1.0 / (1 + np.exp(-(a @ x)))) * a + 0.3 * x)
    assert rel_err(sv.state.x, x) < 1e-15
    for _ in range(8):  # then the memory equals phi'(a . x_prev): the step is f'(x) exactly
        sv.epochs(1)
        x = x - 0.4 * ((1.0 / (1 + np.exp(-(a @ x)))) * a + 0.3 * x)
    assert rel_err(sv.state.x, x) < 1e-14


@pytest.mark.parametrize("loss", [oracle.LOGISTIC, oracle.SQUARED])
def test_lagged_saga_has_the_dense_iterates(loss):
    # Appendix F: deferring the dense part of each step to the next read of a
    # coordinate changes nothing in the sequential case
    rng = np.random.default_rng(22)
    p = random_sparse(rng, 80, 30, 0.1, loss, 0.01)
    dense = oracle.DenseSaga(p, seed=5)
    lag = oracle.LaggedSaga(p, seed=5)
    for _ in range(4):
        dense.epochs(1)
        lag.epochs(1)
        assert rel_err(lag.state.x, dense.state.x) < 1e-12
        assert rel_err(lag.state.abar, dense.state.abar) < 1e-13
        assert rel_err(lag.state.alpha, dense.state.alpha) < 1e-12


# ---------------------------------------------------------------------------
# T12: simulated asynchrony (Section 3.3: bounded overlap tau, Eq. async)
# ---------------------------------------------------------------------------

def delayed_full_miss_brute_force(p, sv, updates, tau):
    """Every write of the last tau updates missing from each read: read s is
    then the state after max(0, s - tau) updates, taken here from a full
    history of states (tiny inputs only)."""
    x, alpha, abar = np.zeros(p.d), np.zeros(p.n), np.zeros(p.d)
    hist = [(x.copy(), alpha.copy(), abar.copy())]
    for s, i in enumerate(oracle.sample_stream(sv.seed, 0, updates, p.n)):
        xr, ar, abr = hist[max(0, s - tau)]
        lo, hi = p.rowptr[i], p.rowptr[i + 1]
        cols, vals = p.colidx[lo:hi], p.val[lo:hi]
        z = 0.0
        for c, v in zip(cols, vals):
            z += v * xr[c]
        delta = oracle.dphi(z, p.b[i], p.loss) - ar[i]
        for c, v in zip(cols, vals):
            x[c] += -sv.gamma * (delta * v + sv.D[c] * (abr[c] + p.lam * xr[c]))
            abar[c] += delta * v / p.n
        alpha[i] += delta
        hist.append((x.copy(), alpha.copy(), abar.copy()))
    return x, alpha, abar


@pytest.mark.parametrize("tau", [0, 7, 40])
def test_delayed_reads_without_misses_are_sparse_saga(tau):
    p = datagen.config1(n=400, d=120, k=12)
    a = oracle.SparseSaga(p, seed=4)
    a.epochs(3)
    b = oracle.DelayedSparseSaga(p, tau=tau, miss=0.0, seed=4)
    b.run(3 * p.n)
    for u, v in ((a.state.x, b.state.x), (a.state.alpha, b.state.alpha), (a.state.abar, b.state.abar)):
        assert np.array_equal(u, v)


@pytest.mark.parametrize("loss", [oracle.LOGISTIC, oracle.SQUARED])
def test_delayed_reads_with_every_write_missing_read_the_state_tau_back(loss):
    rng = np.random.default_rng(31)
    p = random_sparse(rng, 20, 9, 0.4, loss, 0.05)
    for tau in (1, 3, 11):
        sv = oracle.DelayedSparseSaga(p, tau=tau, miss=1.0, seed=2)
        sv.run(240)
        x, alpha, abar = delayed_full_miss_brute_force(p, sv, 240, tau)
        assert rel_err(sv.state.x, x) < 1e-12
        assert rel_err(sv.state.alpha, alpha) < 1e-12
        assert rel_err(sv.state.abar, abar) < 1e-12


def test_delayed_reads_keep_the_running_average_exact():
    # the writes are additions of the same delta to alpha_i and (1/n) a_i to
    # abar, whatever the reads missed
    rng = np.random.default_rng(32)
    p = random_sparse(rng, 300, 60, 0.1, oracle.LOGISTIC, 1e-3)
    sv = oracle.DelayedSparseSaga(p, tau=25, miss=0.5, seed=6)
    sv.run(5 * p.n)
    assert rel_err(sv.state.abar, scipy_csr(p).T @ sv.state.alpha / p.n) < 1e-12


def test_delayed_reads_are_deterministic_and_follow_their_own_stream():
    p = datagen.config1(n=400, d=120, k=12)
    runs = []
    for ds in (11, 11, 12):
        sv = oracle.DelayedSparseSaga(p, tau=20, miss=0.5, delay_seed=ds)
        sv.run(2 * p.n)
        runs.append(sv.state.x.copy())
    assert np.array_equal(runs[0], runs[1])
    assert not np.array_equal(runs[0], runs[2])


def test_delayed_reads_small_overlap_converges_large_overlap_needs_a_smaller_step(golden):
    # Theorem 2: a linear rate for steps below a bound that shrinks with tau
    p = datagen.config1()
    fstar = golden["config1"]["f_lower"]

    def rel_after(tau, miss, scale, epochs=30):
        sv = oracle.DelayedSparseSaga(p, tau=tau, miss=miss)
        sv.gamma *= scale
        sv.run(epochs * p.n)
        return (sv.objective() - fstar) / fstar

    assert rel_after(16, 0.5, 1.0) <= 1e-9
    assert rel_after(64, 1.0, 1.0) <= 1e-9
    half = p.n // 2
    assert rel_after(half, 1.0, 1.0) > 1e-2           # the serial step fails at tau = n/2
    assert rel_after(half, 1.0, 1.0 / 8) < 1e-3       # an eighth of it converges


def test_delayed_reads_iterations_do_not_grow_with_small_overlap(golden):
    # Theorem 2 (and the iteration speedup of Appendix D): below the step
    # bound, the iterations to a given accuracy do not depend on the overlap;
    # the bound itself shrinks with tau, so at the serial step a large
    # overlap costs iterations
    p = datagen.config1()
    fstar = golden["config1"]["f_lower"]

    def epochs_to_1e9(tau, scale):
        sv = oracle.DelayedSparseSaga(p, tau=tau, miss=1.0)
        sv.gamma *= scale
        for ep in range(1, 120):
            sv.run(p.n)
            if (sv.objective() - fstar) / fstar <= 1e-9:
                return ep
        return None

    base = epochs_to_1e9(0, 0.25)
    for tau in (16, 64):
        assert abs(epochs_to_1e9(tau, 0.25) - base) <= 1
    assert epochs_to_1e9(256, 1.0) >= 1.3 * epochs_to_1e9(0, 1.0)
