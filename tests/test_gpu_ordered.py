"""Ordered-mode parity of the production update paths.

ASAGA_MODE_SERIAL runs the asynchronous kernel's code with one active lane
group applying the samples in stream order, so that every path the
asynchronous launch takes can be compared with the sequential oracle
iterate for iterate (x, alpha and abar after every epoch, 1e-12 relative):
the LDS hot set (pending sums combined per workgroup, the first tier
flushed every round and the rest every few rounds, views refreshed from the
returning atomics and reloaded from the shared state), lane groups of 8, 16,
32 and 64 lanes, rows longer than the 2G entries held in registers (the
chunked path), FP64, FP32 and bfloat16 values, and the batched kernel.  A
lost or doubled increment anywhere in the combining breaks the update rule
of Eq. SparseSAGA (Algorithm 2; Property 3 of Section 3.3: every write is
applied) and shows here, where convergence to f* alone would hide it.

The oracle consumes the same values the library does: FP32 and bfloat16
values exactly widened to FP64.
"""
import sys

import numpy as np
import pytest

import datagen
import oracle
from conftest import rel_err

pytestmark = pytest.mark.gpu

A = pytest.importorskip("paper_1606_04809_amd")


def say(*a):
    print(*a, flush=True, file=sys.stderr)


def long_rows_problem(seed=0, n=400, d=900, loss=datagen.LOGISTIC):
    """Rows of 1 .. 400 entries over Zipf-like columns: the most-used columns
    (the hot set after relabelling) sit in the long rows too."""
    rng = np.random.default_rng(seed)
    k = np.concatenate([[1, 2, 17, 33, 65, 129, 257, 400], rng.integers(1, 150, size=n - 8)])
    w = 1.0 / np.arange(1, d + 1) ** 1.1
    w /= w.sum()
    cols = [np.sort(rng.choice(d, size=int(kk), replace=False, p=w)) for kk in k]
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(k, out=rowptr[1:])
    colidx = np.concatenate(cols).astype(np.int32)
    val = rng.lognormal(0.0, 1.0, size=len(colidx))
    val /= np.repeat(np.sqrt(np.add.reduceat(val * val, rowptr[:-1])), k)
    b = np.where(rng.random(n) < 0.5, 1.0, -1.0) if loss == datagen.LOGISTIC else rng.standard_normal(n)
    return datagen.Problem("long_rows", n, d, rowptr, colidx, val, b, loss, 1.0 / n)


def with_values(p, kind):
    """(problem for the oracle, values and val_dtype for the library)."""
    if kind == "f64":
        return p, p.val, A.ASAGA_VAL_F64
    if kind == "f32":
        v32 = p.val.astype(np.float32)
        q = datagen.Problem(p.name + "_f32", p.n, p.d, p.rowptr, p.colidx, v32.astype(np.float64), p.b, p.loss, p.lam)
        return q, v32, A.ASAGA_VAL_F32
    bits = datagen.bf16_round(p.val)
    q = datagen.Problem(p.name + "_bf16", p.n, p.d, p.rowptr, p.colidx, datagen.bf16_widen(bits), p.b, p.loss, p.lam)
    return q, bits, A.ASAGA_VAL_BF16


def compare_ordered(p, epochs, vals=None, val_dtype=None, seed=0, tol=1e-12, **shape):
    """Run the ordered launch with the given shape and compare every epoch."""
    sv = oracle.SparseSaga(p, seed=seed)
    v = p.val if vals is None else vals
    with A.Solver(p.n, p.d, p.rowptr, p.colidx, v, p.b, p.lam, loss=p.loss, val_dtype=val_dtype,
                  mode=A.ASAGA_MODE_SERIAL, seed=seed, **shape) as g:
        info = g.info()
        assert info.gamma == pytest.approx(sv.gamma, rel=1e-14)
        worst = 0.0
        for e in range(epochs):
            g.epochs(1)
            sv.epochs(1)
            x, alpha, abar, t = g.get_state()
            assert t == sv.state.t
            errs = (rel_err(x, sv.state.x), rel_err(alpha, sv.state.alpha), rel_err(abar, sv.state.abar))
            worst = max(worst, *errs)
            assert max(errs) <= tol, (shape, e, errs)
        return info, worst


# the hot-set paths of the asynchronous launch, all switched on: rounds of
# two samples per lane group, the first 64 hot columns flushed every round,
# the other 448 every third round, and the views of columns 200 .. 511
# reloaded at every full flush; four wavefronts share the flushes
HOT = dict(threads_per_block=256, hot_columns=512, hot_tier_columns=64, hot_tier_every=3, flush_every=2,
           hot_reload_from=200)


@pytest.mark.parametrize("lanes", [8, 16, 32, 64])
def test_ordered_hot_set_every_lane_width(lanes):
    """RCV1-shaped rows (~75 entries over Zipf(1.1) columns): with 8 and 16
    lanes every row takes the chunked path (more than 2G entries), with 32
    lanes some rows do."""
    p = datagen.config2(n=6000, d=3000)
    info, worst = compare_ordered(p, 3, lanes_per_sample=lanes, **HOT)
    assert (info.lanes_per_sample, info.threads_per_block, info.hot_columns) == (lanes, 256, 512)
    assert (info.hot_tier_columns, info.hot_tier_every, info.flush_every, info.hot_reload_from) == (64, 3, 2, 200)
    say(f"ordered, {lanes} lanes, hot set 512 (tier 64 every round, rest every 3rd, reload from 200): "
        f"worst rel err {worst:.1e}")


@pytest.mark.parametrize("lanes", [8, 64])
@pytest.mark.parametrize("loss", [datagen.LOGISTIC, datagen.SQUARED])
def test_ordered_long_rows_with_hot_columns(lanes, loss):
    """Rows of 1 .. 400 entries whose most-used columns are in the hot set:
    chunked reads and writes mixing LDS and global columns."""
    p = long_rows_problem(loss=loss)
    cnt = np.bincount(p.colidx, minlength=p.d)
    hot_cols = np.argsort(-cnt, kind="stable")[:128]
    long = np.nonzero(np.diff(p.rowptr) > 2 * lanes)[0]
    assert len(long) > 0
    touched = sum(np.isin(p.colidx[p.rowptr[i]:p.rowptr[i + 1]], hot_cols).any() for i in long)
    assert touched == len(long)
    shape = dict(HOT, hot_columns=128, hot_tier_columns=16, hot_reload_from=40)
    info, worst = compare_ordered(p, 5, lanes_per_sample=lanes, **shape)
    say(f"ordered long rows, {lanes} lanes, loss {loss}: {len(long)} rows beyond {2 * lanes} entries, "
        f"worst rel err {worst:.1e}")


@pytest.mark.parametrize("kind", ["f64", "f32", "bf16"])
def test_ordered_value_types(kind):
    """CSR values in FP64, FP32 and bfloat16: the oracle runs on the exactly
    widened values, which are the instance."""
    q, vals, vdt = with_values(datagen.config2(n=5000, d=2500), kind)
    info, worst = compare_ordered(q, 3, vals=vals, val_dtype=vdt, lanes_per_sample=16, **HOT)
    say(f"ordered, {kind} values: worst rel err {worst:.1e}")


def test_ordered_default_shape_is_unchanged():
    """Without shape options the ordered launch is one 64-lane group on a
    64-thread workgroup with no hot set, as before."""
    p = datagen.config1(n=400, d=120, k=12)
    info, _ = compare_ordered(p, 4)
    assert (info.lanes_per_sample, info.threads_per_block, info.hot_columns) == (64, 64, 0)


def test_ordered_batched_each_instance_matches_its_oracle():
    """A batch in ordered mode: every instance (its own lambda, held-out fold,
    D from its training rows and sample stream seed + k) runs sequentially
    on one workgroup of the batched kernel, with the hot set on, all
    instances in the same launch; each must match the oracle run on its own
    subproblem after every epoch, through the captured-graph path."""
    p = datagen.config2(n=8000, d=3000)
    row_fold = datagen.folds5(p.n, seed=0)
    inst_fold = np.array([0, 3, -1, 2], dtype=np.int32)
    inst_lam = np.array([1e-4, 1e-3, 1e-5, 3e-4])
    subs = []
    for k, (f, lam) in enumerate(zip(inst_fold, inst_lam)):
        rows = np.arange(p.n) if f < 0 else np.nonzero(row_fold != f)[0]
        subs.append(oracle.SparseSaga(datagen.subproblem(p, rows, lam=float(lam)), seed=7 + k))
    with A.from_problem(p, mode=A.ASAGA_MODE_SERIAL, seed=7, lanes_per_sample=16, batch=(row_fold, inst_fold, inst_lam),
                        **HOT) as g:
        for k, sv in enumerate(subs):
            ins = g.instance(k)
            assert ins.m == sv.n and ins.fold == inst_fold[k]
            assert ins.gamma == pytest.approx(sv.gamma, rel=1e-14)
        worst = 0.0
        for e in range(3):
            g.epochs(1)
            for k, sv in enumerate(subs):
                sv.epochs(1)
                x, alpha, abar, t = g.get_state(k)
                assert t == sv.state.t
                errs = (rel_err(x, sv.state.x), rel_err(alpha, sv.state.alpha), rel_err(abar, sv.state.abar))
                worst = max(worst, *errs)
                assert max(errs) <= 1e-12, (e, k, errs)
        # an instance switched off keeps its state
        g.set_active(np.array([1, 0, 1, 1], np.uint8))
        before = g.get_state(1)
        g.epochs(1)
        after = g.get_state(1)
        assert after[3] == before[3] and np.array_equal(after[0], before[0])
    say(f"ordered batched: 4 instances x 3 epochs, worst rel err {worst:.1e}")


def test_ordered_mixed_precision_memory_average_is_exact():
    """FP32 x and alpha (FP64 abar): with no other sample between a read of
    alpha_i and its addition, abar receives exactly the change the FP32
    memory entry took, so abar = (1/n) A^T alpha holds to FP64 rounding,
    with and without the hot set.  The iterates differ from the FP64
    oracle's by FP32 rounding only."""
    p = datagen.config2(n=5000, d=2500)
    sv = oracle.SparseSaga(p)
    sv.epochs(4)
    for shape in (dict(), dict(HOT, lanes_per_sample=16)):
        with A.from_problem(p, mode=A.ASAGA_MODE_SERIAL, precision=A.ASAGA_PREC_MIXED, **shape) as g:
            g.epochs(4)
            x, alpha, abar, t = g.get_state()
        inv = rel_err(abar, oracle.SparseSaga(p).memory_average(alpha))
        dx = rel_err(x, sv.state.x)
        say(f"ordered mixed {shape.get('hot_columns', 0)} hot: invariant {inv:.1e}, x vs FP64 oracle {dx:.1e}")
        assert inv <= 1e-12
        assert dx <= 1e-4


@pytest.mark.parametrize("lanes", [16, 64])
def test_ordered_f32_state_follows_the_oracle_to_fp32_rounding(lanes):
    """FP32 x, alpha and abar (8-byte slots), through every hot-set path
    (tiered flush, refresh, reload, FP32 pending sums with the flush's
    rounding error carried to the next flush): the iterates and the memory
    follow the FP64 oracle's to FP32 rounding, and abar stays the average of
    the stored memory to FP32 rounding, with and without the hot set; the
    hot-set run and the run without it agree to FP32 rounding too."""
    p = datagen.config2(n=5000, d=2500)
    sv = oracle.SparseSaga(p)
    sv.epochs(4)
    runs = {}
    for shape in (dict(lanes_per_sample=lanes), dict(HOT, lanes_per_sample=lanes)):
        with A.from_problem(p, mode=A.ASAGA_MODE_SERIAL, precision=A.ASAGA_PREC_F32, **shape) as g:
            g.epochs(4)
            x, alpha, abar, t = g.get_state()
        assert t == sv.state.t
        inv = rel_err(abar, oracle.SparseSaga(p).memory_average(alpha))
        dx, da = rel_err(x, sv.state.x), rel_err(alpha, sv.state.alpha)
        hot = shape.get("hot_columns", 0)
        say(f"ordered f32, {lanes} lanes, {hot} hot: invariant {inv:.1e}, x vs FP64 oracle {dx:.1e}, "
            f"alpha {da:.1e}")
        assert inv <= 1e-5
        assert dx <= 1e-4 and da <= 1e-4
        runs[hot] = x
    assert rel_err(runs[512], runs[0]) <= 1e-4


def test_ordered_batched_f32_state_follows_each_instance_oracle():
    """The batched kernel in the FP32 layout, ordered: every instance's
    iterate and memory follow its FP64 oracle to FP32 rounding, and its
    running average holds to FP32 rounding."""
    p = datagen.config2(n=6000, d=2500)
    row_fold = datagen.folds5(p.n, seed=0)
    inst_fold = np.array([1, -1, 4], dtype=np.int32)
    inst_lam = np.array([3e-4, 1e-5, 1e-3])
    with A.from_problem(p, mode=A.ASAGA_MODE_SERIAL, seed=3, precision=A.ASAGA_PREC_F32, lanes_per_sample=16,
                        batch=(row_fold, inst_fold, inst_lam), **HOT) as g:
        g.epochs(3)
        for k, (f, lam) in enumerate(zip(inst_fold, inst_lam)):
            rows = np.arange(p.n) if f < 0 else np.nonzero(row_fold != f)[0]
            q = datagen.subproblem(p, rows, lam=float(lam))
            sv = oracle.SparseSaga(q, seed=3 + k)
            sv.epochs(3)
            x, alpha, abar, t = g.get_state(k)
            assert t == sv.state.t
            dx, da = rel_err(x, sv.state.x), rel_err(alpha, sv.state.alpha)
            inv = rel_err(abar, sv.memory_average(alpha))
            say(f"ordered batched f32, instance {k}: x {dx:.1e}, alpha {da:.1e}, invariant {inv:.1e}")
            assert dx <= 1e-4 and da <= 1e-4 and inv <= 1e-5
