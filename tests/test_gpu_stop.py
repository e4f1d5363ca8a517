"""The in-graph stop test of a batch (asaga_set_stop, asaga_stop_report).

After every epoch of a batched call a kernel computes, for each instance
still running, r_k = ||abar_k + lambda_k x_k||^2: the full gradient of the
instance's objective (Section 4.1) with each row's scalar derivative taken
from the memory of Section 2 (the running average of Eq. SparseSAGA), at
O(d) instead of a pass over the rows.  An instance whose r_k falls to its
threshold applies no more samples in that call.

In ordered mode (each instance on one workgroup, samples in stream order)
the batch is deterministic, so a run with the test and one without must
agree bit for bit on every instance at the epoch where the test stopped it;
the proxy itself is checked against the state the library returns, and the
captured graph against plain launches.
"""
import sys

import numpy as np
import pytest

import datagen

pytestmark = pytest.mark.gpu

A = pytest.importorskip("paper_1606_04809_amd")

HOT = dict(threads_per_block=256, hot_columns=512, hot_tier_columns=64, hot_tier_every=3, flush_every=2,
           hot_reload_from=200)


def say(*a):
    print(*a, flush=True, file=sys.stderr)


def small_batch():
    p = datagen.config2(n=8000, d=3000)
    row_fold = datagen.folds5(p.n, seed=0)
    inst_fold = np.array([0, 3, -1, 2], dtype=np.int32)
    inst_lam = np.array([1e-4, 1e-3, 1e-5, 3e-4])
    return p, (row_fold, inst_fold, inst_lam)


def ordered(p, batch, **kw):
    return A.from_problem(p, mode=A.ASAGA_MODE_SERIAL, seed=7, lanes_per_sample=16, batch=batch, **HOT, **kw)


def proxy_from_state(g, k, lam):
    x, alpha, abar, t = g.get_state(k)
    v = abar + lam * x
    return float(np.dot(v, v)), t


@pytest.mark.parametrize("precision", ["f64", "mixed", "f32"])
def test_proxy_is_the_memory_gradient_norm(precision):
    """r_k equals ||abar + lambda x||^2 of the state the library returns
    (summation order aside), for each state layout; the test never fires at
    threshold 0, and every instance runs the whole call."""
    prec = {"f64": A.ASAGA_PREC_F64, "mixed": A.ASAGA_PREC_MIXED, "f32": A.ASAGA_PREC_F32}[precision]
    p, batch = small_batch()
    lam = batch[2]
    with ordered(p, batch, precision=prec) as g:
        proxy, ep = g.stop_report()
        assert np.all(np.isnan(proxy)) and np.all(ep == 0)
        g.set_stop(np.zeros(4))
        g.epochs(2)
        proxy, ep = g.stop_report()
        assert list(ep) == [2, 2, 2, 2]
        for k in range(4):
            want, t = proxy_from_state(g, k, lam[k])
            assert t == 2 * g.instance(k).m
            assert g.instance(k).active == 1
            assert proxy[k] == pytest.approx(want, rel=1e-12), (k, proxy[k], want)
        say(f"{precision}: proxies {['%.3e' % r for r in proxy]}")


def test_stopped_instances_match_a_run_without_the_test():
    """Thresholds of +infinity stop instances 0 and 2 after their first
    epoch; 1 and 3 (threshold 0) run all three.  Each instance's state and
    sample counter equal, bit for bit, those of a run without the test after
    as many epochs; the stopped ones are switched off after the call."""
    p, batch = small_batch()
    with ordered(p, batch) as ref:
        ref.epochs(1)
        one = [ref.get_state(k) for k in range(4)]
        ref.epochs(2)
        three = [ref.get_state(k) for k in range(4)]
    with ordered(p, batch) as g:
        g.set_stop(np.array([np.inf, 0.0, np.inf, 0.0]))
        g.epochs(3)
        proxy, ep = g.stop_report()
        assert list(ep) == [1, 3, 1, 3]
        assert [g.instance(k).active for k in range(4)] == [0, 1, 0, 1]
        for k in range(4):
            want = one[k] if k in (0, 2) else three[k]
            got = g.get_state(k)
            assert got[3] == want[3]
            for a, b in zip(got[:3], want[:3]):
                assert np.array_equal(a, b), k
        # switched on again and disarmed, instance 0 continues where it stopped
        g.set_stop(None)
        g.set_active(np.ones(4, np.uint8))
        g.epochs(2)
        assert g.get_state(0)[3] == three[0][3]
        assert np.array_equal(g.get_state(0)[0], three[0][0])


@pytest.mark.parametrize("plain_launch", [0, 1])
def test_threshold_stops_at_the_first_epoch_at_or_below_it(plain_launch):
    """A run with the test at threshold 0 records each instance's proxy
    after epochs 1..5; with the threshold set to its value after epoch 3,
    each instance stops after the first epoch whose proxy is at or below it
    (epoch 3 where the proxy falls), with that proxy, through the captured
    graph and through plain launches, in a call of six epochs."""
    p, batch = small_batch()
    r = []
    with ordered(p, batch) as ref:
        ref.set_stop(np.zeros(4))
        for e in range(5):
            ref.epochs(1)
            r.append(ref.stop_report()[0])
    r = np.array(r)                       # [epoch - 1, instance]
    thr = r[2].copy()
    expect = [int(np.nonzero(r[:, k] <= thr[k])[0][0]) + 1 for k in range(4)]
    assert min(expect) >= 2
    with ordered(p, batch, plain_launch=plain_launch) as g:
        g.set_stop(thr)
        g.epochs(6)
        proxy, ep = g.stop_report()
        assert list(ep) == expect
        assert np.array_equal(proxy, [r[expect[k] - 1, k] for k in range(4)])
        assert all(g.instance(k).active == 0 for k in range(4))
    say(f"stop epochs {expect}")


def test_set_stop_rejects_bad_thresholds_and_single_contexts():
    p, batch = small_batch()
    with ordered(p, batch) as g:
        with pytest.raises(A.AsagaError):
            g.set_stop(np.array([0.0, -1.0, 0.0, 0.0]))
        with pytest.raises(A.AsagaError):
            g.set_stop(np.array([0.0, np.nan, 0.0, 0.0]))
    with A.from_problem(p, mode=A.ASAGA_MODE_ASYNC) as g:
        with pytest.raises(A.AsagaError):
            A.asaga_set_stop(g.ctx, np.zeros(1))
        with pytest.raises(A.AsagaError):
            A.asaga_stop_report(g.ctx, 1)


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_async_batch_reaches_1e9_with_the_stop_test_choosing_the_checks(precision):
    """Asynchronous batch of six instances (three lambdas, two held-out
    folds), FP64 or FP32 state: the benchmark's policy (one epoch per call,
    exact FP64 checks only where the stop test switched an instance off,
    where it was never checked, or after eight epochs without a check)
    brings every instance within 1e-9 of the oracle's optimum for its own
    rows and lambda, with fewer exact checks than one per instance and
    launch; each instance's abar is the running average of its memory (FP32
    state: to the rounding its atomic additions leave)."""
    import torch

    import bench
    import oracle
    from conftest import rel_err

    p = datagen.config2(n=12_000, d=3000)
    row_fold = datagen.folds5(p.n, seed=0)
    lams = np.array([1e-5, 1e-4, 1e-3])
    inst_fold = np.repeat(np.array([0, 3], dtype=np.int32), 3)
    inst_lam = np.tile(lams, 2)
    subs = [datagen.subproblem(p, np.nonzero(row_fold != f)[0], lam=float(lam)) for f, lam in zip(inst_fold, inst_lam)]
    fstar = np.array([oracle.certified_fstar(s, tol=1e-12, check_every=10)["f_lower"] for s in subs])
    prec = A.ASAGA_PREC_F64 if precision == "f64" else A.ASAGA_PREC_F32
    with A.from_problem(p, mode=A.ASAGA_MODE_ASYNC, precision=prec, batch=(row_fold, inst_fold, inst_lam)) as g:
        res = bench.solve_with_stop_test(g, lambda k: (g.objective(k) - fstar[k]) / fstar[k],
                                         torch.cuda.current_stream())
        say(f"{precision}: {res['launches']} launches, {res['checks']} exact checks "
            f"({res['instance_launches']} instance launches), {res['early_stops']} early stops, "
            f"rel {['%.1e' % r for r in res['rel']]}")
        assert np.all(res["rel"] <= 1e-9)
        assert res["checks"] < res["instance_launches"]
        for k, s in enumerate(subs):
            x, alpha, abar, t = g.get_state(k)
            assert t == res["applied"][k]
            assert g.instance(k).active == 0
            err = rel_err(abar, oracle.SparseSaga(s).memory_average(alpha))
            say(f"instance {k}: abar against its memory {err:.1e}")
            assert err < (1e-11 if precision == "f64" else 1e-4)
