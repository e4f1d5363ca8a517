"""The benchmark's batched stop policy (bench.solve_with_stop_test) on the
host, against a stand-in batch whose instances follow known trajectories.

The stand-in applies the device's rule exactly: after each epoch an instance
still running reports its proxy r_k and is switched off when r_k is at or
below its threshold.  Each instance's relative suboptimality falls
geometrically, and rel/proxy drifts upward over the run, as measured on the
160-instance lambda path (so thresholds calibrated early stop instances too
soon, and the policy has to check and switch them on again).  One instance's
proxy stops falling at a floor (as FP32 state rounding leaves) while its
objective still falls, so only the periodic re-check can end it.
"""
import types

import numpy as np

import bench

TARGET = 1e-9


class StandInBatch:
    def __init__(self, rel0, rate, ratio0, drift, floor=None, m=1000):
        self.n_inst = len(rel0)
        self.rel0, self.rate = np.asarray(rel0, float), np.asarray(rate, float)
        self.ratio0, self.drift = np.asarray(ratio0, float), np.asarray(drift, float)
        self.floor = np.zeros(self.n_inst) if floor is None else np.asarray(floor, float)
        self.m = m
        self.e = np.zeros(self.n_inst, dtype=np.int64)
        self.active = np.ones(self.n_inst, dtype=bool)
        self.thr = None
        self.proxy = np.full(self.n_inst, np.nan)
        self.ran = np.zeros(self.n_inst, dtype=np.int64)
        self.thresholds_seen = []

    def rel(self, k):
        return self.rel0[k] * self.rate[k] ** self.e[k]

    def proxy_of(self, k):
        return max(self.floor[k], self.rel(k) / (self.ratio0[k] * (1.0 + self.drift[k] * self.e[k])))

    def set_stop(self, thr):
        self.thr = None if thr is None else np.array(thr, dtype=float)
        if thr is not None:
            self.thresholds_seen.append(self.thr.copy())

    def set_active(self, a):
        self.active = np.asarray(a).astype(bool)

    def epochs(self, n):
        assert n == 1
        self.proxy[:] = np.nan
        self.ran[:] = 0
        for k in np.nonzero(self.active)[0]:
            self.e[k] += 1
            self.ran[k] = 1
            self.proxy[k] = self.proxy_of(k)
            if self.thr is not None and self.proxy[k] <= self.thr[k]:
                self.active[k] = False

    def stop_report(self):
        return self.proxy.copy(), self.ran.copy()

    def instance(self, k):
        return types.SimpleNamespace(t=int(self.e[k]) * self.m, active=int(self.active[k]))


def crossing(g, k):
    """First epoch at which instance k's suboptimality is within the target."""
    return int(np.ceil(np.log(TARGET / g.rel0[k]) / np.log(g.rate[k])))


def run(g, **kw):
    return bench.solve_with_stop_test(g, g.rel, None, target=TARGET, **kw)


def test_every_instance_ends_within_the_target_soon_after_its_crossing():
    rng = np.random.default_rng(0)
    ni = 40
    g = StandInBatch(rel0=10 ** rng.uniform(-2, 0, ni), rate=rng.uniform(0.3, 0.9, ni),
                     ratio0=10 ** rng.uniform(2, 7, ni), drift=rng.uniform(0.0, 0.2, ni))
    res = run(g)
    assert np.all(res["rel"] <= TARGET)
    for k in range(ni):
        c = crossing(g, k)
        assert c <= g.e[k] <= c + 8, (k, c, g.e[k])
        assert res["applied"][k] == g.e[k] * g.m
    # fewer exact checks than one per instance and launch, and the drifting
    # ratio made some thresholds stop instances early, which ran on
    assert res["checks"] < res["instance_launches"]
    assert res["instance_launches"] == int(g.e.sum())
    assert res["early_stops"] > 0
    # the test is disarmed at the end
    assert g.thr is None


def test_first_launch_checks_every_instance_and_calibrates_its_threshold():
    g = StandInBatch(rel0=[0.5, 0.1, 0.02], rate=[0.8, 0.7, 0.6], ratio0=[1e3, 1e5, 1e6], drift=[0, 0, 0])
    bench.solve_with_stop_test(g, g.rel, None, target=TARGET, max_launches=1, eager=2.0)
    # thresholds armed before the first launch: none; after it: eager * target * proxy / rel
    assert np.all(g.thresholds_seen[0] == 0.0)
    want = [2.0 * TARGET / g.ratio0[k] for k in range(3)]   # proxy / rel = 1 / ratio without drift
    np.testing.assert_allclose(g.thresholds_seen[1], want, rtol=1e-12)


def test_without_drift_the_calibrated_test_stops_each_instance_at_its_crossing():
    """rel/proxy constant: after one calibration the device stops every
    instance exactly where it crosses eager * target, and the only exact
    checks are the first one and the confirming one (eager = 1: at the
    crossing itself)."""
    g = StandInBatch(rel0=[0.5, 0.3, 0.9, 0.05], rate=[0.7, 0.5, 0.8, 0.6], ratio0=[1e4, 1e6, 3e2, 1e5],
                     drift=[0, 0, 0, 0])
    res = run(g, eager=1.0, max_gap=10 ** 6)
    for k in range(4):
        assert g.e[k] == crossing(g, k)
    assert res["checks"] == 2 * 4
    assert res["early_stops"] == 0


def test_a_proxy_stuck_at_a_floor_is_ended_by_the_periodic_check():
    g = StandInBatch(rel0=[0.5, 0.5], rate=[0.7, 0.7], ratio0=[1e4, 1e4], drift=[0, 0], floor=[0.0, 1e-9])
    res = run(g, max_gap=8)
    c = crossing(g, 1)
    assert np.all(res["rel"] <= TARGET)
    assert c <= g.e[1] <= c + 8
    # the instance whose proxy keeps falling ends at its crossing, or one
    # epoch after a stop the eager threshold made just before it
    assert crossing(g, 0) <= g.e[0] <= crossing(g, 0) + 1
