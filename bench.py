"""Benchmark of the asynchronous Sparse SAGA (ASAGA) hot path on one MI355X.

Workload: the RCV1-shaped L2-logistic instance (700,000 x 47,000, ~75
distinct Zipf(1.1) columns per row, TF-IDF-like values (lognormal term
weight x smooth idf), rows L2-normalised, lambda = 1/n), plain FP64
asynchronous ASAGA.  One step = one epoch = n
sample updates of the whole hot path (sample, row fetch, gather and dot,
scalar gradient, scatter of x and abar, memory update).

Prints one JSON line: updates/s, algorithmic HBM GB/s against the 8 TB/s
roofline (per-launch time measured with HIP events on the library's
stream) next to the measured memory-side request ceiling, the time to 1e-9
relative suboptimality from a cold start, the overlap sweep (iterations to
1e-9 against samples in flight at a fixed small step), atomic against racy
updates (Appendix G), the batched leg (160 lambda x fold instances over the
same matrix in bfloat16: FP32 state, mixed precision and FP64 state, to
1e-9 each, against the same instances solved one by one with the plain FP64
kernel), the other workloads (the tiny serial instance, the Covtype-shaped
least squares in FP64 and FP32 then FP64, the URL-shaped instance in FP32
state), and the CPU oracle timed on bounded samples of each workload on this
host's cores, with its own time to 1e-9.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--skip-cpu] [--skip-tta]
                    [--skip-batched] [--no-batched-f64-state] [--plain-instances N]
                    [--library-defaults] [--no-tau-sweep] [--skip-racy] [--skip-configs]
                    [--copy-calibration]

--copy-calibration adds a plain 1 GiB device-to-device copy (known bytes
read and written) so that a profiler's per-dispatch byte counters can be
scaled to bytes in the same run.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "SAGA updates/s + HBM GB/s; time to 1e-9 rel. subopt., plain vs batched"
HBM_PEAK_GBPS = 8000.0
PROFILE_SUMMARY = os.path.join(ROOT, "profiles", "k_update_config2_pmc.txt")
REQUEST_SUMMARY = os.path.join(ROOT, "profiles", "k_update_config2_requests.txt")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def load_golden():
    with open(os.path.join(ROOT, "tests", "golden", "fstar.json")) as fh:
        return json.load(fh)


def host_cpu_model():
    """The host CPU as /proc/cpuinfo (what lscpu reads) names it: model name,
    then family, model and stepping numbers (a virtualised host may shorten
    the name; the numbers still identify the generation), or None."""
    fields = {}
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if not line.strip():
                    break                       # the first processor's block only
                if ":" in line:
                    k, v = line.split(":", 1)
                    fields.setdefault(k.strip(), v.strip())
    except OSError:
        return None
    name = fields.get("model name")
    if name is None:
        return None
    nums = [f"{k} {fields[k]}" for k in ("cpu family", "model", "stepping") if k in fields]
    return f"{name} ({', '.join(nums)})" if nums else name


def kernel_source_digest() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in ("kernels.hip", "asaga.hip", "internal.hpp"):
        with open(os.path.join(ROOT, "paper_1606_04809_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _profile_values(path: str, per_launch_updates: int):
    """The key: value lines of a committed rocprofv3 summary, or None if it is
    missing or was taken on other kernel sources or another workload."""
    try:
        kv = {}
        with open(path) as fh:
            for line in fh:
                if ":" in line and not line.startswith("#"):
                    k, v = line.split(":", 1)
                    kv[k.strip()] = v.strip()
        if kv.get("kernel_source_digest") != kernel_source_digest():
            return None
        if int(kv["updates_per_launch"]) != per_launch_updates:
            return None
        return kv
    except (OSError, KeyError, ValueError):
        return None


def traffic_from_profile(per_launch_updates: int, shape):
    """HBM bytes per launch from the committed rocprofv3 --pmc summary (taken
    at the benchmarked launch shape), or None."""
    kv = _profile_values(PROFILE_SUMMARY, per_launch_updates)
    if kv is None or shape != "benchmarked":
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def requests_from_profile(per_launch_updates: int, shape):
    """Memory-side atomic and read requests per update at the given launch
    shape ("benchmarked" or "library") from the committed counter summary,
    or None."""
    kv = _profile_values(REQUEST_SUMMARY, per_launch_updates)
    if kv is None or shape is None:
        return None
    try:
        return {"atomic_per_update": float(kv[f"{shape}_atomic_requests_per_update"]),
                "read_per_update": float(kv[f"{shape}_read_requests_per_update"])}
    except (KeyError, ValueError):
        return None


def tau_sweep(p, dev_arrays, fstar, stream):
    """Iterations to 1e-9 versus updates in flight, the device-side version
    of the paper's speedup study: one fixed step (1/16 of the serial rule,
    stable at every point here), wavefronts in flight from 64 to 2048; the
    overlap tau of each point is measured by the sampled clock log of
    asaga_overlap over its first two epochs."""
    import numpy as np
    import torch

    import paper_1606_04809_amd as A

    rule = 1.0 / (3.0 * (0.25 * float(np.max(np.add.reduceat(p.val ** 2, p.rowptr[:-1]))) + p.lam))
    out = []
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for waves in (64, 128, 256, 512, 1024, 2048):
        g = A.Solver(p.n, p.d, *dev_arrays, p.lam, loss=p.loss, mode=A.ASAGA_MODE_ASYNC, seed=0, step=rule / 16,
                     waves=waves, stream=stream)
        r = g.overlap(2)
        epochs, rel, secs = 2, (g.objective() - fstar) / fstar, 0.0
        while rel > 1e-9 and epochs < 200:
            e0.record(stream)
            g.epochs(1)
            e1.record(stream)
            torch.cuda.synchronize()
            secs += e0.elapsed_time(e1) / 1e3
            epochs += 1
            rel = (g.objective() - fstar) / fstar
        g.close()
        row = {"waves": waves, "tau_mean": r.tau_mean, "tau_p99": r.tau_p99, "tau_max": r.tau_max,
               "latency_us": r.latency_mean_us, "little": r.little, "updates_per_s": r.updates_per_s,
               "epochs_to_1e-9": epochs if rel <= 1e-9 else None, "final_rel": rel,
               "seconds_to_1e-9": secs + 2 * p.n / r.updates_per_s if rel <= 1e-9 else None}
        log(f"tau sweep: {row}")
        out.append(row)
    return {"step_over_serial_rule": 1.0 / 16, "points": out}


def solve_with_stop_test(g, check, stream, target=1e-9, max_launches=600, eager=2.0, max_gap=8, label=""):
    """Run every instance of a batch to `target`, the in-graph stop test
    choosing which instances the host checks exactly.  Each step is one
    epoch call: the batched launch, then on the device the O(d) proxy r_k =
    ||abar_k + lambda_k x_k||^2 of every running instance, which switches
    off those at or below their threshold.  The host then checks exactly
    (check(k): relative suboptimality from FP64 objectives) only the
    instances the test switched off, those never checked and those
    unchecked for `max_gap` epochs.  A check below `target` ends the
    instance; otherwise it (re)calibrates the threshold to the proxy at
    which rel/proxy as measured there would put the instance at eager *
    target, and an instance the test stopped early runs on.  Returns the
    kernel seconds between HIP events on `stream` (host seconds around each
    call when `stream` is None), the counts of launches, checks and early
    stops, and each instance's last checked value and samples."""
    import numpy as np

    ni = g.n_inst
    active = np.ones(ni, dtype=np.uint8)
    rel = np.full(ni, np.inf)
    thr = np.zeros(ni)                       # 0: not calibrated, never stops
    last = np.full(ni, -(10 ** 9))
    applied = np.zeros(ni, dtype=np.int64)
    g.set_active(active)
    g.set_stop(thr)
    if stream is not None:
        import torch
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    kernel_s, launches, checks, early, pairs = 0.0, 0, 0, 0, 0
    while active.any() and launches < max_launches:
        pairs += int(active.sum())
        if stream is not None:
            e0.record(stream)
            g.epochs(1)
            e1.record(stream)
            torch.cuda.synchronize()
            kernel_s += e0.elapsed_time(e1) / 1e3
        else:
            t0 = time.perf_counter()
            g.epochs(1)
            kernel_s += time.perf_counter() - t0
        launches += 1
        proxy, _ = g.stop_report()
        for k in np.nonzero(active)[0]:
            stopped = thr[k] > 0.0 and proxy[k] <= thr[k]   # the device's rule, same doubles
            if not (stopped or thr[k] == 0.0 or launches - last[k] >= max_gap):
                continue
            checks += 1
            last[k] = launches
            rel[k] = check(int(k))
            if rel[k] <= target:
                active[k] = 0
                applied[k] = g.instance(int(k)).t
                continue
            early += int(stopped)
            thr[k] = eager * target * proxy[k] / rel[k] if rel[k] > 0.0 and proxy[k] > 0.0 else 0.0
        g.set_stop(thr)
        g.set_active(active)
        if label and (launches % 8 == 0 or not active.any()):
            log(f"{label}: {launches} launches, {int(active.sum())} instances still active, "
                f"{checks} exact checks, kernel {kernel_s:.3f} s")
    g.set_stop(None)
    for k in np.nonzero(active)[0]:
        applied[k] = g.instance(int(k)).t
    return {"kernel_s": kernel_s, "launches": launches, "checks": checks, "early_stops": early, "rel": rel,
            "applied": applied, "instance_launches": pairs}


def batched_leg(args, dev, stream):
    """The lambda path x folds workload (160 instances over the bfloat16
    config-2 matrix): all instances in one persistent kernel per epoch,
    replayed from a captured hipGraph, autotuned wavefronts per instance,
    hot-set size and step; each instance is switched off once it is within
    1e-9 of its certified optimum, the in-graph stop test choosing which
    instances the host checks exactly after each launch.  Three state precisions: FP32 x, alpha
    and abar in 8-byte slots (the headline), mixed (FP32 x and alpha, FP64
    abar) and FP64; then the same instances one by one with the plain FP64
    async kernel.  Kernel times (the stop test's O(d) kernels included) are
    between HIP events; the exact objective checks between launches are not
    counted there, and the
    end-to-end wall time of each batched solve, checks and re-planning
    included, is reported beside it."""
    import numpy as np
    import torch

    import datagen
    import paper_1606_04809_amd as A

    t = time.time()
    B = datagen.config5()
    p = B.problem
    gold = load_golden().get("config5")
    if gold is None:
        raise SystemExit("tests/golden/fstar.json has no config5 entry")
    import hashlib
    h = hashlib.sha256(p.digest().encode())
    for a in (B.row_fold, B.inst_fold, B.inst_lambda):
        h.update(np.ascontiguousarray(a).tobytes())
    if gold["digest"] != h.hexdigest():
        raise SystemExit("config5 batch differs from the one its optima were computed on")
    fstar = np.array([e["f_lower"] for e in sorted(gold["instances"], key=lambda e: e["k"])])
    ni = B.n_inst
    log(f"generated config5: {ni} instances in {time.time() - t:.1f}s")

    def to_dev(a):
        return torch.from_numpy(np.ascontiguousarray(a)).to(dev)

    arrs = [to_dev(p.rowptr), to_dev(p.colidx), to_dev(p.val_bf16.view(np.int16)), to_dev(p.b)]
    torch.cuda.synchronize()
    m = np.array([int(np.sum(B.row_fold != f)) for f in B.inst_fold])
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    # algorithmic bytes per update: the row list entry (4), row bounds (16),
    # label (8), bfloat16 values and int32 indices (6 per entry), memory read
    # and write (2 x its size)
    mean_k = p.nnz / p.n

    def run_batched(precision, label):
        g = A.Solver(p.n, p.d, *arrs, p.lam, loss=p.loss, val_dtype=A.ASAGA_VAL_BF16, mode=A.ASAGA_MODE_ASYNC,
                     precision=precision, stream=stream, batch=(B.row_fold, B.inst_fold, B.inst_lambda))
        t = time.time()
        log(f"batched {label}: autotune probing wavefronts per instance, hot-set size and step")
        rep = g.autotune(target=1e-9, probe_epochs=6)
        tune = {"candidates": rep.candidates, "waves_per_instance": rep.waves, "hot_columns": rep.hot_columns,
                "gamma_inst0": rep.gamma, "step_groups": rep.step_groups, "step_cap": rep.step_cap,
                "ms_per_epoch": rep.ms_per_epoch, "est_epochs": rep.est_epochs, "tuning_wall_s": time.time() - t}
        log(f"batched {label} autotune: {tune}")
        # samples each instance applied (with automatic waves an instance
        # holding more workgroups than others applies more per launch)
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        res = solve_with_stop_test(g, lambda k: (g.objective(k) - fstar[k]) / fstar[k], stream,
                                   label=f"batched {label}")
        wall_s = time.perf_counter() - w0
        kernel_s, launches, rel, applied = res["kernel_s"], res["launches"], res["rel"], res["applied"]
        hot = g.info().hot_columns
        g.close()
        epochs = applied / m
        updates = int(applied.sum())
        s_alpha = 8 if precision == A.ASAGA_PREC_F64 else 4
        bpu = 4 + 16 + 8 + 6 * mean_k + 2 * s_alpha
        gbps = bpu * updates / kernel_s / 1e9
        return {"instances": ni, "reached": int(np.sum(rel <= 1e-9)), "launches": launches,
                "exact_checks": res["checks"], "early_stops": res["early_stops"],
                "exact_checks_if_every_launch": res["instance_launches"],
                "epochs_max": float(epochs.max()), "epochs_median": float(np.median(epochs)),
                "seconds_to_1e-9_all": kernel_s, "wall_seconds_to_1e-9_all": wall_s, "updates": updates,
                "updates_per_s": updates / kernel_s, "worst_rel_subopt": float(np.max(rel)),
                "hot_columns_last_launch": hot,
                "roofline": {"bound": "hbm", "achieved": gbps, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                             "frac": gbps / HBM_PEAK_GBPS, "bytes_per_update": bpu,
                             "kernel": "k_update_batched"},
                "autotune": tune}

    out = {"workload": "config5: 32 lambdas (1e-8..1e-2) x 5 uneven folds over the bfloat16 config-2 matrix, "
                       "FP32 x, alpha and abar (8-byte slots, compensated hot-column flushes), one persistent "
                       "kernel per launch from a hipGraph"}
    out.update(run_batched(A.ASAGA_PREC_F32, "FP32 state"))
    log(f"batched FP32 state: {out}")
    out["mixed"] = run_batched(A.ASAGA_PREC_MIXED, "mixed")
    out["mixed"]["workload"] = "the same batch, FP32 x/alpha, FP64 abar, bfloat16 values"
    log(f"batched mixed: {out['mixed']}")
    if args.batched_f64_state:
        # the same batch with FP64 x, alpha and abar (values still bfloat16)
        out["f64_state"] = run_batched(A.ASAGA_PREC_F64, "FP64 state")
        out["f64_state"]["workload"] = "the same batch, FP64 x/alpha/abar, bfloat16 values"
        log(f"batched FP64 state: {out['f64_state']}")
    del arrs

    # the same instances one by one: plain FP64 async kernel, library defaults
    sel = np.unique(np.linspace(0, ni - 1, max(1, min(args.plain_instances, ni))).round().astype(int))
    plain_s, plain_updates, plain_reached, plain_epochs = 0.0, 0, 0, []
    for f in range(5):
        ks = [k for k in sel if B.inst_fold[k] == f]
        if not ks:
            continue
        sub = datagen.subproblem(p, B.rows(ks[0]))
        arrs = [to_dev(a) for a in (sub.rowptr, sub.colidx, sub.val, sub.b)]
        torch.cuda.synchronize()
        for k in ks:
            g = A.Solver(sub.n, sub.d, *arrs, float(B.inst_lambda[k]), loss=sub.loss, mode=A.ASAGA_MODE_ASYNC,
                         stream=stream)
            r, ep = np.inf, 0
            while r > 1e-9 and ep < 600:
                e0.record(stream)
                g.epochs(1)
                e1.record(stream)
                torch.cuda.synchronize()
                plain_s += e0.elapsed_time(e1) / 1e3
                plain_updates += sub.n
                ep += 1
                r = (g.objective() - fstar[k]) / fstar[k]
            plain_reached += int(r <= 1e-9)
            plain_epochs.append(ep)
            if k % 16 == 15:
                log(f"plain instance {k}: {ep} epochs, rel {r:.2e}, total kernel {plain_s:.3f} s")
            g.close()
        del arrs
    scale = ni / len(sel)
    out["plain_one_by_one"] = {
        "instances_run": int(len(sel)), "reached": plain_reached, "seconds_to_1e-9": plain_s,
        "seconds_to_1e-9_all_160_est": plain_s * scale, "updates_per_s": plain_updates / plain_s,
        "epochs_median": float(np.median(plain_epochs)), "epochs_max": int(np.max(plain_epochs)),
        "kernel": "plain FP64 async (k_update, library default shape and step), one instance at a time"}
    out["batched_speedup_vs_plain"] = plain_s * scale / out["seconds_to_1e-9_all"]
    log(f"plain one by one: {out['plain_one_by_one']}")
    return out


def batched_throughput(args, dev, stream, precisions=None):
    """Kernel throughput of the batched update with all 160 instances of the
    config-5 batch active: `warmup` launches, then `steps` launches in one
    asaga_epochs call (replayed from its captured hipGraph), at the default
    step law and automatic workgroups (what asaga_autotune chooses on this
    batch), with the stop test armed at threshold 0 (its O(d) proxy kernel
    after every launch, as in the solve; no instance stops); updates/s from
    the instances' sample counters and HIP events on the library's stream,
    and the algorithmic HBM rate."""
    import numpy as np
    import torch

    import datagen
    import paper_1606_04809_amd as A

    B = datagen.config5()
    p = B.problem
    arrs = [torch.from_numpy(np.ascontiguousarray(a)).to(dev)
            for a in (p.rowptr, p.colidx, p.val_bf16.view(np.int16), p.b)]
    torch.cuda.synchronize()
    mean_k = p.nnz / p.n
    out = {}
    names = {A.ASAGA_PREC_F32: "f32_state", A.ASAGA_PREC_MIXED: "mixed", A.ASAGA_PREC_F64: "f64_state"}
    for prec in precisions or (A.ASAGA_PREC_F32, A.ASAGA_PREC_F64):
        g = A.Solver(p.n, p.d, *arrs, p.lam, loss=p.loss, val_dtype=A.ASAGA_VAL_BF16, mode=A.ASAGA_MODE_ASYNC,
                     precision=prec, stream=stream, batch=(B.row_fold, B.inst_fold, B.inst_lambda))
        g.set_stop(np.zeros(B.n_inst))
        g.epochs(args.warmup)
        torch.cuda.synchronize()
        t0 = sum(g.instance(k).t for k in range(B.n_inst))
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        g.epochs(args.steps)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        updates = sum(g.instance(k).t for k in range(B.n_inst)) - t0
        info = g.info()
        g.close()
        bpu = 4 + 16 + 8 + 6 * mean_k + 2 * (8 if prec == A.ASAGA_PREC_F64 else 4)
        gbps = bpu * updates / (ms / 1e3) / 1e9
        out[names[prec]] = {"launches": args.steps, "ms_per_launch": ms / args.steps, "updates": int(updates),
                            "updates_per_s": updates / (ms / 1e3), "hot_columns": info.hot_columns,
                            "threads_per_block": info.threads_per_block, "bytes_per_update": bpu,
                            "roofline": {"bound": "hbm", "achieved": gbps, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                                         "frac": gbps / HBM_PEAK_GBPS, "kernel": "k_update_batched"}}
        log(f"batched throughput {names[prec]}: {out[names[prec]]}")
    return out


def config4_throughput(args, dev, stream, p=None):
    """Kernel throughput of the URL-shaped instance (bfloat16 values, FP32
    state) at a fixed launch shape: `warmup` epochs, then `steps` timed."""
    import numpy as np
    import torch

    import datagen
    import paper_1606_04809_amd as A

    p = datagen.config4() if p is None else p
    arrs = [torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in
            (p.rowptr, p.colidx, p.val_bf16.view(np.int16), p.b)]
    torch.cuda.synchronize()
    g = A.Solver(p.n, p.d, *arrs, p.lam, loss=p.loss, val_dtype=A.ASAGA_VAL_BF16, mode=A.ASAGA_MODE_ASYNC,
                 precision=A.ASAGA_PREC_F32, waves=args.config4_waves, stream=stream)
    g.epochs(args.warmup)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    g.epochs(args.steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    info = g.info()
    g.close()
    bpu = 6 * p.nnz / p.n + 16 + 8 + 8
    gbps = bpu * p.n / (ms / 1e3) / 1e9
    out = {"waves": info.waves, "threads_per_block": info.threads_per_block, "hot_columns": info.hot_columns,
           "ms_per_epoch": ms, "updates_per_s": p.n / (ms / 1e3), "bytes_per_update": bpu,
           "roofline": {"bound": "hbm", "achieved": gbps, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                        "frac": gbps / HBM_PEAK_GBPS, "kernel": "k_update (FP32 state, bfloat16 values)"}}
    log(f"config4 throughput: {out}")
    return out


def config2_plain_values_leg(dev, stream):
    """The other reading of config 2's values: lognormal(0, 1) alone (no idf
    factor), the same supports and labels recipe.  Its rows share a
    stronger common direction, so the stable asynchronous step is smaller:
    the benchmarked shape and step, then the autotuned ones, each to 1e-9."""
    import numpy as np
    import torch

    import datagen
    import paper_1606_04809_amd as A

    p = datagen.config2(idf=False)
    gold = load_golden()["config2_plain_lognormal"]
    if gold["digest"] != p.digest():
        raise SystemExit("the plain-lognormal config-2 instance differs from the one its optimum was computed on")
    fstar = gold["f_lower"]
    arrs = [torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in (p.rowptr, p.colidx, p.val, p.b)]
    torch.cuda.synchronize()
    rule = 1.0 / (3.0 * (0.25 * float(np.max(np.add.reduceat(p.val ** 2, p.rowptr[:-1]))) + p.lam))
    out = {"workload": "config2 with lognormal(0,1) values and no idf factor (700,000 x 47,000, FP64 async)",
           "oracle_epochs_to_1e-9": gold.get("oracle_tta", {}).get("epochs")}
    g = A.Solver(p.n, p.d, *arrs, p.lam, loss=p.loss, mode=A.ASAGA_MODE_ASYNC, threads_per_block=1024, waves=4096,
                 step=rule / 8, stream=stream)
    ep, secs, rel = run_until(g, fstar, stream, max_epochs=100, every=1)
    out["benchmarked_shape"] = {"waves": 4096, "gamma_over_serial_rule": 0.125, "epochs": ep, "seconds": secs,
                                "final_rel_subopt": rel, "reached": rel <= 1e-9, "ms_per_epoch": 1e3 * secs / ep}
    g.close()
    g = A.Solver(p.n, p.d, *arrs, p.lam, loss=p.loss, mode=A.ASAGA_MODE_ASYNC, stream=stream)
    rep = g.autotune(target=1e-9, probe_epochs=9)
    ep, secs, rel = run_until(g, fstar, stream, max_epochs=200, every=1)
    info = g.info()
    out["autotuned"] = {"waves": info.waves, "threads_per_block": info.threads_per_block,
                        "gamma_over_serial_rule": info.gamma * 3.0 * info.L, "epochs": ep, "seconds": secs,
                        "final_rel_subopt": rel, "reached": rel <= 1e-9, "ms_per_epoch": 1e3 * secs / ep}
    g.close()
    log(f"config2 plain lognormal values: {out}")
    return out


def racy_leg(dev, stream):
    """Appendix G: the same instance, step and launch with atomic additions
    and with plain read-modify-writes (no LDS combining, so every write of
    the racy run goes to the shared state unprotected): relative
    suboptimality after 10, 20, 40 and 60 epochs."""
    import numpy as np

    import datagen
    import paper_1606_04809_amd as A

    p = datagen.config2(n=20_000, d=2000)
    gold = load_golden()["config2_20000x2000"]
    if gold["digest"] != p.digest():
        raise SystemExit("the 20,000-row instance differs from the one its optimum was computed on")
    fstar = gold["f_lower"]
    rule = 1.0 / (3.0 * (0.25 * float(np.max(np.add.reduceat(p.val ** 2, p.rowptr[:-1]))) + p.lam))
    out = {"workload": "RCV1-shaped recipe at 20,000 x 2,000, lambda = 1/n, 512 wavefronts, no hot set, "
                       "step = serial rule / 4, 60 epochs", "target": 1e-9}
    for racy in (0, 1):
        g = A.Solver(p.n, p.d, p.rowptr, p.colidx, p.val, p.b, p.lam, loss=p.loss, mode=A.ASAGA_MODE_ASYNC,
                     waves=512, racy=racy, hot_columns=-1, step=rule / 4, stream=stream)
        rels = []
        for e in range(60):
            g.epochs(1)
            try:
                rels.append((g.objective() - fstar) / fstar)
            except A.AsagaError:
                rels.append(float("inf"))
        g.close()
        key = "racy" if racy else "atomic"
        out[key] = {"rel_subopt_at_epochs": {str(e): rels[e - 1] for e in (10, 20, 40, 60)},
                    "best_rel_subopt": min(rels), "reached_target": min(rels) <= 1e-9}
        log(f"{key}: {out[key]}")
    return out


def config1_leg(stream):
    """The tiny instance in the deterministic serial mode (one lane group in
    the oracle's sample order), 50 epochs, each timed; relative
    suboptimality against the Newton optimum after each."""
    import torch

    import datagen
    import paper_1606_04809_amd as A

    p = datagen.config1()
    gold = load_golden()["config1"]
    if gold["digest"] != p.digest():
        raise SystemExit("config1 differs from the instance f* was computed on")
    fstar = gold["f_star"]
    g = A.from_problem(p, mode=A.ASAGA_MODE_SERIAL, stream=stream)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    secs, first, rel = 0.0, None, float("inf")
    for e in range(1, 51):
        e0.record(stream)
        g.epochs(1)
        e1.record(stream)
        torch.cuda.synchronize()
        secs += e0.elapsed_time(e1) / 1e3
        rel = (g.objective() - fstar) / fstar
        if first is None and rel <= 1e-9:
            first = (e, secs)
    g.close()
    return {"workload": "config1: 2,000 x 500 L2 logistic, serial FP64 (one lane group, oracle sample order)",
            "epochs": 50, "seconds": secs, "updates_per_s": 50 * p.n / secs, "rel_subopt_after_50": rel,
            "epochs_to_1e-9": first[0] if first else None, "seconds_to_1e-9": first[1] if first else None}


def run_until(g, fstar, stream, target=1e-9, max_epochs=800, every=5):
    """Kernel seconds (HIP events) and epochs until (f - f*)/f* <= target."""
    import torch
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    secs, ep, rel = 0.0, 0, float("inf")
    while ep < max_epochs and rel > target:
        e0.record(stream)
        g.epochs(every)
        e1.record(stream)
        torch.cuda.synchronize()
        secs += e0.elapsed_time(e1) / 1e3
        ep += every
        rel = (g.objective() - fstar) / fstar
    return ep, secs, rel


def config3_leg(dev, stream):
    """The Covtype-shaped least squares (581,000 x 54, the same ten dense
    columns in every row): FP64 async, autotuned; then FP32 state (up to 100
    epochs, checked every 10), widened to FP64 and polished to 1e-9 if it
    stalled above it."""
    import numpy as np
    import torch

    import datagen
    import paper_1606_04809_amd as A

    p = datagen.config3()
    gold = load_golden()["config3"]
    if gold["digest"] != p.digest():
        raise SystemExit("config3 differs from the instance f* was computed on")
    fstar = gold["f_star"]
    arrs = [torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in (p.rowptr, p.colidx, p.val, p.b)]
    torch.cuda.synchronize()
    out = {"workload": "config3: 581,000 x 54 L2 least squares, lambda = 1e-4 (FP64 values)"}
    bpu = 12 * p.nnz / p.n + 16 + 8 + 16
    g = A.Solver(p.n, p.d, *arrs, p.lam, loss=p.loss, mode=A.ASAGA_MODE_ASYNC, stream=stream)
    t = time.time()
    rep = g.autotune(target=1e-9, probe_epochs=9)
    tune_s = time.time() - t
    ep, secs, rel = run_until(g, fstar, stream)
    out["fp64"] = {"epochs": ep, "seconds_to_1e-9": secs, "final_rel_subopt": rel, "reached": rel <= 1e-9,
                   "updates_per_s": ep * p.n / secs, "hbm_gbps_algorithmic": bpu * ep * p.n / secs / 1e9,
                   "waves": rep.waves, "threads_per_block": rep.threads_per_block,
                   "gamma_over_serial_rule": rep.gamma * 3.0 * g.info().L,
                   "autotune_wall_s": tune_s}
    g.close()
    log(f"config3 FP64: {out['fp64']}")
    g = A.Solver(p.n, p.d, *arrs, p.lam, loss=p.loss, mode=A.ASAGA_MODE_ASYNC, precision=A.ASAGA_PREC_F32,
                 stream=stream)
    rep = g.autotune(target=1e-9, probe_epochs=9)
    ep32, s32, rel32 = run_until(g, fstar, stream, max_epochs=100, every=10)
    ep64, s64, rel64 = 0, 0.0, rel32
    if rel32 > 1e-9:
        # FP32 x stalled above the target: the FP64 polish finishes
        g.widen()
        ep64, s64, rel64 = run_until(g, fstar, stream, every=10)
    out["fp32_then_fp64"] = {"fp32_epochs": ep32, "fp32_seconds": s32, "rel_subopt_fp32": rel32,
                             "fp64_epochs": ep64, "fp64_seconds": s64, "final_rel_subopt": rel64,
                             "reached": rel64 <= 1e-9, "seconds_to_1e-9": s32 + s64,
                             "fp32_updates_per_s": ep32 * p.n / s32 if s32 > 0 else None,
                             "waves": rep.waves, "threads_per_block": rep.threads_per_block, "gamma": rep.gamma,
                             "fp64_polish_gamma": rep.widen_gamma if ep64 else None}
    g.close()
    log(f"config3 FP32 then FP64: {out['fp32_then_fp64']}")
    return out


def config4_leg(dev, stream, p=None):
    """The URL-shaped instance (2.4M x 3.2M, ~115 binary entries per row,
    bfloat16 values): FP32 state, autotuned shape and step, to 1e-9; if the
    FP32 iterate stalls above it (FP32 x cannot hold this optimum more
    closely than its own rounding, which small steps raise), asaga_widen
    switches to FP64 and the same shape polishes to 1e-9."""
    import numpy as np
    import torch

    import datagen
    import paper_1606_04809_amd as A

    t = time.time()
    p = datagen.config4() if p is None else p
    gold = load_golden()["config4"]
    if gold["digest"] != p.digest():
        raise SystemExit("config4 differs from the instance f* was computed on")
    log(f"config4 ready in {time.time() - t:.1f}s")
    fstar = gold["f_lower"]
    arrs = [torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in
            (p.rowptr, p.colidx, p.val_bf16.view(np.int16), p.b)]
    torch.cuda.synchronize()
    g = A.Solver(p.n, p.d, *arrs, p.lam, loss=p.loss, val_dtype=A.ASAGA_VAL_BF16, mode=A.ASAGA_MODE_ASYNC,
                 precision=A.ASAGA_PREC_F32, stream=stream)
    t = time.time()
    log("config4: autotune probing wavefronts and step, then racing the finalists")
    rep = g.autotune(target=1e-9, probe_epochs=6)
    tune_s = time.time() - t
    info = g.info()
    log(f"config4 autotune: waves {rep.waves}, gamma {rep.gamma:.4g}, {rep.ms_per_epoch:.1f} ms/epoch, "
        f"{rep.est_epochs:.0f} epochs in the race, {tune_s:.1f} s")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    # FP32 epochs until 1e-9, or until the FP32 iterate stalls: less than a
    # 20% lower objective gap in the last 20 epochs
    secs32, ep32, rel, hist = 0.0, 0, float("inf"), []
    while ep32 < 400 and rel > 1e-9 and not (len(hist) > 4 and min(hist[-4:]) > 0.8 * min(hist[:-4])):
        e0.record(stream)
        g.epochs(5)
        e1.record(stream)
        torch.cuda.synchronize()
        secs32 += e0.elapsed_time(e1) / 1e3
        ep32 += 5
        rel = (g.objective() - fstar) / fstar
        hist.append(rel)
    rel32, secs64, ep64 = rel, 0.0, 0
    if rel > 1e-9:
        g.widen()
        ep64, secs64, rel = run_until(g, fstar, stream, max_epochs=400)
    g.close()
    ep, secs = ep32 + ep64, secs32 + secs64
    bpu = 6 * p.nnz / p.n + 16 + 8 + 8
    out = {"workload": "config4: 2,400,000 x 3,200,000 L2 logistic, bfloat16 values, FP32 state (FP64 polish "
                       "if FP32 stalls above the target)",
           "epochs": ep, "seconds_to_1e-9": secs, "final_rel_subopt": rel, "reached": rel <= 1e-9,
           "fp32_epochs": ep32, "fp32_seconds": secs32, "rel_subopt_fp32": rel32, "fp64_polish_epochs": ep64,
           "fp64_polish_seconds": secs64, "fp32_updates_per_s": ep32 * p.n / secs32 if secs32 > 0 else None,
           "fp32_hbm_gbps_algorithmic": bpu * ep32 * p.n / secs32 / 1e9 if secs32 > 0 else None,
           "bytes_per_update_fp32": bpu, "waves": info.waves, "threads_per_block": info.threads_per_block,
           "hot_columns": info.hot_columns, "gamma": info.gamma, "gamma_over_serial_rule": info.gamma * 3.0 * info.L,
           "fp64_polish_gamma": rep.widen_gamma if ep64 else None,
           "autotune_wall_s": tune_s, "autotune_race_epochs": rep.est_epochs}
    log(f"config4: {out}")
    return out

def cpu_legs(args, p2, p4):
    """The CPU oracle (single-thread FP64 Sparse SAGA, the test
    infrastructure's reference) timed on bounded samples of each workload on
    this host, after the GPU work.  Config 2 (the headline): epochs on one
    pinned core.  The oracle's time to 1e-9 is its stored epochs to 1e-9
    (written by tests/golden/make_golden.py) times the seconds per epoch
    measured here, except on config 1, which runs to 1e-9 here.  Config 5:
    one instance per thread on up to 16 host cores at once (the oracle's C
    loop runs outside the interpreter lock), one epoch each; the time for
    all 160 instances is their stored epochs times the per-epoch times
    measured under that load, packed perfectly onto those cores."""
    import dataclasses
    import threading

    import numpy as np

    import datagen
    import oracle

    gold = load_golden()
    out = {}
    prev, core = None, None
    try:
        prev = os.sched_getaffinity(0)
        core = min(prev)
        os.sched_setaffinity(0, {core})
    except (AttributeError, OSError):
        prev = None
    try:
        sv = oracle.SparseSaga(p2, seed=0)
        t = time.perf_counter()
        sv.epochs(args.cpu_epochs)
        dt = time.perf_counter() - t
        tta2 = gold["config2"]["oracle_tta"]["epochs"]
        out["config2"] = {"value": args.cpu_epochs * p2.n / dt, "unit": "updates/s", "cores": 1, "kind": "oracle",
                          "sample": f"{args.cpu_epochs} epochs ({args.cpu_epochs * p2.n} updates) of the config-2 "
                                    f"workload, serial FP64 Sparse SAGA, one thread pinned to one core, {dt:.1f} s",
                          "pinned_core": core, "seconds_per_epoch": dt / args.cpu_epochs,
                          "epochs_to_1e-9": tta2, "seconds_to_1e-9_est": tta2 * dt / args.cpu_epochs}
        log(f"cpu oracle config2: {out['config2']}")
        # config 1: to 1e-9 here, checks not timed
        p1 = datagen.config1()
        f1 = gold["config1"]["f_star"]
        sv = oracle.SparseSaga(p1)
        secs, ep, rel = 0.0, 0, float("inf")
        while rel > 1e-9 and ep < 200:
            t = time.perf_counter()
            sv.epochs(1)
            secs += time.perf_counter() - t
            ep += 1
            rel = (sv.objective() - f1) / f1
        out["config1"] = {"epochs_to_1e-9": ep, "seconds_to_1e-9": secs, "updates_per_s": ep * p1.n / secs,
                          "cores": 1}
        # config 3 and 4: bounded samples
        p3 = datagen.config3()
        sv = oracle.SparseSaga(p3)
        t = time.perf_counter()
        sv.epochs(3)
        dt = time.perf_counter() - t
        e3 = gold["config3"]["oracle_tta"]["epochs"]
        out["config3"] = {"updates_per_s": 3 * p3.n / dt, "seconds_per_epoch": dt / 3, "epochs_to_1e-9": e3,
                          "seconds_to_1e-9_est": e3 * dt / 3, "cores": 1, "sample": "3 epochs"}
        if p4 is not None:
            sv = oracle.SparseSaga(p4)
            t = time.perf_counter()
            sv.epochs(1)
            dt = time.perf_counter() - t
            e4 = gold["config4"]["oracle_tta"]["epochs"]
            out["config4"] = {"updates_per_s": p4.n / dt, "seconds_per_epoch": dt, "epochs_to_1e-9": e4,
                              "seconds_to_1e-9_est": e4 * dt, "cores": 1, "sample": "1 epoch"}
            del sv
        log(f"cpu oracle configs 1, 3, 4: {out.get('config1')}, {out.get('config3')}, {out.get('config4')}")
    finally:
        if prev is not None:
            os.sched_setaffinity(0, prev)

    # config 5: one instance per thread on up to 16 cores
    cores = sorted(prev) if prev is not None else list(range(os.cpu_count() or 1))
    P = max(1, min(16, len(cores)))
    B = datagen.config5()
    g5 = {e["k"]: e for e in gold["config5"]["instances"]}
    by_fold = {}
    for f in range(5):
        k = int(np.nonzero(B.inst_fold == f)[0][0])
        by_fold[f] = B.instance(k)
    ks = np.unique(np.linspace(0, B.n_inst - 1, P).round().astype(int))
    solvers = [oracle.SparseSaga(dataclasses.replace(by_fold[int(B.inst_fold[k])], lam=float(B.inst_lambda[k])))
               for k in ks]
    barrier = threading.Barrier(len(ks))
    secs = [0.0] * len(ks)

    def work(j):
        try:
            os.sched_setaffinity(0, {cores[j % len(cores)]})
        except (AttributeError, OSError):
            pass
        barrier.wait()
        t = time.perf_counter()
        solvers[j].epochs(1)
        secs[j] = time.perf_counter() - t

    t = time.perf_counter()
    threads = [threading.Thread(target=work, args=(j,)) for j in range(len(ks))]
    for th in threads:
        th.start()
    for th in threads:
        th.join()
    wall = time.perf_counter() - t
    if prev is not None:
        os.sched_setaffinity(0, prev)
    per_update = float(np.mean([secs[j] / solvers[j].n for j in range(len(ks))]))
    core_s = sum(g5[k]["oracle_tta"]["epochs"] * g5[k]["m"] * per_update for k in range(B.n_inst))
    m_run = sum(solvers[j].n for j in range(len(ks)))
    out["config5"] = {"cores": len(ks), "updates_per_s": m_run / wall,
                      "sample": f"one epoch each of {len(ks)} instances (spread over lambda and folds), one per "
                                f"thread, {wall:.1f} s",
                      "epochs_to_1e-9_median": float(np.median([g5[k]["oracle_tta"]["epochs"] for k in g5])),
                      "epochs_to_1e-9_max": int(max(g5[k]["oracle_tta"]["epochs"] for k in g5)),
                      "seconds_to_1e-9_all_160_est": core_s / len(ks)}
    log(f"cpu oracle config5: {out['config5']}")
    return out


def copy_calibration(dev):
    """A plain 1 GiB device-to-device copy (known bytes read and written), so
    that a profiler's per-dispatch byte counters can be scaled to bytes."""
    import torch
    src = torch.empty(1 << 27, dtype=torch.float64, device=dev)   # 1 GiB
    dst = torch.empty_like(src)
    src.fill_(1.0)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    log(f"copy calibration: {src.numel() * 8} bytes read and written")
    del src, dst


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--waves", type=int, default=4096)
    ap.add_argument("--lanes", type=int, default=0)
    ap.add_argument("--skip-cpu", action="store_true", help="omit the CPU oracle leg")
    ap.add_argument("--skip-tta", action="store_true", help="omit the time-to-accuracy leg")
    ap.add_argument("--cpu-epochs", type=int, default=30)
    ap.add_argument("--hot", type=int, default=0)
    ap.add_argument("--flush", type=int, default=0)
    # The benchmarked shape: 1024-thread workgroups, one per compute unit
    # (4096 wavefronts), at 1/8 of the serial rule (stable with margin: the
    # measured edge on this workload is near 0.17).  --library-defaults runs
    # the library's own defaults instead (512-thread workgroups, 2048
    # wavefronts, rule x 512 / 2048).
    ap.add_argument("--block", type=int, default=1024)
    ap.add_argument("--step-scale", type=float, default=0.125,
                    help="step as a multiple of the serial rule 1/(3L) (0: the library's asynchronous default)")
    ap.add_argument("--library-defaults", action="store_true",
                    help="throughput and time-to-accuracy legs at the library's default shape and step")
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="use the library's default launch shape and step instead of asaga_autotune's choice")
    ap.add_argument("--skip-batched", action="store_true", help="omit the batched lambda-path x folds leg")
    ap.add_argument("--no-tau-sweep", dest="tau_sweep", action="store_false",
                    help="omit the overlap sweep (samples in flight, measured, and epochs to 1e-9 at a fixed step "
                         "versus wavefronts in flight)")
    ap.add_argument("--skip-racy", action="store_true", help="omit the atomic vs racy comparison (Appendix G)")
    ap.add_argument("--skip-configs", action="store_true",
                    help="omit the legs of the other workloads (tiny serial, Covtype-shaped, URL-shaped)")
    ap.add_argument("--no-batched-f64-state", dest="batched_f64_state", action="store_false",
                    help="omit the batched run with FP64 state (the mixed-precision batched run stays)")
    ap.add_argument("--only", choices=("config2", "batched", "config4"), default=None,
                    help="run only that workload's throughput measurement (for profiling runs): config2 at the "
                         "benchmarked shape, the config-5 batch with every instance active, or config4 at "
                         "--config4-waves wavefronts; --steps and --warmup apply")
    ap.add_argument("--config4-waves", type=int, default=512)
    ap.add_argument("--plain-instances", type=int, default=160,
                    help="instances of the batch also solved one by one with the plain FP64 kernel (spread "
                         "evenly over the 160)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on exactly one GPU (the asynchronous solve of one instance lives in one "
              "device's memory); --gpus must be 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import datagen
    import paper_1606_04809_amd as A

    torch.cuda.init()
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)

    if args.only in ("batched", "config4"):
        if args.copy_calibration:
            copy_calibration(dev)
        if args.only == "batched":
            res = batched_throughput(args, dev, stream,
                                     (A.ASAGA_PREC_F32, A.ASAGA_PREC_MIXED, A.ASAGA_PREC_F64))
        else:
            res = config4_throughput(args, dev, stream)
        print(json.dumps({"only": args.only, "steps": args.steps, "warmup": args.warmup, "result": res}),
              flush=True)
        return
    if args.only == "config2":
        args.no_autotune = args.skip_tta = args.skip_batched = args.skip_racy = True
        args.skip_configs = args.skip_cpu = True
        args.tau_sweep = False

    t = time.time()
    p = datagen.config2()
    log(f"generated config2 n={p.n} d={p.d} nnz={p.nnz} in {time.time() - t:.1f}s")
    gold = load_golden()["config2"]
    if gold["digest"] != p.digest():
        raise SystemExit("config2 instance differs from the one f* was computed on")
    fstar = gold["f_lower"]

    # inputs resident in HBM before timing: the library borrows these tensors
    dev_arrays = [torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in (p.rowptr, p.colidx, p.val, p.b)]
    torch.cuda.synchronize()

    step = 0.0
    if args.step_scale > 0:
        step = args.step_scale / (3.0 * (0.25 * float(np.max(np.add.reduceat(p.val ** 2, p.rowptr[:-1]))) + p.lam))
    if args.library_defaults:
        step = 0.0
        args.waves = args.block = 0

    shape = dict(waves=args.waves, lanes_per_sample=args.lanes, hot_columns=args.hot, flush_every=args.flush,
                 threads_per_block=args.block)

    def make_solver(step=step, shape=shape):
        return A.Solver(p.n, p.d, *dev_arrays, p.lam, loss=p.loss, mode=A.ASAGA_MODE_ASYNC, seed=0, step=step,
                        stream=stream, **shape)

    # ---- autotuning (untimed): launch shape and step for time to 1e-9 ---------
    # The throughput leg runs the library's default shape and step (or the
    # ones given on the command line); the time-to-accuracy leg runs what
    # asaga_autotune chooses for that target.
    tune = None
    tta_step, tta_shape = step, dict(shape)
    if not args.no_autotune:
        t = time.time()
        g = make_solver(0.0)   # the ladder starts from the serial rule
        rep = g.autotune(target=1e-9, probe_epochs=9)
        g.close()
        tune = {"candidates": rep.candidates, "waves": rep.waves, "threads_per_block": rep.threads_per_block,
                "hot_columns": rep.hot_columns,
                "hot_tier_columns": rep.hot_tier_columns, "gamma": rep.gamma, "ms_per_epoch": rep.ms_per_epoch,
                "est_epochs": rep.est_epochs, "est_seconds": rep.est_seconds, "tuning_wall_s": time.time() - t}
        log(f"autotune: {tune}")
        tta_step = rep.gamma
        tta_shape.update(waves=rep.waves, hot_columns=rep.hot_columns, hot_tier_columns=rep.hot_tier_columns)

    if args.copy_calibration:
        copy_calibration(dev)

    # ---- throughput: W warm-up epochs, then K timed epochs -------------------
    g = make_solver()
    info = g.info()
    log(f"async: waves={info.waves} lanes/sample={info.lanes_per_sample} hot={info.hot_columns} "
        f"flush={info.flush_every} block={info.threads_per_block} gamma={info.gamma:.6g} L={info.L:.6g}")
    for _ in range(args.warmup):
        g.epochs(1)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    t0 = time.perf_counter()
    ev[0].record(stream)
    for k in range(args.steps):
        g.epochs(1)
        ev[k + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    g.sync()
    launch_ms = [ev[k].elapsed_time(ev[k + 1]) for k in range(args.steps)]
    total_ms = sum(launch_ms)
    updates = args.steps * p.n
    ups = updates / (total_ms / 1e3)
    f_after = g.objective()
    g.close()
    log(f"throughput: {ups / 1e6:.1f} M updates/s, {total_ms / args.steps:.3f} ms/epoch "
        f"(wall {wall * 1e3 / args.steps:.3f} ms/epoch); f={f_after:.15g}")

    # algorithmic bytes per update (expected over uniform sampling): the CSR
    # stream k*(4+8) + rowptr 16 + label 8 + memory read and write 16
    mean_k = p.nnz / p.n
    bytes_per_update = mean_k * 12.0 + 16.0 + 8.0 + 16.0
    bytes_per_launch = bytes_per_update * p.n
    avg_launch_s = total_ms / args.steps / 1e3
    achieved_gbps = bytes_per_launch / avg_launch_s / 1e9
    # the launch shape the committed counter summaries were taken at, if this is one
    if args.library_defaults:
        prof_shape = "library"
    elif (args.block, args.waves, args.step_scale, args.hot, args.flush, args.lanes) == (1024, 4096, 0.125, 0, 0, 0):
        prof_shape = "benchmarked"
    else:
        prof_shape = None
    traffic = traffic_from_profile(p.n, prof_shape)
    requests = requests_from_profile(p.n, prof_shape)
    # the device's memory-side request ceiling, measured now (random 16-byte
    # slots of a state of d columns: atomics only, and one coherent read plus
    # one atomic, the update's mix)
    ceil_atomic, ceil_mixed = A.asaga_request_ceiling(p.d)
    ceiling = {"atomic_per_s": ceil_atomic, "read_plus_atomic_per_s": ceil_mixed}
    log(f"memory-side request ceiling: {ceil_mixed:.3e}/s (atomics only: {ceil_atomic:.3e}/s)")
    if requests is not None:
        # memory-side requests per second at this run's measured update rate
        total = (requests["atomic_per_update"] + requests["read_per_update"]) * ups
        per_update = requests["atomic_per_update"] + requests["read_per_update"]
        requests.update(atomic_per_s=requests["atomic_per_update"] * ups, read_per_s=requests["read_per_update"] * ups,
                        frac_of_ceiling=total / ceil_mixed, source=os.path.relpath(REQUEST_SUMMARY, ROOT),
                        # the request roofline: updates/s at which this many
                        # memory-side requests per update meet the ceiling
                        roofline_updates_per_s=ceil_mixed / per_update)
        log(f"memory-side requests: {total:.3e}/s = {total / ceil_mixed:.2f} of the ceiling")

    # ---- time to 1e-9 relative suboptimality from a cold start ----------------
    def time_to_target(step, shape, runs=5):
        """Kernel seconds to 1e-9 from x = 0, the median of `runs` runs
        (each checked after every epoch, the checks not timed)."""
        res = []
        for _ in range(runs):
            g = make_solver(step, shape)
            ti = g.info()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            kernel_s = 0.0
            rel = float("inf")
            epochs = 0
            while epochs < 100:
                e0.record(stream)
                g.epochs(1)
                e1.record(stream)
                torch.cuda.synchronize()
                kernel_s += e0.elapsed_time(e1) / 1e3
                epochs += 1
                rel = (g.objective() - fstar) / fstar
                if rel <= 1e-9:
                    break
            g.close()
            res.append((kernel_s, epochs, rel))
        secs = sorted(r[0] for r in res)
        mid = sorted(res)[len(res) // 2]
        return {"target": 1e-9, "reached": all(r[2] <= 1e-9 for r in res), "epochs": mid[1], "seconds": mid[0],
                "runs": runs, "seconds_each": [r[0] for r in res], "epochs_each": [r[1] for r in res],
                "seconds_min": secs[0], "seconds_max": secs[-1], "final_rel_subopt": mid[2], "waves": ti.waves,
                "threads_per_block": ti.threads_per_block, "hot_columns": ti.hot_columns, "gamma": ti.gamma,
                "gamma_over_serial_rule": ti.gamma * 3.0 * ti.L}

    tta = tta_tuned = tta_svrg = None
    if not args.skip_tta:
        tta = time_to_target(step, shape)
        log(f"time to 1e-9 (benchmarked shape): {tta}")
        # sparse SVRG (Appendix C variant) on the same kernel, shape and step
        tta_svrg = time_to_target(step, dict(shape, method=A.ASAGA_METHOD_SVRG))
        log(f"time to 1e-9 (sparse SVRG, same shape and step): {tta_svrg}")
        if tune is not None:
            tta_tuned = time_to_target(tta_step, tta_shape)
            log(f"time to 1e-9 (autotuned shape): {tta_tuned}")

    sweep = None
    if args.tau_sweep:
        log("overlap sweep: 64 to 2048 wavefronts at 1/16 of the serial step")
        sweep = tau_sweep(p, dev_arrays, fstar, stream)
    del dev_arrays
    racy = None if args.skip_racy else racy_leg(dev, stream)
    batched = None
    if not args.skip_batched:
        batched = batched_leg(args, dev, stream)
        # kernel throughput with every instance active (3 launches after 1)
        batched["throughput_all_active"] = batched_throughput(argparse.Namespace(steps=3, warmup=1), dev, stream)
    others, p4 = None, None
    if not args.skip_configs:
        others = {"config1": config1_leg(stream), "config2_plain_values": config2_plain_values_leg(dev, stream)}
        log(f"config1: {others['config1']}")
        others["config3"] = config3_leg(dev, stream)
        import datagen as _dg
        t = time.time()
        p4 = _dg.config4()
        log(f"generated config4 n={p4.n} d={p4.d} nnz={p4.nnz} in {time.time() - t:.1f}s")
        others["config4"] = config4_leg(dev, stream, p4)
        torch.cuda.empty_cache()

    # ---- CPU oracle on bounded samples -------------------------------------------
    cpu = None
    if not args.skip_cpu:
        legs = cpu_legs(args, p, p4)
        cpu = dict(legs["config2"])
        cpu["host_cpu"] = host_cpu_model()
        cpu["host_cpus"] = os.cpu_count()
        cpu["other_workloads"] = {k: v for k, v in legs.items() if k != "config2"}

    out = {
        "metric": METRIC,
        "value": ups,
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": total_ms / args.steps,
        "ms_per_step_median": sorted(launch_ms)[len(launch_ms) // 2],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded RCV1-shaped stand-in; the paper's datasets are not available)",
        "config": {"workload": "config2: plain FP64 async ASAGA, L2 logistic, lambda=1/n, CSR 700000 x 47000, "
                               "Poisson(75) Zipf(1.1) columns, TF-IDF-like values, rows L2-normalised",
                   "n": p.n, "d": p.d, "nnz": p.nnz, "epochs_per_step": 1, "waves": info.waves,
                   "lanes_per_sample": info.lanes_per_sample, "hot_columns": info.hot_columns,
                   "flush_every": info.flush_every, "threads_per_block": info.threads_per_block,
                   "gamma": info.gamma, "gamma_over_serial_rule": info.gamma * 3.0 * info.L},
        "hbm_gbps_algorithmic": achieved_gbps,
        "roofline": {"bound": "hbm", "achieved": achieved_gbps, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": achieved_gbps / HBM_PEAK_GBPS, "traffic": traffic,
                     "kernel": "k_update (async, FP64)", "bytes_per_update": bytes_per_update,
                     "launch_ms": avg_launch_s * 1e3,
                     # the counters' bytes (beyond L2, some served by the Infinity
                     # Cache) per second at this run's launch time
                     "traffic_gbps": traffic / avg_launch_s / 1e9 if traffic else None,
                     "traffic_frac": traffic / avg_launch_s / 1e9 / HBM_PEAK_GBPS if traffic else None,
                     "memory_side_requests": requests, "request_ceiling": ceiling},
        "time_to_1e-9": tta,
        "time_to_1e-9_autotuned": tta_tuned,
        "time_to_1e-9_svrg": tta_svrg,
        "autotune": tune,
        "batched": batched,
        "tau_sweep": sweep,
        "atomic_vs_racy": racy,
        "other_workloads": others,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
