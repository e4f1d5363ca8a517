"""Writes tests/golden/fstar.json: the optimum f* of each full-size workload,
computed by the CPU oracle only (never by the HIP library).

    python tests/golden/make_golden.py [config1 config2 config3 config4 config5]

* config1 (2,000 x 500 logistic): damped Newton on the dense objective;
  f* = oracle objective at the Newton point.
* config3 (581,000 x 54 least squares): ridge closed form
  (A'A/n + lambda I)^-1 A'b/n by Cholesky; f* = oracle objective there.
* config2, config4 (large logistic): the oracle's own serial Sparse SAGA run
  until the strong-convexity certificate ||grad f||^2/(2 lambda) <= 1e-12 f
  holds; f* lies in [f_lower, f_upper].

* config2_20000x2000 (the RCV1-shaped recipe at 20,000 x 2,000): the same
  certificate, for the benchmark's comparison of atomic and racy updates.
* config2_plain_lognormal (config 2 with lognormal values and no idf
  factor, the other reading of its values): the same certificate.

* config5 (160 lambda x fold instances over the bfloat16 config-2 matrix):
  the same certificate per instance, to 1e-11, one instance per worker
  process.

Each entry records the sha256 digest of the generated instance, so a test
can check that it regenerated the same problem.

    python tests/golden/make_golden.py tta [config1 ... config5]

adds to each entry the oracle's own epochs (serial step rule, seed 0,
checked after every epoch) to 1e-9 relative suboptimality against the
stored f*, with the host seconds they took ("oracle_tta"; per instance for
config5).
"""
from __future__ import annotations

import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import datagen  # noqa: E402
import oracle  # noqa: E402

OUT = os.path.join(HERE, "fstar.json")


def entry_newton(p):
    sv = oracle.SparseSaga(p)
    x = oracle.logistic_newton(p)
    f = sv.objective(x)
    g = sv.gradient(x)
    return {"f_star": f, "f_lower": f - float(g @ g) / (2 * p.lam), "f_upper": f, "method": "damped Newton",
            "grad_norm": float(np.linalg.norm(g))}


def entry_ridge(p):
    sv = oracle.SparseSaga(p)
    x = oracle.ridge_solution_csr(p)
    f = sv.objective(x)
    g = sv.gradient(x)
    return {"f_star": f, "f_lower": f - float(g @ g) / (2 * p.lam), "f_upper": f, "method": "ridge closed form",
            "grad_norm": float(np.linalg.norm(g))}


def entry_certificate(p, epochs_per_check=5):
    r = oracle.certified_fstar(p, tol=1e-12, check_every=epochs_per_check, max_epochs=3000,
                               log=lambda s: print("   ", s, flush=True))
    return {"f_star": r["f_lower"], "f_lower": r["f_lower"], "f_upper": r["f_upper"],
            "method": "oracle Sparse SAGA + strong-convexity certificate", "epochs": r["epochs"],
            "converged": bool(r["converged"])}


_BATCH = None


def _batch_digest(B) -> str:
    import hashlib
    h = hashlib.sha256(B.problem.digest().encode())
    for a in (B.row_fold, B.inst_fold, B.inst_lambda):
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def _config5_instance(k):
    t = time.time()
    q = _BATCH.instance(k)
    r = oracle.certified_fstar(q, tol=1e-11, check_every=5, max_epochs=600)
    e = {"k": int(k), "fold": int(_BATCH.inst_fold[k]), "lambda": float(_BATCH.inst_lambda[k]), "m": int(q.n),
         "f_star": r["f_lower"], "f_lower": r["f_lower"], "f_upper": r["f_upper"], "epochs": r["epochs"],
         "converged": bool(r["converged"]), "seconds": round(time.time() - t, 1)}
    print(f"  instance {k}: {e}", flush=True)
    return e


def entry_config5(workers):
    import multiprocessing as mp
    global _BATCH
    _BATCH = datagen.config5()
    order = sorted(range(_BATCH.n_inst), key=lambda k: _BATCH.inst_lambda[k])
    with mp.get_context("fork").Pool(workers) as pool:
        inst = sorted(pool.imap_unordered(_config5_instance, order), key=lambda e: e["k"])
    return {"method": "oracle Sparse SAGA + strong-convexity certificate per instance", "instances": inst,
            "converged": all(e["converged"] for e in inst), "digest": _batch_digest(_BATCH),
            "n": _BATCH.problem.n, "d": _BATCH.problem.d, "nnz": _BATCH.problem.nnz, "n_inst": _BATCH.n_inst}


def oracle_epochs_to(p, fstar, target=1e-9, max_epochs=3000):
    """The oracle's own serial Sparse SAGA (serial step rule, seed 0) from
    x = 0: epochs until (f - f*)/f* <= target, checked after every epoch,
    and the host seconds its updates took (the checks not counted)."""
    sv = oracle.SparseSaga(p)
    secs, ep, rel = 0.0, 0, float("inf")
    while ep < max_epochs:
        t = time.perf_counter()
        sv.epochs(1)
        secs += time.perf_counter() - t
        ep += 1
        rel = (sv.objective() - fstar) / fstar
        if rel <= target:
            break
    return {"target": target, "epochs": ep, "reached": bool(rel <= target), "final_rel": rel,
            "host_seconds": round(secs, 2), "seconds_per_epoch": secs / ep}


def _config5_tta(k):
    q = _BATCH.instance(k)
    r = oracle_epochs_to(q, _FSTAR5[k], max_epochs=600)
    print(f"  instance {k}: {r}", flush=True)
    return k, r


_FSTAR5 = None


def add_tta(names, workers):
    """Adds the oracle's own epochs to 1e-9 ("oracle_tta") to stored entries."""
    import multiprocessing as mp
    global _BATCH, _FSTAR5
    data = json.load(open(OUT))
    for name in names:
        t = time.time()
        if name == "config5":
            _BATCH = datagen.config5()
            if data[name]["digest"] != _batch_digest(_BATCH):
                raise SystemExit("config5 differs from the stored batch")
            _FSTAR5 = {e["k"]: e["f_lower"] for e in data[name]["instances"]}
            order = sorted(range(_BATCH.n_inst), key=lambda k: _BATCH.inst_lambda[k])
            with mp.get_context("fork").Pool(workers) as pool:
                res = dict(pool.imap_unordered(_config5_tta, order))
            for e in data[name]["instances"]:
                e["oracle_tta"] = res[e["k"]]
        else:
            p = SCALED[name]() if name in SCALED else datagen.by_name(name)
            if data[name]["digest"] != p.digest():
                raise SystemExit(f"{name} differs from the stored instance")
            data[name]["oracle_tta"] = oracle_epochs_to(p, data[name]["f_lower"])
            print(f"{name}: {data[name]['oracle_tta']}", flush=True)
        print(f"{name}: oracle epochs to 1e-9 in {time.time() - t:.1f} s", flush=True)
        json.dump(data, open(OUT, "w"), indent=1, sort_keys=True)


# scaled-down RCV1-shaped instances the benchmark also runs (the Appendix G
# comparison of atomic and racy updates)
SCALED = {"config2_20000x2000": lambda: datagen.config2(n=20_000, d=2000),
          "config2_plain_lognormal": lambda: datagen.config2(idf=False)}


def main(names):
    data = json.load(open(OUT)) if os.path.exists(OUT) else {}
    for name in names:
        t = time.time()
        if name == "config5":
            e = entry_config5(int(os.environ.get("GOLDEN_WORKERS", "8")))
            e["seconds"] = round(time.time() - t, 1)
            print(f"config5: converged {e['converged']} in {e['seconds']} s", flush=True)
            data = json.load(open(OUT)) if os.path.exists(OUT) else {}
            data[name] = e
            json.dump(data, open(OUT, "w"), indent=1, sort_keys=True)
            continue
        p = SCALED[name]() if name in SCALED else datagen.by_name(name)
        print(f"{name}: generated n={p.n} d={p.d} nnz={p.nnz} in {time.time() - t:.1f}s", flush=True)
        if name == "config1":
            e = entry_newton(p)
        elif name == "config3":
            e = entry_ridge(p)
        else:
            e = entry_certificate(p)
        e.update({"digest": p.digest(), "n": p.n, "d": p.d, "nnz": p.nnz, "lambda": p.lam,
                  "seconds": round(time.time() - t, 1)})
        print(f"{name}: {e}", flush=True)
        data[name] = e
        json.dump(data, open(OUT, "w"), indent=1, sort_keys=True)


if __name__ == "__main__":
    if sys.argv[1:2] == ["tta"]:
        add_tta(sys.argv[2:] or ["config1", "config3", "config2", "config4", "config5"],
                int(os.environ.get("GOLDEN_WORKERS", "7")))
    else:
        main(sys.argv[1:] or ["config1", "config3", "config2", "config4"])
