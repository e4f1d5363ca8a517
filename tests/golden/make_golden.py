"""Writes tests/golden/fstar.json: the optimum f* of each full-size workload,
computed by the CPU oracle only (never by the HIP library).

    python tests/golden/make_golden.py [config1 config2 config3 config4]

* config1 (2,000 x 500 logistic): damped Newton on the dense objective;
  f* = oracle objective at the Newton point.
* config3 (581,000 x 54 least squares): ridge closed form
  (A'A/n + lambda I)^-1 A'b/n by Cholesky; f* = oracle objective there.
* config2, config4 (large logistic): the oracle's own serial Sparse SAGA run
  until the strong-convexity certificate ||grad f||^2/(2 lambda) <= 1e-12 f
  holds; f* lies in [f_lower, f_upper].

Each entry records the sha256 digest of the generated instance, so a test
can check that it regenerated the same problem.
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


def main(names):
    data = json.load(open(OUT)) if os.path.exists(OUT) else {}
    for name in names:
        t = time.time()
        p = datagen.by_name(name)
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
    main(sys.argv[1:] or ["config1", "config3", "config2", "config4"])
