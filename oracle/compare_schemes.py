"""Dense, lagged and sparse SAGA on the CPU (the comparison of Appendix F):
passes over the data and seconds to a relative suboptimality, one thread,
FP64, the same sample stream and step for all three.

    python oracle/compare_schemes.py [--target 1e-9] [--epochs 80]

Workloads: a 20,000-row slice of the RCV1-shaped instance (sparse) and a
20,000-row slice of the Covtype-shaped one (dense columns).  f* is the
oracle's certified optimum of each slice.  CPU only; part of the oracle's
test infrastructure.
"""
from __future__ import annotations

import argparse
import os
import sys
import time

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

import datagen  # noqa: E402
import oracle  # noqa: E402


def run(scheme, p, fstar, target, max_epochs):
    sv = scheme(p, seed=0)
    secs, rel = 0.0, float("inf")
    for e in range(1, max_epochs + 1):
        t = time.perf_counter()
        sv.epochs(1)
        secs += time.perf_counter() - t
        rel = (sv.objective() - fstar) / fstar
        if rel <= target:
            return e, secs, rel
    return None, secs, rel


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--target", type=float, default=1e-9)
    ap.add_argument("--epochs", type=int, default=80)
    args = ap.parse_args()
    workloads = [("RCV1-shaped slice (20,000 x 5,000, ~75 nnz/row)", datagen.config2(n=20_000, d=5000)),
                 ("Covtype-shaped slice (20,000 x 54, 12 nnz/row)", datagen.config3(n=20_000))]
    print(f"| workload | scheme | passes to {args.target:g} | seconds | seconds per pass |")
    print("|---|---|---|---|---|")
    for name, p in workloads:
        fstar = oracle.certified_fstar(p, tol=1e-12, check_every=10)["f_lower"]
        for label, scheme in (("dense", oracle.DenseSaga), ("lagged", oracle.LaggedSaga),
                              ("sparse", oracle.SparseSaga)):
            ep, secs, rel = run(scheme, p, fstar, args.target, args.epochs)
            per = secs / (ep if ep else args.epochs)
            print(f"| {name} | {label} | {ep if ep else f'> {args.epochs} (rel {rel:.1e})'} | {secs:.2f} | "
                  f"{per * 1e3:.1f} ms |", flush=True)


if __name__ == "__main__":
    main()
