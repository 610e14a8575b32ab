"""Writes bench_oracle.json: FP64 oracle results for the benchmark's
workloads, against which bench.py states the error of each timed
reduced-precision result.

Calls only the oracle (oracle/) and the seeded input generators
(paper_2306_06581_amd/workloads.py, which hold none of the method's
arithmetic).  Every value is the oracle's, run to the same tolerance as the
benchmark (residual <= 1e-6, Alg. 1/2 stop test as read in the oracle).

    python tests/golden/make_bench_oracle.py [--workers N] [--only KEY]

Takes about three minutes on 8 cores.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import sparsink_oracle as O  # noqa: E402
from paper_2306_06581_amd import workloads as W  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "bench_oracle.json")


def workloads():
    """key -> (problem, log_domain); keys match bench.py's.  The OT workload at
    n = m = 16384, d = 10 with s in {4, 8, 16} n ln n: the oracle builds each
    whole sketch (2.7e8 pairs) in about a minute on 8 cores."""
    out = {}
    for f in (4.0, 8.0, 16.0):
        out[f"ot_t5_d10_n16384_s{f:g}"] = (W.ot_t5_d10(16384, seed=0, s_factor=f), False)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workers", type=int, default=os.cpu_count() or 1)
    ap.add_argument("--only", default=None)
    args = ap.parse_args()
    res = json.load(open(OUT)) if os.path.exists(OUT) else {}
    for key, (p, log_domain) in workloads().items():
        if args.only and key != args.only:
            continue
        t0 = time.perf_counter()
        opt = O.Options(eps=p.eps, s=p.s, lam=p.lam, seed=p.seed, tol=1e-6, max_iter=5000,
                        log_domain=log_domain)
        r = O.spar_sink(p.x, p.y, p.a, p.b, opt, workers=args.workers)
        res[key] = {
            "workload": p.name, "n": p.n, "m": p.m, "eps": p.eps,
            "lambda": None if not math.isfinite(p.lam) else p.lam, "s": p.s,
            "log_domain": log_domain, "tol": 1e-6,
            "estimate": r.estimate.estimate, "sparse_objective": r.estimate.sparse_objective,
            "iters": r.sinkhorn.iters, "err": r.sinkhorn.err, "converged": r.sinkhorn.converged,
            "nnz": r.nnz, "empty_rows": r.empty_rows, "empty_cols": r.empty_cols,
        }
        print(f"{key}: estimate {r.estimate.estimate:.15g} iters {r.sinkhorn.iters} "
              f"nnz {r.nnz} ({time.perf_counter() - t0:.0f} s)", flush=True)
        with open(OUT, "w") as f:
            json.dump(res, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main()
