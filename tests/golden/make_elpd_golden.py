"""Write the oracle's per-fold LogS estimates used by the device-vs-oracle
Monte Carlo agreement tests (tests/test_gpu_elpd_agreement.py).

Each file elpd_<workload>_folds<k0>-<k1>.json holds, for the first folds of a
workload, the oracle's full-length run (all warm-up and sampling transitions
of the workload, same seeds and chain ids as the full run): per-fold elpd_k
(eq cv-score), its Monte Carlo standard error (batch means, eq mc-var) and
R-hat.  Only the oracle (oracle/) and the seeded input generator run here.

Usage (repository root):  python tests/golden/make_elpd_golden.py [c4|c2|c5 ...]
The full set takes about two hours of numpy on 8 cores.
"""
from __future__ import annotations

import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

# (workload, first fold, last fold + 1): C2 in full; the first 25 folds of the
# Poisson GLM (200 chains); the first 20 blocks of the blocked logistic GLM
# (80 chains; every chain still sweeps all 100000 rows each gradient)
SUBSETS = {"c2": (0, 50), "c4": (0, 25), "c5": (0, 20)}


def golden_path(name: str) -> str:
    k0, k1 = SUBSETS[name]
    return os.path.join(HERE, f"elpd_{name}_folds{k0}-{k1}.json")


def make(name: str) -> dict:
    from oracle import diagnostics, sampler
    from paper_2310_07002_amd import workloads as W
    w = W.make(name)
    k0, k1 = SUBSETS[name]
    sub = W.fold_subset(w, k0, k1)
    t0 = time.perf_counter()
    run = sampler.start(sub)
    done = 0
    while done < sub.n_iter:
        step = min(100, sub.n_iter - done)
        sampler.advance(sub, run, step)
        done += step
        print(f"{name}: {done}/{sub.n_iter} transitions, {time.perf_counter() - t0:.0f} s", flush=True)
    d = diagnostics.from_accumulators(run.acc, sub.K, sub.L, sub.batch_size)
    return {
        "workload": name, "folds": [k0, k1], "L": sub.L, "chains": sub.C,
        "n_warmup": sub.n_warmup, "n_samples": sub.n_samples, "batch_size": sub.batch_size,
        "n_leapfrog": sub.n_leapfrog, "step_size": sub.step_size, "seed": int(sub.seed),
        "elpd_fold": [float(x) for x in d["elpd_fold"]],
        "mcse_fold": [float(x) for x in d["mcse_fold"]],
        "rhat_fold": [float(x) for x in d["rhat_fold"]],
        "elpd": d["elpd"], "mcse": d["mcse"], "accept_rate": d["accept_rate"],
        "n_draws": int(d["n_draws"]),
        "writer": "tests/golden/make_elpd_golden.py (fp64 numpy oracle)",
        "seconds": time.perf_counter() - t0,
    }


def main(names):
    for name in names:
        out = make(name)
        with open(golden_path(name), "w") as f:
            json.dump(out, f, indent=1)
            f.write("\n")
        print(f"wrote {golden_path(name)}: elpd {out['elpd']:.4f} +- {out['mcse']:.4f}", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or ["c4", "c2", "c5"])
