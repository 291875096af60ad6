"""Throughput of the PCV hot path on one MI355X.

A step is one HMC transition of every fold x chain state: momentum refresh,
S fused masked value/gradient evaluations with their leapfrog updates,
Metropolis test, log predictive and online accumulation.  Inputs are resident
in HBM before timing starts.

Metric: gradient evaluations per second over all fold x chain states
(C * S * steps / wall).  Default workload: blocked CV of a logistic GLM,
n=100000, p=128, 10000 folds x 4 chains (40000 chains), S=8, bf16 hi+lo split
MFMA contractions (BF16X3), synthetic data.

Also reported on the same JSON line:
  roofline      the gradient kernel's algorithmic flops per launch (4 n p C)
                over its mean launch time from HIP events on the library's
                stream during the timed region, against the dense bf16 peak;
                HBM traffic from committed rocprofv3 counter summaries if any;
                on matrix-core workloads also the sustained rate of the same
                bf16 MFMA on random and on constant operands (mfma_ceiling)
  cpu_baseline  the fp64 CPU oracle on a bounded sample of the same workload
  parity_vs_oracle  the device's log density and gradient against the oracle
                at the starting positions of that sample's chains
  plain_fp64    the unfused fp64 library path (DGEMM + materialised eta) on
                the same workload, a few steps, and the speedup over it
Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c5]
       [--precision bf16x3|bf16x5|fp64|fp32|fp64u] [--no-cpu-baseline]
       [--no-plain-fp64] [--no-time-to-rhat] [--no-autotune] [--no-mfma-ceiling]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"bf16": 2.5e15, "fp32": 157.3e12, "fp64": 78.6e12}
PREC_NAMES = {"fp64": 0, "fp32": 1, "bf16x3": 2, "bf16x5": 3, "fp64u": 4}
PREC_DTYPE = {"fp64": "f64", "fp32": "f32", "bf16x3": "bf16", "bf16x5": "bf16", "fp64u": "f64"}
PREC_PEAK = {"fp64": "fp64", "fp32": "fp32", "bf16x3": "bf16", "bf16x5": "bf16", "fp64u": "fp64"}
DEFAULT_PREC = {"c1": "fp64", "c2": "fp32", "c3": "fp64", "c4": "bf16x3", "c5": "bf16x3"}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def workload_label(w, prec):
    return (f"{w.name}: n={w.n} p={w.p} d={w.d} K={w.K} L={w.L} C={w.C} S={w.n_leapfrog} "
            f"eps={w.step_size} precision={prec}")


def baseline_folds(w) -> int:
    """Folds of the bounded CPU sample (the first ones of the workload, so the
    same chains and random streams): every fold of the small workloads, 25
    folds x 8 chains of the Poisson GLM and 50 folds x 4 chains of the
    blocked logistic GLM."""
    if w.n * w.p <= 1e6:
        return w.K
    return min(w.K, max(1, 200 // w.L))


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_parity(w, theta, lp_dev, g_dev):
    """Error of the device's log density and gradient against the fp64 oracle
    at the same positions, on the chains of the CPU sample."""
    from oracle import folds, model
    from paper_2310_07002_amd import workloads as W
    sub = W.fold_subset(w, 0, baseline_folds(w))
    roles = folds.roles_of(sub)
    foc = np.arange(sub.C) // sub.L
    th = theta[:sub.C]
    lp_o = model.log_density(sub, th, roles, foc)
    g_o = model.grad_log_density(sub, th, roles, foc)
    rel_v = np.abs(lp_dev[:sub.C] - lp_o) / np.abs(lp_o)
    rel_g = np.linalg.norm(g_dev[:sub.C] - g_o, axis=1) / np.linalg.norm(g_o, axis=1)
    return {"reference": "fp64 oracle", "chains": sub.C, "at": "the chains' starting positions",
            "logp_rel_max": float(rel_v.max()), "grad_normwise_rel_max": float(rel_g.max()),
            "grad_normwise_rel_median": float(np.median(rel_g))}


def cpu_baseline(w, budget_s=15.0, numpy_budget_s=8.0):
    """The oracle as it stands, on a bounded sample: the first folds of the
    same workload (same chains, same random streams), from the chains'
    starts, as many transitions as fit in the time budget.  The value is the
    plain C oracle (fp64 loops, chains spread over the host's threads with
    OpenMP); the numpy oracle (BLAS for the contractions) is timed beside it
    on the same sample."""
    from oracle import c_oracle, sampler
    from paper_2310_07002_amd import workloads as W
    host = os.cpu_count() or 1
    threads = max(1, min(host, int(os.environ.get("OMP_NUM_THREADS") or host)))
    k_sub = baseline_folds(w)
    sub = W.fold_subset(w, 0, k_sub)

    cap = w.n_iter                   # at most the whole run (warm-up included)

    def timed(step, budget):
        t0 = time.perf_counter()
        iters = 0
        while True:
            step()
            iters += 1
            if time.perf_counter() - t0 > budget or iters >= cap:
                return iters, time.perf_counter() - t0

    try:
        run_c = c_oracle.Run(sub, threads)
    except (OSError, RuntimeError) as e:      # no C compiler or library on this host
        log(f"bench: C oracle unavailable ({e}); timing the numpy oracle only")
        run_c = None
    if run_c is not None:
        it_c, dt_c = timed(lambda: run_c.advance(1), budget_s)
    blas = None
    try:
        from threadpoolctl import threadpool_info
        blas = max((i.get("num_threads") or 0) for i in threadpool_info()) or None
    except Exception:
        pass
    run_np = sampler.start(sub)
    it_np, dt_np = timed(lambda: sampler.advance(sub, run_np, 1), numpy_budget_s if run_c is not None else budget_s)
    per_iter = sub.C * sub.n_leapfrog
    numpy_leg = {"value": per_iter * it_np / dt_np, "transitions": it_np, "seconds": dt_np, "blas_threads": blas}
    if run_c is None:
        return {"value": numpy_leg["value"], "unit": "gradient evals/s", "cores": blas or host, "kind": "oracle",
                "cpu": cpu_model(), "host_cpus": host,
                "sample": f"first {k_sub} folds x {sub.L} chains ({sub.C} chains) of the same workload, "
                          f"{it_np} transitions of {sub.n_leapfrog} leapfrog steps from the chains' starts, "
                          f"{dt_np:.1f} s; fp64 numpy oracle, BLAS on {blas or host} threads",
                "numpy_oracle": numpy_leg}
    return {"value": per_iter * it_c / dt_c, "unit": "gradient evals/s", "cores": threads,
            "kind": "oracle", "cpu": cpu_model(), "host_cpus": host,
            "sample": f"first {k_sub} folds x {sub.L} chains ({sub.C} chains) of the same workload, "
                      f"{it_c} transitions of {sub.n_leapfrog} leapfrog steps from the chains' starts, "
                      f"{dt_c:.1f} s; plain C fp64 oracle (oracle/c), chains over {threads} OpenMP threads",
            "numpy_oracle": numpy_leg}


def current_config(s):
    """The context's launch shape, or None on the plain fp64 path (which has none)."""
    from paper_2310_07002_amd import binding
    try:
        return s.launch_config()
    except binding.PcvError:
        return None


def traffic_from_profiles(w, prec, kernel_name, config):
    """HBM bytes per launch of the gradient kernel from the committed counter
    summary, or None if there is none, if it holds no counters for launch
    shape `config`, or if the kernel's sources (its .hip file and the shared
    device header) changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"traffic_{w.name}_{prec}.json")
    csrc = os.path.join(ROOT, "paper_2310_07002_amd", "csrc")
    srcs = [os.path.join(csrc, "k_mfma.hip" if kernel_name.startswith("k_mfma") else "k_valu.hip"),
            os.path.join(csrc, "pcv_internal.h")]
    if not os.path.exists(path) or not all(os.path.exists(x) for x in srcs):
        return None
    try:
        with open(path) as f:
            t = json.load(f)
        hh = hashlib.sha256()
        for x in srcs:
            with open(x, "rb") as f:
                hh.update(f.read())
        h = hh.hexdigest()[:16]
        if t.get("kernel_source_sha256_16") != h:
            return None
        if t.get("launch_config") == config:
            return t.get("bytes_per_launch")
        return t.get("other_launch_configs", {}).get(str(config), {}).get("bytes_per_launch")
    except Exception:
        return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c5")
    ap.add_argument("--precision", default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain-fp64", action="store_true")
    ap.add_argument("--plain-steps", type=int, default=2)
    ap.add_argument("--no-time-to-rhat", action="store_true",
                    help="skip the second metric (wall time from init to R-hat_max < 1.01 at a batch end)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the analytic launch shape instead of timing candidates first")
    ap.add_argument("--launch-config", type=int, default=None,
                    help="apply this launch shape (pcv_autotune's encoding) instead of tuning, "
                         "e.g. to profile the shape a full run chose")
    ap.add_argument("--no-mfma-ceiling", action="store_true",
                    help="skip timing the bf16 MFMA calibration kernel (matrix-core workloads)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one 512 MiB device-to-device copy first (reference kernel for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported "
              "(the path would shard whole folds across GPUs, see the design notes)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2310_07002_amd import binding, workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.calibrate_copy:
        src = torch.ones(512 * 2 ** 20 // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    prec = args.precision or DEFAULT_PREC[args.workload]
    log(f"bench: generating workload {args.workload}")
    w = W.make(args.workload)
    stream = torch.cuda.current_stream()
    log(f"bench: init {workload_label(w, prec)}")
    # the throughput leg counts only the untimed warm-up steps as warm-up, so
    # every timed transition is a sampling transition: log predictive and
    # online accumulators run inside the timed region
    import dataclasses
    wt = dataclasses.replace(w, n_warmup=args.warmup)
    s = binding.PCV.from_workload(wt, precision=PREC_NAMES[prec], stream=stream)
    tune = None
    if args.launch_config is not None:
        s.set_launch_config(args.launch_config)
        log(f"bench: launch config {args.launch_config} applied")
    elif not args.no_autotune and prec != "fp64u":
        torch.cuda.synchronize()
        ta = time.perf_counter()
        tune = s.autotune()
        tune["seconds"] = time.perf_counter() - ta
        kname = s.timing_read(reset=True)[2]
        tune["knob"] = ("waves per workgroup" if "fused" in kname else
                        ("256 x kernel shape (0: 16x16x32, 1: 32x32x16, 2: 32x32x16 free schedule, "
                         "3: 16x16x32 with 16 chains per wave) + row splits") if "mfma" in kname
                        else "1024 x waves per workgroup + row splits")
        log(f"bench: autotune chose {tune['knob']} = {tune['config']} ({tune['ms']:.4f} ms) in {tune['seconds']:.2f} s")
    s.step(args.warmup)
    torch.cuda.synchronize()
    s.timing_read(reset=True)
    s.timing_enable(True)           # HIP events around every hot-kernel launch (eager launches)
    log(f"bench: timing {args.steps} transitions")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(args.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    s.timing_enable(False)
    k_ms, k_n, k_name = s.timing_read(reset=True)
    wall = t1 - t0
    k_steps = args.steps
    # the same transitions replayed as the captured graph (the production
    # path of the split paths; the fused VALU path is one launch either way)
    torch.cuda.synchronize()
    g0 = time.perf_counter()
    s.step(args.steps)
    torch.cuda.synchronize()
    g_wall = time.perf_counter() - g0
    grads = w.C * w.n_leapfrog * args.steps
    value = grads / wall
    ms_per_step = wall / args.steps * 1e3
    log(f"bench: {value:.4e} gradient evals/s, {ms_per_step:.3f} ms/transition, kernel {k_name}: "
        f"{k_n} launches, {k_ms / max(k_n, 1):.4f} ms each")

    # roofline of the gradient kernel
    flops_per_launch = 4.0 * w.n * w.p * w.C
    if prec in ("fp64", "fp32"):
        # the fused transition kernel runs many transitions per launch
        grads_per_launch = w.C * w.n_leapfrog * k_steps / max(k_n, 1)
        flops_per_launch = 4.0 * w.n * w.p * grads_per_launch
    avg_s = k_ms / max(k_n, 1) / 1e3
    achieved = flops_per_launch / avg_s / 1e12 if avg_s > 0 else None
    peak = PEAK[PREC_PEAK[prec]] / 1e12
    roofline = {"bound": "mfma" if prec.startswith("bf16") else "alu",
                "kernel": k_name, "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                "frac": (achieved / peak) if achieved else None,
                "traffic": traffic_from_profiles(w, prec, k_name, current_config(s)),
                "alg_flops_per_launch": flops_per_launch, "mean_launch_ms": avg_s * 1e3,
                "launches": k_n}
    if prec.startswith("bf16"):
        # issued bf16 products per algorithmic product: (forward terms + 3 adjoint terms) / 2
        ratio = (3 + 3) / 2 if prec == "bf16x3" else (5 + 3) / 2
        roofline["issued_mfma_frac"] = achieved * ratio / peak if achieved else None
        if not args.no_mfma_ceiling:
            # the sustained rate of the same bf16 MFMA on random and on
            # constant operands (the part lowers its clock to hold its power
            # limit, more so the more the operand bits switch)
            rnd = binding.pcv_calib_mfma(1, 40)
            cst = binding.pcv_calib_mfma(0, 40)
            roofline["mfma_ceiling"] = {
                "kernel": "k_calib_mfma (v_mfma_f32_32x32x16_bf16, 2 waves per SIMD, operands from LDS)",
                "random_bf16_tflops": rnd, "constant_operands_tflops": cst,
                "issued_frac_of_random_ceiling": achieved * ratio / rnd if achieved else None}
            log(f"bench: bf16 MFMA ceiling {rnd:.0f} TFLOP/s on random operands, {cst:.0f} on constant ones; "
                f"the gradient kernel issues {achieved * ratio:.0f}")

    acc_check = s.diagnostics()
    assert acc_check["n_draws"] == 2 * args.steps, "timed transitions must be post-warm-up"
    line = {"metric": "gradient evals/sec over all fold×chain states", "value": value,
            "unit": "gradient evals/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": PREC_DTYPE[prec], "precision_mode": prec,
            "data": "synthetic (seeded; shaped like the paper's CV workloads, no datasets)",
            "config": {"workload": workload_label(w, prec), "folds": w.K, "chains_per_fold": w.L,
                       "chains": w.C, "leapfrog_steps": w.n_leapfrog, "parallelism": "single GPU"},
            "roofline": roofline,
            "timed_transitions": "post-warm-up (log predictive and online accumulators included)",
            "graph_replay": {"ms_per_step": g_wall / args.steps * 1e3,
                             "value": w.C * w.n_leapfrog * args.steps / g_wall}}
    if tune is not None:
        line["autotune"] = tune

    dev_eval = None
    if not args.no_cpu_baseline:
        # log pi and its gradient at the starting positions, checked against
        # the oracle on the CPU sample's chains in the baseline leg
        lp_d, g_d = s.logdensity_grad(torch.tensor(w.init_pos, device="cuda"))
        torch.cuda.synchronize()
        n_keep = baseline_folds(w) * w.L
        dev_eval = (lp_d[:n_keep].cpu().numpy(), g_d[:n_keep].cpu().numpy())
        del lp_d, g_d
    s.close()
    del s

    if not args.no_plain_fp64 and prec != "fp64u":
        log("bench: plain fp64 path (library DGEMM, eta materialised)")
        try:
            b = binding.PCV.from_workload(w, precision=PREC_NAMES["fp64u"], stream=stream)
            b.step(1)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            b.step(args.plain_steps)
            torch.cuda.synchronize()
            dtp = time.perf_counter() - t0
            pv = w.C * w.n_leapfrog * args.plain_steps / dtp
            line["plain_fp64"] = {"value": pv, "ms_per_step": dtp / args.plain_steps * 1e3,
                                  "steps": args.plain_steps, "speedup": value / pv}
            b.close()
            del b
        except Exception as e:  # report, never hide
            line["plain_fp64"] = {"error": str(e)}

    if not args.no_time_to_rhat:
        log("bench: full run for wall time to Rhat_max < 1.01")
        r = binding.PCV.from_workload(w, precision=PREC_NAMES[prec], stream=stream)
        if args.launch_config is not None:
            r.set_launch_config(args.launch_config)
        elif tune is not None:
            r.autotune()              # tuning is reported separately, outside the clock
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r.step(w.n_warmup)
        reached = None
        done = 0
        per_batch = w.batch_size
        while done < w.n_samples:
            r.step(per_batch)
            done += per_batch
            if done >= 2 * per_batch:
                dd = r.diagnostics()
                if dd["rhat_max"] < 1.01 and reached is None:
                    reached = {"seconds": time.perf_counter() - t0, "draws": done, "elpd": dd["elpd"],
                               "mcse": dd["mcse"], "rhat_max": dd["rhat_max"]}
                    break
        torch.cuda.synchronize()
        dd = r.diagnostics()
        line["time_to_rhat_max_1.01"] = reached or {"reached": False, "seconds": time.perf_counter() - t0,
                                                    "final_rhat_max": dd["rhat_max"], "elpd": dd["elpd"],
                                                    "mcse": dd["mcse"], "draws": dd["n_draws"]}
        if reached is None:
            # Rhat_max of many folds is judged against its block-shuffle
            # benchmark (Section 4.2): R replicates of Rhat_max from chains
            # rebuilt of blocks drawn across each fold's chains
            rep = np.sort(r.shuffle_benchmark(100, seed=w.seed + 7))
            q = {f"q{int(x * 100):02d}": float(np.quantile(rep, x)) for x in (0.05, 0.5, 0.95)}
            line["time_to_rhat_max_1.01"]["shuffle_benchmark"] = {
                "replicates": 100, **q, "max": float(rep[-1]),
                "final_rhat_max_quantile": float(np.mean(rep <= dd["rhat_max"]))}
        r.close()

    if not args.no_cpu_baseline:
        log("bench: cpu baseline (oracle, bounded sample)")
        line["cpu_baseline"] = cpu_baseline(w)
        line["parity_vs_oracle"] = oracle_parity(w, w.init_pos, *dev_eval)
    # the same number of transitions at the other paths' measured rates
    tr = line.get("time_to_rhat_max_1.01")
    if tr and tr.get("draws") is not None and tr.get("reached", True):
        n_tr = w.n_warmup + tr["draws"]
        ext = {"transitions": n_tr}
        pf = line.get("plain_fp64", {})
        if "ms_per_step" in pf:
            ext["plain_fp64_seconds"] = pf["ms_per_step"] * n_tr / 1e3
        cb = line.get("cpu_baseline")
        if cb:
            ext["oracle_seconds"] = w.C * w.n_leapfrog * n_tr / cb["value"]
        tr["extrapolated_same_transitions"] = ext
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
