"""Benchmark: Sinkhorn sweeps/s of the NFFT path vs the direct GPU path on one MI355X.

Workload (one GPU): star tree, K = 10 marginals, N = 100000 points each in d = 3,
points uniform in [-1/4, 1/4)^3, uniform-random normalised weights, eta = 0.05,
oversampled grid 128^3, window cutoff m = 6 (M = 32, tau = 1, eps_B = 1/8, p = 3).
A step is one Sinkhorn sweep (Algorithm 2): 18 Gaussian-kernel products plus the FP64
scaling updates and reductions.

Prints one JSON line.  `value` is NFFT sweeps/s with all inputs resident on the GPU.
Beside it: the direct O(N^2) GPU path on the same workload, the NFFT-vs-direct accuracy
of the scaling vectors (gauge fixed) after the same sweeps, the roofline of the
dominant kernel (HIP events around each launch), and the FP64 CPU oracle timed on a
bounded sample (a baseline only).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
PEAK_FP32_TFLOPS = 157.3


def gauge_fix(phi, mu):
    out = [np.array(p, dtype=np.float64) for p in phi]
    tot = 0.0
    for k in range(1, len(out)):
        g = float(np.sum(mu[k] * np.log(out[k])))
        out[k] = out[k] * np.exp(-g)
        tot += g
    out[0] = out[0] * np.exp(tot)
    return out


def step_work(step, info, inst, n_jobs_level):
    """Algorithmic flops and bytes of one launch of the sweep schedule."""
    d = info["d"]
    m = info["m"]
    taps = (2 * m) ** d
    L = info["box_len"][:d]
    M = info["M"]
    H, B = M + 1, 2 * M + 1
    N = inst.sizes[0]
    cells = int(np.prod(L))
    kind = step["kind"]
    jobs = n_jobs_level
    if kind == "spread":
        # per point: v (8 B), cell (4 B), frac (4d B); taps: 1 mul + 1 add each
        return {"flops": 2.0 * taps * N * jobs, "bytes": (12 + 4 * d) * N * jobs}
    if kind == "interp":
        return {"flops": 2.0 * taps * N * jobs, "bytes": (12 + 4 * d) * N * jobs + 4 * cells * jobs}
    if kind == "fold":
        return {"flops": 0.0, "bytes": 4.0 * cells * jobs * 2}
    if kind == "fft":
        fk = step["fft_kind"]
        if d == 3:
            sizes = {0: (4 * cells, 8 * H * L[0] * L[1]), 1: (8 * H * L[0] * L[1], 8 * H * B * L[0]),
                     2: (8 * H * B * L[0], 8 * L[0] * H * B), 3: (8 * L[0] * H * B, 8 * L[0] * L[1] * H),
                     4: (8 * L[0] * L[1] * H, 4 * cells)}
            rd, wr = sizes[fk]
            n = info["n"]
            lines = {0: L[0] * L[1] / 2, 1: H * L[0], 2: H * B, 3: L[0] * H, 4: L[0] * L[1] / 2}[fk]
            fl = lines * 5.0 * n * np.log2(n) * (2 if fk == 2 else 1)
            return {"flops": fl * jobs, "bytes": (rd + wr) * jobs}
    return {"flops": 0.0, "bytes": 0.0}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--N", type=int, default=100_000)
    ap.add_argument("--direct-steps", type=int, default=10)
    ap.add_argument("--acc-sweeps", type=int, default=20)
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--profile-sweeps", type=int, default=5)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    from paper_2208_03120_amd import mot, workloads as W

    inst = W.star_nfft(seed=2, N=args.N)
    fs = mot.fastsum_params(M=32, n=128, m=6, p=3, tau=1.0, eps_B=0.125)
    t_plan = time.perf_counter()
    plan = mot.Plan(inst.points, inst.weights, W.TREE, inst.parent, inst.eta, path=mot.NFFT,
                    fastsum=fs)
    t_plan = time.perf_counter() - t_plan
    info = plan.info()

    # ---- timed NFFT sweeps
    plan.sinkhorn(args.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rc, done, S_last, err = plan.sinkhorn(args.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    nfft_s = (t1 - t0) / args.steps
    value = args.steps / (t1 - t0)

    # ---- per-launch device times (HIP events on the plan's stream)
    prof = plan.profile(args.profile_sweeps)

    # ---- direct GPU path on the same workload
    dplan = mot.Plan(inst.points, inst.weights, W.TREE, inst.parent, inst.eta, path=mot.DIRECT,
                     precision=mot.PREC_MIXED)
    dplan.sinkhorn(1)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    dplan.sinkhorn(args.direct_steps)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    direct_s = (t3 - t2) / args.direct_steps

    # ---- accuracy: same number of sweeps from phi = 1 on both paths
    ones = [np.ones(n) for n in inst.sizes]
    plan.set_scalings(ones)
    dplan.set_scalings(ones)
    plan.sinkhorn(args.acc_sweeps)
    dplan.sinkhorn(args.acc_sweeps)
    g_n = gauge_fix(plan.scalings(), inst.weights)
    g_d = gauge_fix(dplan.scalings(), inst.weights)
    phi_rel = max(float(np.max(np.abs(a - b) / np.abs(b))) for a, b in zip(g_n, g_d))
    Pn, _ = plan.marginals()
    Pd, _ = dplan.marginals()
    marg_viol = max(float(np.sum(np.abs(a - b))) for a, b in zip(Pn, Pd))
    dplan.close()

    # ---- roofline of the dominant launch
    K = inst.K
    dom = max(prof, key=lambda s: s["ms"])
    wk = step_work(dom, info, inst, K - 1)
    if dom["kind"] in ("spread", "interp"):
        achieved = wk["flops"] / (dom["ms"] * 1e-3) / 1e12
        roof = {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / PEAK_FP32_TFLOPS, "traffic": None,
                "kernel": dom["kind"], "ms_per_launch": dom["ms"],
                "work": "2 flop per window tap, (2m)^d taps per point, 9 products per launch"}
    else:
        achieved = wk["bytes"] / (dom["ms"] * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": achieved / PEAK_HBM_GBS, "traffic": None,
                "kernel": dom["kind"] + (str(dom["fft_kind"]) if dom["kind"] == "fft" else ""),
                "ms_per_launch": dom["ms"]}
    breakdown = {}
    for s in prof:
        key = s["kind"] + (str(s["fft_kind"]) if s["kind"] == "fft" else "")
        breakdown[key] = round(breakdown.get(key, 0.0) + s["ms"], 4)

    # ---- CPU oracle on a bounded sample: one direct product restricted to a prefix
    # of the targets, grown until it takes about --cpu-seconds
    import oracle
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    xs, v = inst.points[1], np.asarray(inst.weights[1])
    nt = 256
    while True:
        c0 = time.perf_counter()
        oracle.kernel_apply(inst.points[0][:nt], xs, v, inst.eta)
        dt = time.perf_counter() - c0
        if dt > 0.25 * args.cpu_seconds or nt >= inst.sizes[0]:
            break
        nt = min(inst.sizes[0], nt * 4)
    t_product = dt * inst.sizes[0] / nt
    cpu_sweeps = 1.0 / (2 * (K - 1) * t_product)

    out = {
        "metric": "Sinkhorn iters/s NFFT vs direct at rel err<=1e-5; p50/p99 solve latency",
        "value": value,
        "unit": "sweeps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": nfft_s * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "star tree K=10, N=%d per marginal, d=3, eta=0.05, NFFT grid 128^3, "
                               "m=6, M=32, tau=1, eps_B=1/8, p=3" % args.N,
                   "sweep_products": 2 * (K - 1), "updates": "f64", "seed": 2},
        "direct_sweeps_per_s": 1.0 / direct_s,
        "direct_ms_per_step": direct_s * 1e3,
        "speedup_vs_direct": direct_s / nfft_s,
        "accuracy": {"sweeps": args.acc_sweeps, "phi_gauge_fixed_max_rel_err": phi_rel,
                     "marginal_l1_diff_vs_direct": marg_viol,
                     "nfft_root_marginal_l1_after_timed_sweeps": err},
        "roofline": roof,
        "kernel_ms_per_sweep": breakdown,
        "plan_seconds": t_plan,
        "cpu_baseline": {"value": cpu_sweeps, "unit": "sweeps/s", "cores": cores, "kind": "oracle",
                         "sample": "FP64 oracle direct product of %d of %d targets x %d sources "
                                   "(%.2f s), scaled to %d products per sweep"
                                   % (nt, inst.sizes[0], inst.sizes[1], dt, 2 * (K - 1))},
    }
    print(json.dumps(out))
    plan.close()


if __name__ == "__main__":
    main()
