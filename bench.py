"""Throughput of the sparse FCT hot path on one MI355X.

One step = fct_sample -> fct_dct -> fct_solve (FP64) for the D=6,
|n|_1 <= 12 (18,564 coefficients) exp-cos workload on its four seeded
Chebyshev-Lobatto grids (341,100 samples), inputs already resident in HBM.
Plan construction is precomputation and is not timed.  The recovered
coefficients are checked against the stored oracle minimiser; only steps at
max-relative error <= 1e-10 count as recovered.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "recovered coeffs/sec + grid samples/sec at 1e-10 rel err; p50/p99 solve latency"
TOL = 1e-10


def cpu_baseline(prob, c_gold):
    """The oracle as it stands, on the same workload: sample, DCT by direct
    sums, least squares by the exact-Gram normal equations."""
    import oracle as O
    try:
        from threadpoolctl import threadpool_info
        threads = max([t.get("num_threads", 1) for t in threadpool_info()] + [1])
    except Exception:
        threads = os.cpu_count() or 1
    t0 = time.perf_counter()
    samples = O.sample_problem(prob)
    c, _, _ = O.fct_solve(prob.support, prob.grids, samples, "normal")
    dt = time.perf_counter() - t0
    err = O.max_rel_err(c, c_gold)
    return {"value": prob.n / dt, "unit": "coeffs/s", "cores": int(threads), "kind": "oracle",
            "sample": (f"one full job of the same workload ({prob.n} coefficients, "
                       f"{prob.total_points} samples): oracle sample + direct-sum DCT-I + "
                       f"normal-equation Cholesky, {dt:.1f} s, max_rel vs QR {err:.1e}")}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--eager", action="store_true", help="launch CGLS chunks without graphs")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the FCT path here is built and timed on a "
              "single MI355X (multi-GPU sharding is a design note, not built).", file=sys.stderr)
        sys.exit(2)

    import torch
    import workloads as W
    from paper_2309_14584_amd import fct

    torch.cuda.set_device(0)
    dev = torch.device("cuda", 0)
    prob = W.config2()
    c_gold = np.load(os.path.join(ROOT, "tests", "golden", "cfg2_coeffs_qr.npy"))
    plan = fct.Plan(prob.support, prob.grids)
    samples = torch.empty(plan.P, dtype=torch.float64, device=dev)
    b = torch.empty(plan.M, dtype=torch.float64, device=dev)
    c = torch.empty(plan.n, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()

    def step():
        plan.sample(prob.family, prob.params, out=samples)
        plan.dct(samples, out=b)
        return plan.solve(b, out=c, use_graph=not args.eager)[1]

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    lat = []
    iters = []
    t_start = time.perf_counter()
    for _ in range(args.steps):
        t0 = time.perf_counter()
        info = step()
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - t0)
        iters.append(info.iterations)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start

    c_host = c.cpu().numpy()
    err = float(np.max(np.abs(c_host - c_gold)) / np.max(np.abs(c_gold)))
    ok = err <= TOL
    ms = 1e3 * elapsed / args.steps
    coeffs_per_s = (prob.n * args.steps / elapsed) if ok else 0.0
    out = {
        "metric": METRIC,
        "value": coeffs_per_s,
        "unit": "coeffs/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": prob.name, "D": prob.D, "total_degree": 12,
                   "n_support": prob.n, "grids": prob.K, "total_points": prob.total_points,
                   "rows": plan.M, "family": "exp(-sum a x^2) cos(sum w x)", "seed": prob.seed},
        "grid_samples_per_s": (prob.total_points * args.steps / elapsed) if ok else 0.0,
        "p50_ms": 1e3 * float(np.percentile(lat, 50)),
        "p99_ms": 1e3 * float(np.percentile(lat, 99)),
        "max_rel_err": err,
        "cgls_iterations": int(np.median(iters)),
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(prob, c_gold)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
