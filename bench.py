#!/usr/bin/env python3
"""Benchmark: LASSO solves/sec of UoI_LASSO on one MI355X.

One step = one whole UoI_LASSO fit (Alg. 1: bootstrap index streams, gathered
Gram, factor, the bootstrap x lambda ADMM sweep with float64 KKT verification,
support intersection, estimation splits, masked OLS refits, loss, argmin,
average) on the workload  n=5000, p=1000, Toeplitz(0.5) design, 100 nonzero
coefficients, SNR 5, B1 = q = B2 = 48 (2304 selection solves per step).
Inputs are synthetic and already resident in HBM when the timed region starts.

value = (selection solves per step that reach the float64 KKT tolerance
1e-6) / (seconds per step), i.e. whole-fit throughput.  The JSON line also
carries the roofline of the dominant kernel (live hipEvent timing of its
launches on the library's stream inside the timed region), the other solver
organisations for comparison (plain one-solve-per-workgroup float64 and
batched float64), and the CPU oracle timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0       # MI355X HBM3E, GB/s
PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3}  # MI355X dense matrix peaks, TFLOP/s


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--variant", default="mixed", choices=["mixed", "fp64", "plain"],
                    help="solver organisation of the headline value")
    ap.add_argument("--no-compare", action="store_true", help="skip the other variants")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-boots", type=int, default=6,
                    help="bootstraps of the CPU oracle sample (B1 = B2 = this)")
    return ap.parse_args()


VARIANTS = {"mixed": dict(precision="mixed", solver="batched"),
            "fp64": dict(precision="fp64", solver="batched"),
            "plain": dict(precision="fp64", solver="plain")}


def run_variant(api, torch, X, y, pr, variant, steps, warmup, tol):
    kw = VARIANTS[variant]
    q = pr.lambdas.size
    for _ in range(warmup):
        o = api.lasso_fit(X, y, pr.lambdas, pr.B1, pr.B2, pr.seed, kkt_tol=tol, timing=True, **kw)
        int(((o["kkt"] <= tol) & (o["iters"] >= 0)).sum().item())  # warm torch's kernels too
    torch.cuda.synchronize()
    outs = []
    t0 = time.perf_counter()
    for _ in range(steps):
        outs.append(api.lasso_fit(X, y, pr.lambdas, pr.B1, pr.B2, pr.seed, kkt_tol=tol, timing=True,
                                  **kw))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    # outside the timed region: count the solves that met the float64 KKT tolerance
    conv = 0
    kst = None
    for out in outs:
        conv += int(((out["kkt"] <= tol) & (out["iters"] >= 0)).sum().item())
        ks = out["kstat"]
        if kst is None:
            kst = {k: dict(v) for k, v in ks.items()}
        else:
            for k in kst:
                for f in ("ms", "bytes", "flops", "launches"):
                    kst[k][f] += ks[k][f]
    ms_step = 1000.0 * dt / steps
    solves_step = conv / steps
    return dict(ms_per_step=ms_step, solves_per_step=solves_step,
                solves_per_s=solves_step / (dt / steps), total_solves=pr.B1 * q,
                kstat=kst, stage_ms=outs[-1]["stage_ms"], max_iters=outs[-1]["max_iters"])


def roofline(kst, variant):
    """Dominant kernel = the ADMM iteration kernel of the variant (largest device time)."""
    slot = {"mixed": "admm32", "fp64": "admm64", "plain": "plain"}[variant]
    cands = {k: v for k, v in kst.items() if v["launches"] > 0}
    dom = max(cands, key=lambda k: cands[k]["ms"])
    k = cands[dom]
    sec = k["ms"] / 1000.0
    dt = "f32" if dom == "admm32" else "f64"
    gbs = k["bytes"] / sec / 1e9
    tfl = k["flops"] / sec / 1e12
    t_hbm = k["bytes"] / (HBM_PEAK_GBS * 1e9)
    t_mfma = k["flops"] / (PEAK_TFLOPS[dt] * 1e12)
    if t_hbm >= t_mfma:
        r = dict(bound="hbm", achieved=round(gbs, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                 frac=round(gbs / HBM_PEAK_GBS, 4))
    else:
        r = dict(bound="mfma", achieved=round(tfl, 2), peak=PEAK_TFLOPS[dt], unit="TFLOP/s",
                 frac=round(tfl / PEAK_TFLOPS[dt], 4))
    r.update(kernel={"admm32": "k_bgemm<float> ADMM iteration", "admm64": "k_bgemm<double> ADMM iteration",
                     "plain": "k_admm_plain", "gram": "k_gram_f64"}[dom],
             traffic=None, launches=int(k["launches"]),
             avg_launch_us=round(1000.0 * k["ms"] / max(k["launches"], 1), 2),
             algorithmic_bytes_per_launch=k["bytes"] / max(k["launches"], 1),
             algorithmic_flops_per_launch=k["flops"] / max(k["launches"], 1),
             headline_variant_slot=slot)
    return r


def cpu_baseline(pr, boots):
    """The oracle as it stands (C, float64, OpenMP over bootstraps) on a bounded sample."""
    import oracle
    oracle.build()
    n, p = pr.X.shape
    q = pr.lambdas.size
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    t0 = time.perf_counter()
    r = oracle.uoi_lasso(pr.X, pr.y, pr.lambdas, boots, boots, pr.seed, tol=1e-12)
    dt = time.perf_counter() - t0
    solves = boots * q
    return dict(value=round(solves / dt, 3), unit="solves/s", cores=min(threads, boots),
                kind="oracle",
                sample=f"full UoI_LASSO fit with B1=B2={boots} of the 48 bootstraps (same n, p, q); "
                       f"{solves} selection solves in {dt:.1f} s; OpenMP over bootstraps",
                status=r["status"])


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {a.gpus}); "
              "multi-GPU sharding is described in DESIGN.md but not built", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1808_06992_amd import _lib as api
    from paper_1808_06992_amd import synth
    api.load()
    if not torch.cuda.is_available():
        print("bench.py: no HIP device", file=sys.stderr)
        sys.exit(1)
    pr = synth.lasso_toeplitz(0)
    X = torch.as_tensor(pr.X).cuda()
    y = torch.as_tensor(pr.y).cuda()
    tol = 1e-6
    print(f"[bench] workload n={pr.X.shape[0]} p={pr.X.shape[1]} B1={pr.B1} q={pr.lambdas.size} "
          f"B2={pr.B2}; headline variant {a.variant}", file=sys.stderr, flush=True)
    head = run_variant(api, torch, X, y, pr, a.variant, a.steps, a.warmup, tol)
    print(f"[bench] {a.variant}: {head['ms_per_step']:.2f} ms/step, {head['solves_per_s']:.0f} solves/s, "
          f"stages {head['stage_ms']}", file=sys.stderr, flush=True)
    compare = {}
    if not a.no_compare:
        for v in VARIANTS:
            if v == a.variant:
                continue
            r = run_variant(api, torch, X, y, pr, v, 1 if v == "plain" else max(1, a.steps // 2), 1, tol)
            compare[v] = dict(solves_per_s=round(r["solves_per_s"], 1),
                              ms_per_step=round(r["ms_per_step"], 3), max_iters=r["max_iters"])
            print(f"[bench] {v}: {r['ms_per_step']:.2f} ms/step, {r['solves_per_s']:.0f} solves/s",
                  file=sys.stderr, flush=True)
    line = {
        "metric": "LASSO solves/sec (bootstrap x lambda) at KKT tol 1e-6, batched/mixed vs plain",
        "value": round(head["solves_per_s"], 1),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(head["ms_per_step"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if a.variant == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": "UoI_LASSO n=5000 p=1000 Toeplitz(0.5) design, 100 nonzeros, SNR 5, "
                               "B1=48 q=48 B2=48, KKT tol 1e-6",
                   "variant": a.variant, "solves_per_step": head["total_solves"],
                   "converged_per_step": head["solves_per_step"], "max_iters": head["max_iters"]},
        "roofline": roofline(head["kstat"], a.variant),
        "stage_ms": {k: round(v, 3) for k, v in head["stage_ms"].items()},
        "compare": compare,
    }
    if compare.get("plain"):
        line["vs_plain"] = round(head["solves_per_s"] / max(compare["plain"]["solves_per_s"], 1e-9), 2)
    if not a.no_cpu:
        line["cpu_baseline"] = cpu_baseline(pr, a.cpu_boots)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
