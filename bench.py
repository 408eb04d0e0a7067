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
carries

* the roofline of the dominant kernel: algorithmic bytes or flops of its
  launches over their hipEvent-timed duration on the library's stream inside
  the timed region, and the HBM traffic that rocprofv3 counters measured for
  it (read from the summary under profiles/, and only while the kernel's
  sources are unchanged since the counters were taken);
* the other solver organisations at the same tolerance: plain (one solve per
  workgroup, float64), batched float64, batched mixed, each with and without
  ADMM over-relaxation, and the mixed sweep started by the learned network;
* the error of every variant against the CPU oracle on the bootstraps the
  oracle sample shares with the GPU run, and the oracle's own throughput;
* UoI_VAR fits of the two VAR workloads (p192 T10000, p1000 T20000), with the
  ADMM penalty rho = 1 and scaled to the data (--no-var skips them).

Profiling helpers (no GPU needed):  --summarize-trace DIR and
--summarize-pmc DIR print the text summaries kept under profiles/ from
rocprofv3 CSV output; --copy-calibration runs a 1 GiB device copy first so a
counter run also measures the scale of FETCH_SIZE/WRITE_SIZE.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0                      # MI355X HBM3E, GB/s
# MI355X dense matrix peaks, TFLOP/s.  The float32 ADMM product runs as six
# bfloat16 MFMA products of split operands, so its float32-equivalent peak is
# the bfloat16 peak (2500) / 6.
PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3, "f32_bf16x6": 2500.0 / 6}
TOL = 1e-6
COPY_BYTES = 1 << 30

# kstat slot -> (kernel name in profiles, sources whose change voids a stored traffic figure)
CSRC = os.path.join("paper_1808_06992_amd", "csrc")
KERNELS = {
    "admm32": ("uoi::k_bgemm_bf3<N, N, true, uoi::AdmmEpiBf3<N> >", ["bgemm.hpp", "admm.hip", "common.hpp"]),
    "admm64": ("uoi::k_bgemm<double, 1, N, uoi::AdmmEpi<double, 1, N> >", ["bgemm.hpp", "admm.hip", "common.hpp"]),
    "plain": ("uoi::k_admm_plain", ["admm.hip", "common.hpp"]),
    "gram": ("uoi::k_gram_f64<0, true>", ["gram.hip", "common.hpp"]),
}


def kernel_matches(slot, name):
    pat = re.escape(KERNELS[slot][0]).replace("N", r"\d+")
    return re.match(pat, _short(name)) is not None
WORKLOAD = "lasso_n5000_p1000"


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--variant", default="mixed", help="headline variant (see VARIANTS)")
    ap.add_argument("--relax", type=float, default=1.8, help="ADMM over-relaxation of the relaxed variants")
    ap.add_argument("--no-compare", action="store_true", help="skip the other variants")
    ap.add_argument("--no-mlp", action="store_true", help="skip the learned warm-start variant")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-var", action="store_true",
                    help="skip the UoI_VAR fits (p192 T10000 and p1000 T20000, rho 1 and rho scaled to the data)")
    ap.add_argument("--var-only", action="store_true",
                    help="run only the UoI_VAR fits and print their results as one JSON line {\"var\": ...} "
                         "(for profiling them on their own; not the benchmark line)")
    ap.add_argument("--cpu-boots", type=int, default=48,
                    help="bootstraps of the CPU oracle sample (B1 = B2 = this)")
    ap.add_argument("--mlp-seeds", type=int, default=4, help="design seeds of the network's training set")
    ap.add_argument("--tune-file", metavar="PATH",
                    help="the library's autotuner reads recorded launch shapes from PATH and appends new ones "
                         "(UOI_TUNE_FILE); counter runs use it so that no tuning launch is counted")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run a 1 GiB device copy first (scale of the HBM counters)")
    ap.add_argument("--summarize-trace", metavar="DIR", help="print a kernel-time summary and exit")
    ap.add_argument("--summarize-pmc", metavar="DIR", help="print a per-dispatch counter summary and exit")
    ap.add_argument("--make-traffic", nargs=3, metavar=("SLOT", "FETCH_DIR", "WRITE_DIR"),
                    help="print the HBM-traffic summary of a kernel slot from two counter runs and exit")
    return ap.parse_args()


def variants(relax):
    return {
        "plain": dict(precision="fp64", solver="plain", relax=1.0),
        "plain_relaxed": dict(precision="fp64", solver="plain", relax=relax),
        "fp64": dict(precision="fp64", solver="batched", relax=relax),
        "fp64_unrelaxed": dict(precision="fp64", solver="batched", relax=1.0),
        "mixed": dict(precision="mixed", solver="batched", relax=relax),
        "mixed_unrelaxed": dict(precision="mixed", solver="batched", relax=1.0),
    }


# --------------------------------------------------------------------------- helpers

def sources_digest(files):
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, CSRC, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def stored_traffic(slot, workload=WORKLOAD):
    """Per-launch HBM bytes of the slot's kernel from the committed counter
    summary, or None when absent or taken on other sources."""
    name, files = KERNELS[slot]
    path = os.path.join(ROOT, "profiles", f"traffic_{slot}_{workload}.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        m = re.match(r"\s*([a-z_0-9]+)\s*:\s*(.+?)\s*$", line)
        if m:
            kv[m.group(1)] = m.group(2)
    if kv.get("sources_sha256") != sources_digest(files):
        return None
    try:
        return float(kv["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def run_variant(api, torch, X, y, pr, kw, steps, warmup, mlp=None):
    for _ in range(warmup):
        o = api.lasso_fit(X, y, pr.lambdas, pr.B1, pr.B2, pr.seed, kkt_tol=TOL, timing=True, mlp=mlp, **kw)
        int(((o["kkt"] <= TOL) & (o["iters"] >= 0)).sum().item())  # warm torch's kernels too
    torch.cuda.synchronize()
    outs = []
    t0 = time.perf_counter()
    for _ in range(steps):
        outs.append(api.lasso_fit(X, y, pr.lambdas, pr.B1, pr.B2, pr.seed, kkt_tol=TOL, timing=True,
                                  mlp=mlp, **kw))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    # outside the timed region: count the solves that met the float64 KKT tolerance
    conv = 0
    kst = None
    for out in outs:
        conv += int(((out["kkt"] <= TOL) & (out["iters"] >= 0)).sum().item())
        ks = out["kstat"]
        if kst is None:
            kst = {k: dict(v) for k, v in ks.items()}
        else:
            for k in kst:
                for f in ("ms", "bytes", "flops", "launches"):
                    kst[k][f] += ks[k][f]
    last = outs[-1]
    st = last["stage_ms"]
    sel_ms = st["index+gram"] + st["factor"] + st["admm"] + st["support"]
    solves_step = conv / steps
    return dict(ms_per_step=1000.0 * dt / steps, solves_per_step=solves_step,
                solves_per_s=solves_step / (dt / steps), total_solves=pr.B1 * pr.lambdas.size,
                selection_ms=sel_ms, selection_solves_per_s=solves_step / (sel_ms / 1000.0),
                kstat=kst, stage_ms=st, max_iters=last["max_iters"],
                mean_iters=float(last["iters"].double().mean().item()),
                warm_used=int(last["warm_used"]))


def selection_betas(api, X, y, pr, kw, mlp=None):
    out = api.lasso_fit(X, y, pr.lambdas, pr.B1, pr.B2, pr.seed, kkt_tol=TOL, sel_beta=True, mlp=mlp, **kw)
    return out["sel_beta"].cpu().numpy(), out["beta"].cpu().numpy()


def roofline(kst, workload=WORKLOAD):
    """Dominant kernel = the timed kernel slot with the largest device time.  Its
    HBM traffic comes from the workload's committed counter summary, if any."""
    cands = {k: v for k, v in kst.items() if v["launches"] > 0}
    dom = max(cands, key=lambda k: cands[k]["ms"])
    k = cands[dom]
    sec = k["ms"] / 1000.0
    dt = "f32_bf16x6" if dom == "admm32" else "f64"
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
    launches = max(int(k["launches"]), 1)
    r.update(traffic=stored_traffic(dom, workload), kernel=KERNELS[dom][0], slot=dom, launches=int(k["launches"]),
             avg_launch_us=round(1000.0 * k["ms"] / launches, 2),
             algorithmic_bytes_per_launch=round(k["bytes"] / launches),
             algorithmic_flops_per_launch=round(k["flops"] / launches),
             kernel_ms_per_step_share=None)
    return r


def cpu_baseline(pr, boots):
    """The oracle as it stands (C, float64, OpenMP over bootstraps) on a bounded sample."""
    import oracle
    oracle.build()
    q = pr.lambdas.size
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    t0 = time.perf_counter()
    r = oracle.uoi_lasso(pr.X, pr.y, pr.lambdas, boots, boots, pr.seed, tol=1e-12, keep_selection=True)
    dt = time.perf_counter() - t0
    solves = boots * q
    base = dict(value=round(solves / dt, 3), unit="solves/s", cores=min(threads, boots), kind="oracle",
                sample=f"full UoI_LASSO fit with B1=B2={boots} of the 48 bootstraps (same n, p, q); "
                       f"{solves} selection solves in {dt:.1f} s; OpenMP over bootstraps",
                status=r["status"])
    return base, r


def err_vs_oracle(gpu, orc, full):
    """Selection solves of the bootstraps both runs share: max and median of
    ||b_gpu - b_oracle||_inf / ||b_oracle||_inf, and differing support bits
    (undecided bits included, so a few may differ at tolerance 1e-6); with the
    full bootstrap counts also the relative error of the final coefficients."""
    import numpy as np
    sel_orc = orc["sel_beta"]
    k = sel_orc.shape[0]
    g = gpu[0][:k]
    scale = np.maximum(np.abs(sel_orc).max(axis=-1), 1e-300)
    rel = np.abs(g - sel_orc).max(axis=-1) / scale
    r = dict(sel_beta_max_rel=float(rel.max()), sel_beta_median_rel=float(np.median(rel)),
             solves_compared=int(rel.size), support_bits_differing=int(((g != 0) != (sel_orc != 0)).sum()))
    if full:
        r["beta_star_max_rel"] = float(np.abs(gpu[1] - orc["beta"]).max() / max(np.abs(orc["beta"]).max(), 1e-300))
    return r


def copy_calibration(torch):
    """A plain 1 GiB device copy (read 1 GiB, write 1 GiB) for counter scaling."""
    src = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst


# --------------------------------------------------------------------------- rocprofv3 summaries

def _short(name):
    name = re.sub(r"\(.*", "", name)
    name = re.sub(r"^void ", "", name)
    return name[:110]


def summarize_trace(d):
    files = glob.glob(os.path.join(d, "**", "*kernel_trace.csv"), recursive=True)
    if not files:
        sys.exit(f"no *kernel_trace.csv under {d}")
    agg = {}
    for f in files:
        for row in csv.DictReader(open(f)):
            nm = _short(row["Kernel_Name"])
            dur = (int(row["End_Timestamp"]) - int(row["Start_Timestamp"])) / 1000.0
            a = agg.setdefault(nm, [0, 0.0, 1e300, 0.0])
            a[0] += 1
            a[1] += dur
            a[2] = min(a[2], dur)
            a[3] = max(a[3], dur)
    tot = sum(v[1] for v in agg.values())
    print(f"kernel time {tot / 1000.0:.3f} ms over {sum(v[0] for v in agg.values())} dispatches")
    print(f"{'total ms':>10} {'calls':>7} {'avg us':>10} {'min us':>10} {'max us':>10}  kernel")
    for nm, (c, us, mn, mx) in sorted(agg.items(), key=lambda x: -x[1][1]):
        print(f"{us / 1000.0:10.3f} {c:7d} {us / c:10.2f} {mn:10.2f} {mx:10.2f}  {nm}")


def summarize_pmc(d):
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        sys.exit(f"no *counter_collection.csv under {d}")
    agg, disp = {}, {}
    for f in files:
        for row in csv.DictReader(open(f)):
            nm = _short(row["Kernel_Name"])
            key = (nm, row["Counter_Name"])
            agg[key] = agg.get(key, 0.0) + float(row["Counter_Value"])
            disp.setdefault(nm, set()).add((f, row.get("Dispatch_Id", row.get("Correlation_Id", ""))))
    print(f"{'per dispatch':>16} {'dispatches':>10}  counter  kernel")
    for (nm, cn), v in sorted(agg.items()):
        n = len(disp[nm])
        print(f"{v / n:16.1f} {n:10d}  {cn}  {nm}")


def _pmc_rows(d):
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        sys.exit(f"no *counter_collection.csv under {d}")
    rows = []
    for f in files:
        rows += list(csv.DictReader(open(f)))
    return rows


def make_traffic(slot, fetch_dir, write_dir):
    """HBM bytes per launch of the slot's kernel: FETCH_SIZE and WRITE_SIZE (KiB
    per dispatch), each scaled by what the same counter reads for the 1 GiB
    calibration copy (a device-to-device copy kernel that reads and writes 1 GiB)."""
    out = {}
    for tag, d, cn in (("fetch", fetch_dir, "FETCH_SIZE"), ("write", write_dir, "WRITE_SIZE")):
        rows = [r for r in _pmc_rows(d) if r["Counter_Name"] == cn]
        cal = [float(r["Counter_Value"]) for r in rows
               if "copyBuffer" in r["Kernel_Name"] and float(r["Counter_Value"]) >= COPY_BYTES / 1024 / 4]
        ker = [float(r["Counter_Value"]) for r in rows if kernel_matches(slot, r["Kernel_Name"])]
        if not cal or not ker:
            sys.exit(f"{d}: calibration copies {len(cal)}, {slot} dispatches {len(ker)}")
        cal_kib = sum(cal) / len(cal)
        out[tag] = dict(kib=sum(ker) / len(ker), n=len(ker), cal_kib=cal_kib, scale=(COPY_BYTES / 1024) / cal_kib)
    tb = sum(v["kib"] * 1024 * v["scale"] for v in out.values())
    print(f"kernel: {KERNELS[slot][0]}")
    print(f"slot: {slot}")
    print(f"workload: {WORKLOAD} (UoI_LASSO n=5000 p=1000 B1=q=B2=48), bench.py --steps 1 --warmup 0")
    print(f"sources_sha256: {sources_digest(KERNELS[slot][1])}")
    for tag, v in out.items():
        print(f"{tag}_kib_per_dispatch: {v['kib']:.1f}")
        print(f"{tag}_dispatches: {v['n']}")
        print(f"{tag}_calibration_copy_kib_per_gib: {v['cal_kib']:.1f}")
        print(f"{tag}_scale: {v['scale']:.5f}")
    print(f"traffic_bytes_per_launch: {tb:.0f}")


# --------------------------------------------------------------------------- main

def var_fits(api, torch, synth, log):
    """UoI_VAR fits of the two VAR workloads (mixed, relax 1.8, KKT 1e-6): one
    warm-up and one timed fit each, with the paper's rho = 1 and with rho scaled
    to the data (rho = 0: the mean diagonal of the Grams).  A selection solve is
    one (bootstrap, lambda, equation) LASSO of dimension p.  Each timed fit also
    reports its stage times and the roofline object of its dominant kernel (per
    launch averages over the fit's launches, partly active ones included)."""
    out = {}
    for name, mk in (("var_p192_T10000", synth.var_small), ("var_p1000_T20000", synth.var_large)):
        pr = mk(0)
        s = torch.as_tensor(pr.series).cuda()
        nsol = pr.B1 * pr.lambdas.size * pr.series.shape[1]
        res = {"B1": pr.B1, "q": int(pr.lambdas.size), "B2": pr.B2, "selection_solves": nsol}
        for label, rho in (("rho_1", 1.0), ("rho_data", 0.0)):
            kw = dict(kkt_tol=1e-6, precision="mixed", relax=1.8, rho=rho, timing=True)
            api.var_fit(s, pr.lambdas, pr.B1, pr.B2, 0, **kw)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            o = api.var_fit(s, pr.lambdas, pr.B1, pr.B2, 0, **kw)
            torch.cuda.synchronize()
            t = time.perf_counter() - t0
            it = o["iters"].float()
            res[label] = dict(ms_per_fit=round(1000 * t, 2), solves_per_s=round(nsol / t, 1),
                              mean_iters=round(float(it.mean()), 2), max_iters=int(it.max()),
                              unconverged=int(o["n_unconverged"]), status=int(o["status"]),
                              stage_ms={k: round(v, 3) for k, v in o["stage_ms"].items()},
                              roofline=roofline(o["kstat"], name))
            log(f"{name} {label}: {1000 * t:.1f} ms/fit, {nsol / t:.0f} solves/s, mean iters {float(it.mean()):.1f}")
        out[name] = res
    return out


def main():
    a = parse()
    if a.summarize_trace:
        summarize_trace(a.summarize_trace)
        return
    if a.summarize_pmc:
        summarize_pmc(a.summarize_pmc)
        return
    if a.make_traffic:
        make_traffic(*a.make_traffic)
        return
    if a.gpus != 1:
        print(f"bench.py: runs on one GPU (asked for --gpus {a.gpus}); splitting the bootstraps "
              "over several GPUs is not implemented", file=sys.stderr)
        sys.exit(2)
    if a.tune_file:
        os.environ["UOI_TUNE_FILE"] = os.path.abspath(a.tune_file)
    import torch
    from paper_1808_06992_amd import _lib as api
    from paper_1808_06992_amd import synth
    api.load()
    if not torch.cuda.is_available():
        print("bench.py: no HIP device", file=sys.stderr)
        sys.exit(1)
    V = variants(a.relax)
    if a.variant not in V:
        sys.exit(f"unknown variant {a.variant}; choose from {sorted(V)}")
    if a.copy_calibration:
        copy_calibration(torch)
    if a.var_only:
        log = lambda s: print(f"[bench] {s}", file=sys.stderr, flush=True)  # noqa: E731
        print(json.dumps({"var": var_fits(api, torch, synth, log)}), flush=True)
        return
    pr = synth.lasso_toeplitz(0)
    X = torch.as_tensor(pr.X).cuda()
    y = torch.as_tensor(pr.y).cuda()
    log = lambda s: print(f"[bench] {s}", file=sys.stderr, flush=True)  # noqa: E731
    log(f"workload n={pr.X.shape[0]} p={pr.X.shape[1]} B1={pr.B1} q={pr.lambdas.size} B2={pr.B2}; "
        f"headline {a.variant} {V[a.variant]}")
    head = run_variant(api, torch, X, y, pr, V[a.variant], a.steps, a.warmup)
    log(f"{a.variant}: {head['ms_per_step']:.2f} ms/step, {head['solves_per_s']:.0f} solves/s, "
        f"mean iters {head['mean_iters']:.1f}, stages "
        + json.dumps({k: round(v, 2) for k, v in head["stage_ms"].items()}))
    compare, sels = {}, {}
    if not a.no_compare:
        sels[a.variant] = selection_betas(api, X, y, pr, V[a.variant])
        for v, kw in V.items():
            if v == a.variant:
                continue
            plain = kw["solver"] == "plain"
            r = run_variant(api, torch, X, y, pr, kw, 1 if plain else max(2, a.steps // 2), 1)
            compare[v] = dict(kw, solves_per_s=round(r["solves_per_s"], 1), ms_per_step=round(r["ms_per_step"], 3),
                              selection_solves_per_s=round(r["selection_solves_per_s"], 1),
                              mean_iters=round(r["mean_iters"], 2), max_iters=r["max_iters"],
                              stage_ms={k: round(x, 3) for k, x in r["stage_ms"].items()})
            sels[v] = selection_betas(api, X, y, pr, kw)
            log(f"{v}: {r['ms_per_step']:.2f} ms/step, {r['solves_per_s']:.0f} solves/s, "
                f"mean iters {r['mean_iters']:.1f}")
        if not a.no_mlp:
            try:
                from paper_1808_06992_amd import warmstart as ws
                t0 = time.perf_counter()
                seeds = list(range(1000, 1000 + a.mlp_seeds))
                net, hist, ntrain = ws.fit_network(seeds, B1=8, M=64)
                t_train = time.perf_counter() - t0
                kw = V[a.variant]
                r = run_variant(api, torch, X, y, pr, kw, max(2, a.steps // 2), 1, mlp=net)
                compare[a.variant + "_mlp"] = dict(
                    kw, warm_start="mlp", solves_per_s=round(r["solves_per_s"], 1),
                    ms_per_step=round(r["ms_per_step"], 3),
                    selection_solves_per_s=round(r["selection_solves_per_s"], 1),
                    mean_iters=round(r["mean_iters"], 2), max_iters=r["max_iters"], warm_used=r["warm_used"],
                    stage_ms={k: round(x, 3) for k, x in r["stage_ms"].items()},
                    training=dict(design_seeds=seeds, solves=ntrain, epochs=len(hist),
                                  final_loss=hist[-1], first_loss=hist[0], seconds=round(t_train, 1)))
                sels[a.variant + "_mlp"] = selection_betas(api, X, y, pr, kw, mlp=net)
                log(f"{a.variant}_mlp: {r['ms_per_step']:.2f} ms/step, {r['solves_per_s']:.0f} solves/s, "
                    f"mean iters {r['mean_iters']:.1f}, warm starts used {r['warm_used']}, "
                    f"training {t_train:.1f} s on {ntrain} solves")
            except Exception as e:  # reported, never hidden
                compare[a.variant + "_mlp"] = dict(error=f"{type(e).__name__}: {e}")
    rl = roofline(head["kstat"])
    rl["kernel_ms_per_step_share"] = round(
        head["kstat"][rl["slot"]]["ms"] / a.steps / head["ms_per_step"], 4)
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
        "dtype": "f32+f64" if V[a.variant]["precision"] == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": "UoI_LASSO n=5000 p=1000 Toeplitz(0.5) design, 100 nonzeros, SNR 5, "
                               "B1=48 q=48 B2=48, KKT tol 1e-6",
                   "variant": a.variant, **V[a.variant], "solves_per_step": head["total_solves"],
                   "converged_per_step": head["solves_per_step"], "max_iters": head["max_iters"],
                   "mean_iters": round(head["mean_iters"], 2)},
        "selection_solves_per_s": round(head["selection_solves_per_s"], 1),
        "roofline": rl,
        "stage_ms": {k: round(v, 3) for k, v in head["stage_ms"].items()},
        "compare": compare,
    }
    for ref in ("plain", "plain_relaxed"):
        if compare.get(ref, {}).get("solves_per_s"):
            line["vs_" + ref] = round(head["solves_per_s"] / compare[ref]["solves_per_s"], 2)
    if not a.no_var:
        try:
            line["var"] = var_fits(api, torch, synth, log)
        except Exception as e:  # reported, never hidden
            line["var"] = dict(error=f"{type(e).__name__}: {e}")
    if not a.no_cpu:
        boots = min(a.cpu_boots, pr.B1)
        base, orc = cpu_baseline(pr, boots)
        line["cpu_baseline"] = base
        if sels:
            full = boots == pr.B1 and pr.B1 == pr.B2
            line["err_vs_oracle"] = {v: err_vs_oracle(s, orc, full) for v, s in sels.items()}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
