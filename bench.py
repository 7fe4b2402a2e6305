"""Benchmark: ALTO sparse MTTKRP / CP-ALS on one MI355X.

One step = the whole hot path over one synthetic tensor whose COO input is
already in HBM: alto_build (linearize, radix-sort, coalesce, partition,
intervals, coverage) followed by CP-ALS for the configured number of
iterations (per mode: execution choice, MTTKRP, merge, FP64 normal
equations), FP32 factors, execution chosen by the library (the trained
selector network when its weights are present, else the reuse rule).

value = MTTKRP nonzeros processed per second over the whole step
        (iterations x modes x distinct nonzeros / step time).

Extra fields: per-mode MTTKRP time, nnz/s and % of the 8 TB/s HBM peak in
algorithmic bytes for every strategy, FP32 and BF16 factors; CP-ALS ms per
iteration and fit for the plain FP32 form (reuse rule, no network) and the
network-chosen FP32 and BF16 forms; `roofline` for the MTTKRP kernel;
`cpu_baseline` (the FP64 oracle on a bounded sample, one host core).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
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

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="zipf4_1Mx100kx10kx500_150M")
    ap.add_argument("--iters", type=int, default=20, help="CP-ALS iterations per step")
    ap.add_argument("--reps", type=int, default=10, help="timed repetitions per mode for per-mode MTTKRP")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-selector", action="store_true", help="do not load the selector weights")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="target oracle CPU time")
    ap.add_argument("--mttkrp-only", action="store_true",
                    help="only per-mode MTTKRP repetitions of the chosen plan (for counter collection)")
    ap.add_argument("--format", action="store_true",
                    help="format generation and storage on every workload: alto_build time and index "
                         "bytes vs COO (prints its own JSON line instead of the benchmark line)")
    return ap.parse_args()


def logical_bytes_per_nnz(N, R, key_bits, fbytes):
    """Algorithmic bytes one nonzero moves in a mode-n MTTKRP: its index and
    value, N-1 gathered factor rows, and its R-wide FP32 output update."""
    return key_bits / 8 + 4 + (N - 1) * R * fbytes + 4 * R


def format_experiment(alto, torch, synth, dev, reps=3):
    """alto_build time (encode, sort, coalesce, partition; inputs resident in
    HBM) and stored index bytes vs uint32 COO coordinates (Eq. 1 vs the COO
    count) for every workload."""
    res = []
    for name, rec in synth.WORKLOADS.items():
        coords, vals = synth.coo(rec)
        c_dev = torch.from_numpy(coords.view(np.int32)).to(dev)
        v_dev = torch.from_numpy(vals).to(dev)
        del coords, vals
        torch.cuda.synchronize()
        times = []
        info = None
        for _ in range(reps + 1):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            t = alto.AltoTensor.build(c_dev, v_dev, rec.dims)
            e1.record()
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1))
            info = t.info()
            t.close()
        ms = float(np.median(times[1:]))  # the first build also loads kernels
        M = info["nnz"]
        r = {"workload": name, "dims": list(rec.dims), "nnz_draws": rec.nnz, "nnz": M,
             "index_bits": info["index_bits"], "key_bits": info["key_bits"],
             "alto_index_bytes": info["index_bytes"], "coo_index_bytes": info["coo_index_bytes"],
             "index_bytes_ratio_coo_over_alto": info["coo_index_bytes"] / max(1.0, info["index_bytes"]),
             "build_ms": ms, "build_draws_per_s": rec.nnz / (ms * 1e-3)}
        res.append(r)
        log(f"format {name}: B={r['index_bits']} W={r['key_bits']} index {info['index_bytes'] / 1e9:.3f} GB vs "
            f"COO {info['coo_index_bytes'] / 1e9:.3f} GB; alto_build {ms:.2f} ms "
            f"({r['build_draws_per_s'] / 1e9:.2f} G draws/s)")
        del c_dev, v_dev
        torch.cuda.empty_cache()
    return res


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(--gpus must be 1)", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2102_10245_amd as alto
    import synth

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    alto.lib()  # fail loudly if the HIP library is missing
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    if args.format:
        print(json.dumps({"format_experiment": format_experiment(alto, torch, synth, dev)}))
        return
    have_sel = (not args.no_selector) and alto.load_default_selector()
    rec = synth.WORKLOADS[args.workload]
    R = rec.rank
    t0 = time.time()
    coords, vals = synth.coo(rec)
    log(f"generated {rec.name}: {coords.shape[1]} draws in {time.time() - t0:.1f}s; selector "
        f"{'loaded' if have_sel else 'absent (reuse rule)'}")
    c_dev = torch.from_numpy(coords.view(np.int32)).to(dev)
    v_dev = torch.from_numpy(vals).to(dev)
    init = synth.factors(rec.seed + 1, rec.dims, R)
    init_f32 = [torch.from_numpy(f).to(dev) for f in init]
    init_bf16 = [f.to(torch.bfloat16) for f in init_f32]
    work = {"f32": [f.clone() for f in init_f32], "bf16": [f.clone() for f in init_bf16]}
    src = {"f32": init_f32, "bf16": init_bf16}
    N = len(rec.dims)
    torch.cuda.synchronize()

    def step(prec="f32", timers=None):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)] if timers is not None else None
        for w, s in zip(work[prec], src[prec]):
            w.copy_(s)
        if ev:
            ev[0].record()
        t = alto.AltoTensor.build(c_dev, v_dev, rec.dims)
        if ev:
            ev[1].record()
        lam, fit = t.cp_als(work[prec], args.iters)
        if ev:
            ev[2].record()
        info = t.info()
        plan = [t.select(m, R, prec) for m in range(N)]
        t.close()
        if timers is not None:
            torch.cuda.synchronize()
            timers.append((ev[0].elapsed_time(ev[1]), ev[1].elapsed_time(ev[2])))
        return info, fit, plan

    if args.mttkrp_only:
        # a plain 1 GiB device copy first: its counter readings calibrate the
        # HBM byte counters (FETCH_SIZE / WRITE_SIZE) against a known size
        a = torch.empty(1 << 28, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        a.fill_(1.0)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
        t = alto.AltoTensor.build(c_dev, v_dev, rec.dims)
        per_mode = time_modes(alto, torch, t, init_f32, R, N, args.reps, "f32", "auto")
        print(json.dumps({"mttkrp_only": per_mode}))
        t.close()
        return

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = []
    for k in range(args.steps):
        infos.append(step())
        log(f"step {k + 1}/{args.steps} done")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    info, fit_f32, plan_f32 = infos[-1]
    M = info["nnz"]
    ms_per_step = 1e3 * elapsed / args.steps
    value = args.iters * N * M / (elapsed / args.steps)

    # the forms: network-chosen FP32 / BF16, and the plain FP32 form (reuse rule)
    forms = {}
    for name, prec, sel in (("selector_f32", "f32", have_sel), ("selector_bf16", "bf16", have_sel),
                            ("plain_f32", "f32", False)):
        if not sel:
            alto.selector_load(None)
        tim = []
        _, fit, plan = step(prec, tim)
        if have_sel:
            alto.load_default_selector()
        forms[name] = {"build_ms": tim[0][0], "cp_als_ms_per_iter": tim[0][1] / args.iters,
                       "fit": float(fit[-1]) if len(fit) else None,
                       "plan": [{"strategy": s, "num_segments": L} for s, L in plan]}
        log(f"{name}: CP-ALS {tim[0][1] / args.iters:.2f} ms/iter, fit {forms[name]['fit']:.6f}, plan {plan}")

    # per-mode MTTKRP for every strategy and precision on the built tensor
    t = alto.AltoTensor.build(c_dev, v_dev, rec.dims)
    per_mode = {}
    for prec, fs in (("f32", init_f32), ("bf16", init_bf16)):
        for st in ("auto", "atomic", "staged", "sorted"):
            per_mode[f"{st}_{prec}"] = time_modes(alto, torch, t, fs, R, N, args.reps, prec, st)
    kb = t.info()["key_bits"]
    t.close()

    # roofline of the MTTKRP kernel under the chosen FP32 plan: algorithmic
    # bytes per launch over the mean launch time (all modes pooled)
    main_modes = per_mode["auto_f32"]
    tot_bytes = sum(m["logical_bytes"] for m in main_modes)
    tot_ms = sum(m["ms"] for m in main_modes)
    achieved = tot_bytes / (tot_ms * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(rec.name),
                "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, calibrated)",
                "kernel": "mttkrp_k (64-bit index, order 4, R=32, FP32 factors), mean over the 4 modes"}

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(rec, coords, vals, init, R, N, args.cpu_seconds)

    out = {
        "metric": "MTTKRP nnz/s & % HBM peak per mode; CP-ALS iter ms, FP32 vs BF16-factor",
        "value": value,
        "unit": "nnz/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": rec.name, "dims": list(rec.dims), "nnz_draws": rec.nnz, "nnz": M,
            "zipf": list(rec.zipf), "values": rec.values, "rank": R, "cp_als_iters": args.iters,
            "index_bits": info["index_bits"], "key_bits": kb, "num_segments": info["num_segments"],
            "execution": "selector" if have_sel else "reuse rule",
            "plan": [{"strategy": s, "num_segments": L} for s, L in plan_f32],
        },
        "roofline": roofline,
        "cpu_baseline": cpu,
        "forms": forms,
        "per_mode": per_mode,
        "fit_f32": float(fit_f32[-1]) if len(fit_f32) else None,
    }
    print(json.dumps(out))


def measured_traffic(workload):
    """HBM bytes per MTTKRP launch from the committed counter profile, or None
    when there is none for this workload or the kernel source changed since."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "mttkrp_zipf4_150M_r32_f32_hbm_traffic.json")
    src = os.path.join(ROOT, "paper_2102_10245_amd", "csrc", "mttkrp_impl.h")
    if not os.path.exists(path) or workload != "zipf4_1Mx100kx10kx500_150M":
        return None
    with open(path) as f:
        prof = json.load(f)
    with open(src, "rb") as f:
        if hashlib.sha1(f.read()).hexdigest() != prof.get("kernel_source_sha1"):
            return None
    return round(prof["hbm_bytes_per_launch"])


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def time_modes(alto, torch, t, factors, R, N, reps, prec, strategy):
    info = t.info()
    M = info["nnz"]
    fb = 4 if prec == "f32" else 2
    res = []
    for mode in range(N):
        out = torch.empty((info["dims"][mode], R), dtype=torch.float32, device=factors[0].device)
        strat, L = t.select(mode, R, prec) if strategy == "auto" else (strategy, 0)
        t.mttkrp(factors, mode, out=out, strategy=strategy)  # warmup (plans, orders)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            t.mttkrp(factors, mode, out=out, strategy=strategy)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        lb = logical_bytes_per_nnz(N, R, info["key_bits"], fb) * M
        res.append({"mode": mode, "strategy": strat, "num_segments": L or info["num_segments"], "ms": ms,
                    "nnz_per_s": M / (ms * 1e-3), "logical_bytes": lb, "logical_GBps": lb / (ms * 1e-3) / 1e9,
                    "pct_hbm_peak": 100.0 * lb / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS})
        log(f"mode {mode} {prec} {strategy}->{strat}: {ms:.3f} ms, {M / (ms * 1e-3) / 1e9:.2f} G nnz/s, "
            f"{res[-1]['pct_hbm_peak']:.1f}% of HBM peak (algorithmic bytes)")
    return res


def cpu_baseline(rec, coords, vals, init, R, N, seconds):
    """The FP64 oracle's COO MTTKRP (one host core) on the first S draws of
    the same tensor, all modes; S sized for about `seconds` of work."""
    import oracle
    oracle.build(force=False)
    init = [np.asarray(f, np.float64) for f in init]
    s = 200000
    t0 = time.perf_counter()
    for mode in range(N):
        oracle.mttkrp(rec.dims, coords[:, :s], vals[:s], init, mode)
    dt = time.perf_counter() - t0
    s = int(min(coords.shape[1], max(s, s * seconds / max(dt, 1e-9))))
    t0 = time.perf_counter()
    for mode in range(N):
        oracle.mttkrp(rec.dims, coords[:, :s], vals[:s], init, mode)
    dt = time.perf_counter() - t0
    return {"value": s * N / dt, "unit": "nnz/s", "cores": 1, "kind": "oracle",
            "sample": f"first {s} COO draws of {rec.name}, MTTKRP on all {N} modes, FP64 COO loop, "
                      f"{dt:.1f} s"}


if __name__ == "__main__":
    main()
