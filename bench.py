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
compulsory bytes (each nonzero's index and value, each factor row and each
output row moved once) for every strategy, FP32 and BF16 factors; CP-ALS ms
per iteration and fit for the plain FP32 form (reuse rule, no network), the
network-chosen FP32 and BF16 forms and FP32 / BF16 under one fixed plan;
`roofline` for the MTTKRP kernel (compulsory bytes over the mean launch
time, with the counter-measured HBM traffic beside it); `cpu_baseline` (the
FP64 oracle on a bounded sample, all host cores and one core); the
alto_build time and the device memory the tensor handle holds.

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
    ap.add_argument("--prec", default="f32", choices=("f32", "bf16"),
                    help="factor precision of the --mttkrp-only repetitions")
    ap.add_argument("--plan", default="auto",
                    help="plan of the --mttkrp-only repetitions: auto (the library's choice) or "
                         "STRATEGY:L, e.g. sorted:512, one plan for every mode")
    ap.add_argument("--format", action="store_true",
                    help="format generation and storage on every workload: alto_build time and index "
                         "bytes vs COO (prints its own JSON line instead of the benchmark line)")
    return ap.parse_args()


def logical_bytes_per_nnz(N, R, key_bits, fbytes):
    """Algorithmic bytes one nonzero moves in a mode-n MTTKRP: its index and
    value, N-1 gathered factor rows, and its R-wide FP32 output update."""
    return key_bits / 8 + 4 + (N - 1) * R * fbytes + 4 * R


def compulsory_bytes(info, R, fbytes, mode):
    """The least HBM traffic a mode-n MTTKRP can have: every nonzero's index
    and value read once, every factor row of the other modes read once, and
    every output row written once."""
    dims = info["dims"]
    return (info["nnz"] * (info["key_bits"] / 8 + 4)
            + sum(d * R * fbytes for m, d in enumerate(dims) if m != mode) + dims[mode] * R * 4)


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

    def step(prec="f32", timers=None, strategy="auto", num_segments=0):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)] if timers is not None else None
        for w, s in zip(work[prec], src[prec]):
            w.copy_(s)
        if ev:
            ev[0].record()
        t = alto.AltoTensor.build(c_dev, v_dev, rec.dims)
        if ev:
            ev[1].record()
        lam, fit = t.cp_als(work[prec], args.iters, strategy=strategy, num_segments=num_segments)
        if ev:
            ev[2].record()
        info = t.info()
        plan = ([t.select(m, R, prec) for m in range(N)] if strategy == "auto"
                else [(strategy, num_segments or info["num_segments"])] * N)
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
        fs = init_f32 if args.prec == "f32" else init_bf16
        st, _, L = args.plan.partition(":")
        per_mode = time_modes(alto, torch, t, fs, R, N, args.reps, args.prec, st, int(L or 0))
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

    # the forms: network-chosen FP32 / BF16, the plain FP32 form (reuse rule,
    # no network), and FP32 / BF16 under one fixed plan (sorted, L = 512)
    forms = {}
    for name, prec, sel, st, L in (("selector_f32", "f32", have_sel, "auto", 0),
                                   ("selector_bf16", "bf16", have_sel, "auto", 0),
                                   ("plain_f32", "f32", False, "auto", 0),
                                   ("fixed_sorted512_f32", "f32", have_sel, "sorted", 512),
                                   ("fixed_sorted512_bf16", "bf16", have_sel, "sorted", 512)):
        if not sel:
            alto.selector_load(None)
        tim = []
        finfo, fit, plan = step(prec, tim, st, L)
        if have_sel:
            alto.load_default_selector()
        forms[name] = {"build_ms": tim[0][0], "cp_als_ms_per_iter": tim[0][1] / args.iters,
                       "fit": float(fit[-1]) if len(fit) else None,
                       "plan": [{"strategy": s, "num_segments": L} for s, L in plan],
                       "device_bytes": {k: finfo[k] for k in ("tensor_bytes", "partition_bytes", "order_bytes",
                                                              "scratch_bytes")}}
        log(f"{name}: CP-ALS {tim[0][1] / args.iters:.2f} ms/iter, fit {forms[name]['fit']:.6f}, plan {plan}")

    # per-mode MTTKRP for every strategy and precision on the built tensor
    t = alto.AltoTensor.build(c_dev, v_dev, rec.dims)
    per_mode = {}
    for prec, fs in (("f32", init_f32), ("bf16", init_bf16)):
        # the fixed strategies at the library's default segment count (8 per CU)
        for st in ("auto", "atomic", "staged", "sorted"):
            per_mode[f"{st}_{prec}"] = time_modes(alto, torch, t, fs, R, N, args.reps, prec, st,
                                                  0 if st == "auto" else 8 * alto.compute_units())
    kb = t.info()["key_bits"]
    t.close()

    # roofline of the MTTKRP kernel under the chosen FP32 plan: compulsory
    # HBM bytes per launch over the mean launch time (all modes pooled)
    main_modes = per_mode["auto_f32"]
    tot_bytes = sum(m["compulsory_bytes"] for m in main_modes)
    tot_logical = sum(m["logical_bytes"] for m in main_modes)
    tot_ms = sum(m["kernel_ms"] for m in main_modes)
    tot_call_ms = sum(m["ms"] for m in main_modes)
    achieved = tot_bytes / (tot_ms * 1e-3) / 1e9
    traffic = measured_traffic(rec.name)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "bytes": "compulsory: nnz*(W/8+4) + sum over other modes I_m*R*4 + I_n*R*4 per launch",
                "compulsory_bytes_per_launch": round(tot_bytes / N),
                "mean_launch_ms": tot_ms / N,
                "timing": "HIP events recorded by the library on the launch stream around the MTTKRP kernels "
                          "of each call (alto_timing_enable / alto_timing_read)",
                "mean_call_ms": tot_call_ms / N,
                "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, calibrated)",
                "traffic_frac": (round(traffic / (tot_ms / N * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
                                 if traffic else None),
                "logical_GBps": round(tot_logical / (tot_ms * 1e-3) / 1e9, 1),
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
        "build_ms": forms["selector_f32"]["build_ms"],
        "footprint": {**forms["selector_f32"]["device_bytes"], "coo_input_bytes": rec.nnz * (4 * N + 4),
                      "note": "device bytes the tensor handle holds after the FP32 CP-ALS of one step"},
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


def time_modes(alto, torch, t, factors, R, N, reps, prec, strategy, num_segments=0):
    info = t.info()
    M = info["nnz"]
    fb = 4 if prec == "f32" else 2
    res = []
    for mode in range(N):
        out = torch.empty((info["dims"][mode], R), dtype=torch.float32, device=factors[0].device)
        strat, L = t.select(mode, R, prec) if strategy == "auto" else (strategy, num_segments)
        t.mttkrp(factors, mode, out=out, strategy=strategy, num_segments=num_segments)  # warmup (plans, orders)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        alto.timing_read()
        alto.timing_enable(True)
        e0.record()
        for _ in range(reps):
            t.mttkrp(factors, mode, out=out, strategy=strategy, num_segments=num_segments)
        e1.record()
        torch.cuda.synchronize()
        alto.timing_enable(False)
        ms = e0.elapsed_time(e1) / reps
        # the MTTKRP kernels alone: the library's event pair around them on
        # the launch stream (output clear and launch gaps excluded)
        k_ms, k_n = alto.timing_read()
        kernel_ms = k_ms / k_n if k_n == reps else None
        lb = logical_bytes_per_nnz(N, R, info["key_bits"], fb) * M
        cb = compulsory_bytes(info, R, fb, mode)
        res.append({"mode": mode, "strategy": strat, "num_segments": L or info["num_segments"], "ms": ms,
                    "kernel_ms": kernel_ms, "nnz_per_s": M / (ms * 1e-3), "compulsory_bytes": cb,
                    "pct_hbm_peak": 100.0 * cb / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                    "logical_bytes": lb, "logical_GBps": lb / (ms * 1e-3) / 1e9})
        log(f"mode {mode} {prec} {strategy}->{strat}: {ms:.3f} ms, {M / (ms * 1e-3) / 1e9:.2f} G nnz/s, "
            f"{res[-1]['pct_hbm_peak']:.1f}% of HBM peak (compulsory bytes)")
    return res


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(rec, coords, vals, init, R, N, seconds):
    """The FP64 oracle's COO MTTKRP on the first S draws of the same tensor,
    all modes: on every host core (OpenMP, thread-private outputs added at
    the end) and on one core, each leg sized for about `seconds` of work."""
    import oracle
    oracle.build(force=False)
    init = [np.asarray(f, np.float64) for f in init]

    def timed(fn, s):
        t0 = time.perf_counter()
        for mode in range(N):
            fn(rec.dims, coords[:, :s], vals[:s], init, mode)
        return time.perf_counter() - t0

    def leg(fn, s0):
        # two probes separate the per-call cost (thread-private outputs of
        # I_n x R doubles are cleared and added up) from the per-nonzero one
        d0, d1 = timed(fn, s0), timed(fn, 4 * s0)
        per_nnz = max((d1 - d0) / (3 * s0), 1e-12)
        fixed = max(d0 - per_nnz * s0, 0.0)
        s = int(min(coords.shape[1], max(4 * s0, (seconds - fixed) / per_nnz)))
        used = 1
        t0 = time.perf_counter()
        for mode in range(N):
            r = fn(rec.dims, coords[:, :s], vals[:s], init, mode)
            if isinstance(r, tuple):
                used = r[1]
        dt = time.perf_counter() - t0
        return s, dt, used

    s_all, dt_all, threads = leg(oracle.mttkrp_par, 1_000_000)
    s_one, dt_one, _ = leg(oracle.mttkrp, 200_000)
    return {"value": s_all * N / dt_all, "unit": "nnz/s", "cores": threads, "kind": "oracle",
            "sample": f"first {s_all} COO draws of {rec.name}, MTTKRP on all {N} modes, FP64 COO loop on "
                      f"{threads} threads (OpenMP, private outputs), {dt_all:.1f} s",
            "one_core": {"value": s_one * N / dt_one, "unit": "nnz/s", "cores": 1,
                         "sample": f"first {s_one} COO draws, all {N} modes, one thread, {dt_one:.1f} s"},
            "nproc": os.cpu_count(), "cpu_model": cpu_model(),
            "omp_num_threads": os.environ.get("OMP_NUM_THREADS")}


if __name__ == "__main__":
    main()
