"""Benchmark: ALTO sparse MTTKRP / CP-ALS on one MI355X.

One step = the whole hot path over one synthetic tensor, inputs already in
HBM: alto_build (linearize, radix-sort, coalesce, partition, intervals,
coverage) followed by CP-ALS (per mode: strategy choice, MTTKRP, merge,
FP64 normal equations) for the configured number of iterations.

value = MTTKRP nonzeros processed per second over the whole step
        (iterations x modes x distinct nonzeros / step time).

Extra fields: per-mode MTTKRP nnz/s, logical GB/s and % of the 8 TB/s HBM
peak (FP32 and BF16 factors), CP-ALS ms per iteration (FP32 vs BF16),
build time, fits; `roofline` for the MTTKRP kernel; `cpu_baseline` (the
FP64 oracle on a bounded sample, one host core).

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
    ap.add_argument("--reps", type=int, default=20, help="timed repetitions per mode for per-mode MTTKRP")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="target oracle CPU time")
    ap.add_argument("--mttkrp-only", action="store_true",
                    help="only the per-mode MTTKRP repetitions (for counter collection)")
    return ap.parse_args()


def logical_bytes_per_nnz(N, R, key_bits, fbytes):
    """Algorithmic bytes one nonzero moves in a mode-n MTTKRP: its index and
    value, N-1 gathered factor rows, and its R-wide FP32 output update."""
    return key_bits / 8 + 4 + (N - 1) * R * fbytes + 4 * R


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
    rec = synth.WORKLOADS[args.workload]
    R = rec.rank
    t0 = time.time()
    coords, vals = synth.coo(rec)
    print(f"[bench] generated {rec.name}: {coords.shape[1]} draws in {time.time() - t0:.1f}s", file=sys.stderr,
          flush=True)
    c_dev = torch.from_numpy(coords.view(np.int32)).to(dev)
    v_dev = torch.from_numpy(vals).to(dev)
    init = synth.factors(rec.seed + 1, rec.dims, R)
    init_f32 = [torch.from_numpy(f).to(dev) for f in init]
    init_bf16 = [f.to(torch.bfloat16) for f in init_f32]
    work_f32 = [f.clone() for f in init_f32]
    work_bf16 = [f.clone() for f in init_bf16]
    N = len(rec.dims)
    torch.cuda.synchronize()

    def step(prec="f32", timers=None):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)] if timers is not None else None
        work = work_f32 if prec == "f32" else work_bf16
        src = init_f32 if prec == "f32" else init_bf16
        for w, s in zip(work, src):
            w.copy_(s)
        if ev:
            ev[0].record()
        t = alto.AltoTensor.build(c_dev, v_dev, rec.dims)
        if ev:
            ev[1].record()
        lam, fit = t.cp_als(work, args.iters)
        if ev:
            ev[2].record()
        info = t.info()
        t.close()
        if timers is not None:
            torch.cuda.synchronize()
            timers.append((ev[0].elapsed_time(ev[1]), ev[1].elapsed_time(ev[2])))
        return info, fit

    if args.mttkrp_only:
        t = alto.AltoTensor.build(c_dev, v_dev, rec.dims)
        per_mode = time_modes(alto, torch, t, init_f32, R, N, args.reps, "f32")
        print(json.dumps({"mttkrp_only": per_mode}))
        t.close()
        return

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = []
    for _ in range(args.steps):
        infos.append(step())
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    info, fit_f32 = infos[-1]
    M = info["nnz"]
    ms_per_step = 1e3 * elapsed / args.steps
    value = args.iters * N * M / (elapsed / args.steps)

    # build / CP-ALS split (FP32 and BF16 factors), event-timed
    tim_f32, tim_bf16 = [], []
    step("f32", tim_f32)
    _, fit_bf16 = step("bf16", tim_bf16)

    # per-mode MTTKRP on the built tensor
    t = alto.AltoTensor.build(c_dev, v_dev, rec.dims)
    per_f32 = time_modes(alto, torch, t, init_f32, R, N, args.reps, "f32")
    per_bf16 = time_modes(alto, torch, t, init_bf16, R, N, args.reps, "bf16")
    kb = t.info()["key_bits"]
    t.close()

    # roofline of the MTTKRP (the dominant kernel): algorithmic bytes per
    # launch over the mean launch time, all modes pooled
    tot_bytes = sum(m["logical_bytes"] for m in per_f32)
    tot_ms = sum(m["ms"] for m in per_f32)
    achieved = tot_bytes / (tot_ms * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                "kernel": "mttkrp_k (FP32 factors, all modes, mean per launch)"}

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
            "parallelism": "single GPU",
        },
        "roofline": roofline,
        "cpu_baseline": cpu,
        "per_mode_f32": per_f32,
        "per_mode_bf16": per_bf16,
        "build_ms": float(np.mean([a for a, _ in tim_f32])),
        "cp_als_ms_per_iter_f32": float(np.mean([b for _, b in tim_f32])) / args.iters,
        "cp_als_ms_per_iter_bf16": float(np.mean([b for _, b in tim_bf16])) / args.iters,
        "fit_f32": float(fit_f32[-1]) if len(fit_f32) else None,
        "fit_bf16": float(fit_bf16[-1]) if len(fit_bf16) else None,
    }
    print(json.dumps(out))


def time_modes(alto, torch, t, factors, R, N, reps, prec):
    info = t.info()
    M = info["nnz"]
    fb = 4 if prec == "f32" else 2
    res = []
    for mode in range(N):
        out = torch.empty((info["dims"][mode], R), dtype=torch.float32, device=factors[0].device)
        strat, L = t.select(mode, R, prec)
        t.mttkrp(factors, mode, out=out)  # warmup (plans the segment lists)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            t.mttkrp(factors, mode, out=out)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        lb = logical_bytes_per_nnz(N, R, info["key_bits"], fb) * M
        res.append({"mode": mode, "strategy": strat, "ms": ms, "nnz_per_s": M / (ms * 1e-3),
                    "logical_bytes": lb, "logical_GBps": lb / (ms * 1e-3) / 1e9,
                    "pct_hbm_peak": 100.0 * lb / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS})
        print(f"[bench] mode {mode} {prec} {strat}: {ms:.3f} ms, {M / (ms * 1e-3) / 1e9:.2f} G nnz/s, "
              f"{res[-1]['pct_hbm_peak']:.1f}% of HBM peak (logical bytes)", file=sys.stderr, flush=True)
    return res


def cpu_baseline(rec, coords, vals, init, R, N, seconds):
    """The FP64 oracle's COO MTTKRP (one host core) on the first S draws of
    the same tensor, all modes; S sized for about `seconds` of work."""
    import oracle
    oracle.build(force=False)
    init = [np.asarray(f, np.float64) for f in init]
    s = 20000
    t0 = time.perf_counter()
    for mode in range(N):
        oracle.mttkrp(rec.dims, coords[:, :s], vals[:s], init, mode)
    dt = time.perf_counter() - t0
    per_nnz_mode = dt / (s * N)
    s = int(min(coords.shape[1], max(s, seconds / max(per_nnz_mode * N, 1e-12))))
    t0 = time.perf_counter()
    for mode in range(N):
        oracle.mttkrp(rec.dims, coords[:, :s], vals[:s], init, mode)
    dt = time.perf_counter() - t0
    return {"value": s * N / dt, "unit": "nnz/s", "cores": 1, "kind": "oracle",
            "sample": f"first {s} COO draws of {rec.name}, MTTKRP on all {N} modes, FP64 COO loop, "
                      f"{dt:.1f} s"}


if __name__ == "__main__":
    main()
