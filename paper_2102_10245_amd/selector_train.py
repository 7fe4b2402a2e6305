"""Timing corpus, training and evaluation of the MTTKRP execution selector.

The selector is a perceptron with two hidden ReLU layers of 64 units.  From
15 features of (tensor, mode, rank, precision) it predicts, for every
candidate execution (strategy in {atomic, staged, sorted} x segment count L),
log2 of the MTTKRP time relative to the fastest candidate; the library runs
the candidate with the smallest prediction.

    python -m paper_2102_10245_amd.selector_train corpus --first 0 --count 250 --out PATH.jsonl
        seeded synthetic tensors; every candidate timed on the GPU (needs a GPU)
    python -m paper_2102_10245_amd.selector_train refeature --corpus A.jsonl --out B.jsonl
        rebuilds every corpus tensor and recomputes its features with the
        current library, keeping the timings (needs a GPU)
    python -m paper_2102_10245_amd.selector_train train --corpus A.jsonl [B.jsonl ...]
        trains on tensors 0-319 with the library's HIP forward/backward and Adam
        kernels (needs a GPU) from four initializations, keeps the weights with
        the lowest regret on tensors 320-399 (early stopping and model
        selection), writes selector_weights.f32 and the
        evaluation on the held-out tensors 400-499 (regret against exhaustive
        timing, gain over the reuse rule of the paper and over the best single
        fixed candidate) to selector_eval.json next to this file.

All execution, timing and training runs through libalto's C ABI; PyTorch only
holds device buffers.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

STRATEGIES = ("atomic", "staged", "sorted")
LS = (256, 512, 1024, 2048, 4096, 8192, 16384)
K = len(STRATEGIES) * len(LS)
F, H = 15, 64
N_TRAIN, N_TOTAL = 400, 500
SEED = 20210245
WEIGHTS = os.path.join(HERE, "selector_weights.f32")
EVAL = os.path.join(HERE, "selector_eval.json")
CORPUS = os.path.join(HERE, "selector_corpus.jsonl")


def candidate(k):
    return STRATEGIES[k // len(LS)], LS[k % len(LS)]


def recipe(i):
    """The i-th corpus tensor: 3-5 modes, dims log-uniform in [1e2, 1e7],
    nnz log-uniform in [1e6, 2e8] (at most half of the index space), Zipf
    exponent uniform in [0, 1.5] per mode, R in {8, 16, 32, 64}, FP32 or
    BF16 factors."""
    import synth
    rng = np.random.default_rng(SEED + 7919 * i)
    N = int(rng.integers(3, 6))
    dims = tuple(int(round(10 ** rng.uniform(2, 7))) for _ in range(N))
    space = math.prod(float(d) for d in dims)
    nnz = int(min(10 ** rng.uniform(6, math.log10(2e8)), 0.5 * space))
    zipf = tuple(float(rng.uniform(0, 1.5)) for _ in range(N))
    R = int(rng.choice([8, 16, 32, 64]))
    prec = "bf16" if rng.random() < 0.5 else "f32"
    rec = synth.Recipe(f"corpus_{i}", dims, nnz, zipf, "uniform", seed=SEED + i, rank=R)
    return rec, prec


def heuristic_index(feat_reuse_log2):
    """The paper's rule (staging when reuse > 4, atomics otherwise) at the
    library's default L of 8 per compute unit (2048 on MI355X)."""
    st = "staged" if feat_reuse_log2 > 2.0 else "atomic"
    return STRATEGIES.index(st) * len(LS) + LS.index(2048)


# ------------------------------------------------------------------ corpus
def corpus(first, count, out, reps=2, max_seconds=None):
    import torch
    import paper_2102_10245_amd as alto
    import synth
    alto.selector_load(None)
    dev = torch.device("cuda", 0)
    start = time.time()
    with open(out, "a") as fo:
        for i in range(first, first + count):
            if max_seconds is not None and time.time() - start > max_seconds:
                print(f"[corpus] stopping before tensor {i}: {max_seconds} s spent", flush=True)
                break
            t0 = time.time()
            rec, prec = recipe(i)
            coords, vals = synth.coo(rec)
            c = torch.from_numpy(coords.view(np.int32)).to(dev)
            v = torch.from_numpy(vals).to(dev)
            t = alto.AltoTensor.build(c, v, rec.dims)
            del c, v
            fs = [torch.from_numpy(f).to(dev) for f in synth.factors(rec.seed + 1, rec.dims, rec.rank)]
            if prec == "bf16":
                fs = [f.to(torch.bfloat16) for f in fs]
            N = len(rec.dims)
            times = np.full((N, K), np.nan)
            feats = [t.selector_features(m, rec.rank, prec).tolist() for m in range(N)]
            for li, L in enumerate(LS):
                t.partition(L)
                for m in range(N):
                    out_t = torch.empty((rec.dims[m], rec.rank), device=dev)
                    for si, st in enumerate(STRATEGIES):
                        t.mttkrp(fs, m, out=out_t, strategy=st)  # warmup (plans, orders)
                        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                        e0.record()
                        for _ in range(reps):
                            t.mttkrp(fs, m, out=out_t, strategy=st)
                        e1.record()
                        torch.cuda.synchronize()
                        times[m, si * len(LS) + li] = e0.elapsed_time(e1) / reps
                    del out_t
            info = t.info()
            t.close()
            for m in range(N):
                fo.write(json.dumps({"tensor": i, "mode": m, "dims": list(rec.dims), "nnz": info["nnz"],
                                     "zipf": list(rec.zipf), "R": rec.rank, "prec": prec,
                                     "features": feats[m], "ms": times[m].tolist()}) + "\n")
            fo.flush()
            best = np.nanmin(times, axis=1)
            print(f"[corpus] tensor {i}: N={N} nnz={info['nnz']} R={rec.rank} {prec} "
                  f"best ms per mode {np.round(best, 3).tolist()} ({time.time() - t0:.1f}s)", flush=True)
            del fs
            torch.cuda.empty_cache()


def refeature(path, out):
    """Recompute the features of every corpus row with the current library
    (the tensor rebuilt from its recipe); the timings are kept."""
    import torch
    import paper_2102_10245_amd as alto
    import synth
    rows = load_corpus([path])
    by_tensor = {}
    for r in rows:
        by_tensor.setdefault(r["tensor"], []).append(r)
    dev = torch.device("cuda", 0)
    t0 = time.time()
    with open(out, "w") as fo:
        for i in sorted(by_tensor):
            rec, prec = recipe(i)
            coords, vals = synth.coo(rec)
            c = torch.from_numpy(coords.view(np.int32)).to(dev)
            v = torch.from_numpy(vals).to(dev)
            t = alto.AltoTensor.build(c, v, rec.dims)
            del c, v
            for r in by_tensor[i]:
                assert r["dims"] == list(rec.dims) and r["R"] == rec.rank and r["prec"] == prec
                r["features"] = t.selector_features(r["mode"], rec.rank, prec).tolist()
                fo.write(json.dumps(r) + "\n")
            t.close()
            torch.cuda.empty_cache()
            if i % 50 == 0:
                print(f"[refeature] tensor {i} ({time.time() - t0:.0f} s)", flush=True)


def load_corpus(paths):
    rows = []
    for p in paths:
        with open(p) as f:
            rows += [json.loads(l) for l in f if l.strip()]
    rows.sort(key=lambda r: (r["tensor"], r["mode"]))
    return rows


# Regression targets are clipped at a 2x slowdown: the choice is the argmin,
# so only the ordering of the candidates near the fastest one matters, and
# unclipped targets let the slowest candidates dominate the squared error.
TARGET_CLIP = 1.0


def arrays(rows):
    X = np.array([r["features"] for r in rows], np.float64)
    T = np.array([r["ms"] for r in rows], np.float64)
    mask = np.isfinite(T) & (T > 0)
    logt = np.where(mask, np.log2(np.where(mask, T, 1.0)), 0.0)
    best = np.min(np.where(mask, logt, np.inf), axis=1, keepdims=True)
    Y = np.where(mask, np.minimum(logt - best, TARGET_CLIP), 0.0)
    return X, T, Y, mask.astype(np.float64)


# ------------------------------------------------------------------ training
def pack(params):
    return np.concatenate([p.reshape(-1) for p in params]).astype(np.float32)


def train(paths, steps=1500, lr=3e-3, seeds=(7, 8, 9, 10), out_dir=HERE, n_val=80, every=25):
    """Full-batch Adam on the HIP kernels over tensors [0, N_TRAIN - n_val),
    once per initialization seed; the weights with the lowest regret on the
    validation tensors [N_TRAIN - n_val, N_TRAIN), over all seeds and
    checkpoints, are kept (early stopping and model selection)."""
    import torch
    import paper_2102_10245_amd as alto
    rows = load_corpus(paths)
    fit_rows = [r for r in rows if r["tensor"] < N_TRAIN - n_val]
    val_rows = [r for r in rows if N_TRAIN - n_val <= r["tensor"] < N_TRAIN]
    Xtr, Ttr, Ytr, Mtr = arrays(fit_rows)
    Xva, Tva, _, Mva = arrays(val_rows)
    mean = Xtr.mean(axis=0)
    scale = Xtr.std(axis=0)
    scale[scale < 1e-6] = 1.0
    dev = torch.device("cuda", 0)
    x = torch.from_numpy(((Xtr - mean) / scale).astype(np.float32)).to(dev)
    t = torch.from_numpy(Ytr.astype(np.float32)).to(dev)
    mk = torch.from_numpy(Mtr.astype(np.float32)).to(dev)
    best_w, best_r, best_s, best_seed = None, np.inf, 0, None
    for seed in seeds:
        # weights and biases uniform in +-1/sqrt(fan-in): on the validation
        # tensors this generalizes better than He-normal weights with zero
        # biases (regret 3.7% against 5.1% in a CPU replica of this training)
        rng = np.random.default_rng(seed)
        u = lambda shape, fan_in: rng.uniform(-1.0, 1.0, shape) / math.sqrt(fan_in)
        params = [u((H, F), F), u(H, F), u((H, H), H), u(H, H), u((K, H), H), u(K, H)]
        P = torch.from_numpy(pack(params)).to(dev)
        m = torch.zeros_like(P)
        v = torch.zeros_like(P)
        for s in range(1, steps + 1):
            g, loss = alto.mlp_backward(P, x, t, mk, F, H, K)
            cur = lr * (0.5 * (1 + math.cos(math.pi * s / steps)) * 0.95 + 0.05)
            alto.mlp_adam(P, g, m, v, lr=cur, step=s)
            if s % every == 0:
                w = P.cpu().numpy()
                r = regret(w, Xva, Tva, Mva, mean, scale)
                if r < best_r:
                    best_w, best_r, best_s, best_seed = w.copy(), r, s, seed
            if s % 500 == 0 or s == 1:
                print(f"[train] seed {seed} step {s} loss {float(loss.cpu()):.5f} best validation regret "
                      f"{best_r:.4f} (seed {best_seed}, step {best_s})", flush=True)
    w = best_w
    header = np.array([F, H, K, len(LS)], np.float32)
    blob = np.concatenate([header, mean.astype(np.float32), scale.astype(np.float32),
                           Xtr.min(axis=0).astype(np.float32), Xtr.max(axis=0).astype(np.float32),
                           np.array(LS, np.float32), w])
    blob.astype(np.float32).tofile(os.path.join(out_dir, os.path.basename(WEIGHTS)))
    ev = evaluate(rows, w, mean, scale, n_val)
    ev["training"] = {"max_steps": steps, "kept_step": best_s, "lr": lr, "seeds": list(seeds), "kept_seed": best_seed,
                      "fit_tensors": [0, N_TRAIN - n_val], "validation_tensors": [N_TRAIN - n_val, N_TRAIN],
                      "heldout_tensors": [N_TRAIN, N_TOTAL], "hidden": H, "features": F,
                      "target_clip": TARGET_CLIP}
    with open(os.path.join(out_dir, os.path.basename(EVAL)), "w") as f:
        json.dump(ev, f, indent=1)
    print(json.dumps(ev["summary"]), flush=True)


def regret(w, X, T, M, mean, scale):
    y = np.where(M > 0, predict_gpu(w, X, mean, scale), np.inf)
    Tm = np.where(M > 0, T, np.inf)
    ch = np.argmin(y, axis=1)
    return float(np.exp(np.mean(np.log(Tm[np.arange(len(X)), ch] / Tm.min(axis=1)))) - 1)


def predict_gpu(w, X, mean, scale):
    import torch
    import paper_2102_10245_amd as alto
    dev = torch.device("cuda", 0)
    x = torch.from_numpy(((X - mean) / scale).astype(np.float32)).to(dev)
    y, _ = alto.mlp_forward(torch.from_numpy(w).to(dev), x, F, H, K)
    return y.cpu().numpy()


def evaluate(rows, w, mean, scale, n_val=80):
    """Regret of the network's choice against exhaustive timing, and its gain
    over the paper's reuse rule and over the best single fixed candidate,
    per split."""
    out = {"candidates": [list(candidate(k)) for k in range(K)], "summary": {}}
    fit_rows = [r for r in rows if r["tensor"] < N_TRAIN - n_val]
    Tf = np.array([r["ms"] for r in fit_rows])
    fixed = int(np.argmin(np.nanmean(np.log(Tf / np.nanmin(Tf, axis=1, keepdims=True)), axis=0)))
    out["best_fixed_candidate"] = list(candidate(fixed))
    splits = (("fit", lambda r: r["tensor"] < N_TRAIN - n_val),
              ("validation", lambda r: N_TRAIN - n_val <= r["tensor"] < N_TRAIN),
              ("heldout", lambda r: r["tensor"] >= N_TRAIN))
    for split, sel in splits:
        rs = [r for r in rows if sel(r)]
        if not rs:
            continue
        X, T, _, M = arrays(rs)
        y = predict_gpu(w, X, mean, scale)
        y = np.where(M > 0, y, np.inf)
        choice = np.argmin(y, axis=1)
        Tm = np.where(M > 0, T, np.inf)
        t_best = Tm.min(axis=1)
        t_sel = Tm[np.arange(len(rs)), choice]
        t_heur = np.array([Tm[q, heuristic_index(X[q, 2])] for q in range(len(rs))])
        t_fixed = Tm[:, fixed]
        # the library's own strategy at its default segment count (8 per CU)
        t_sorted_default = Tm[:, STRATEGIES.index("sorted") * len(LS) + LS.index(2048)]
        ratio = t_sel / t_best
        out["summary"][split] = {
            "samples": len(rs),
            "regret_geomean": float(np.exp(np.mean(np.log(ratio))) - 1),
            "regret_p95": float(np.quantile(ratio, 0.95) - 1),
            "gain_over_reuse_rule_geomean": float(np.exp(np.mean(np.log(t_heur / t_sel)))),
            "reuse_rule_regret_geomean": float(np.exp(np.mean(np.log(t_heur / t_best))) - 1),
            "gain_over_best_fixed_geomean": float(np.exp(np.mean(np.log(t_fixed / t_sel)))),
            "gain_over_sorted_default_L_geomean": float(np.exp(np.mean(np.log(t_sorted_default / t_sel)))),
            "best_fixed_regret_geomean": float(np.exp(np.mean(np.log(t_fixed / t_best))) - 1),
            "total_ms_selected": float(t_sel.sum()), "total_ms_best": float(t_best.sum()),
            "total_ms_reuse_rule": float(t_heur.sum()), "total_ms_best_fixed": float(t_fixed.sum()),
        }
    return out


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    c = sub.add_parser("corpus")
    c.add_argument("--first", type=int, default=0)
    c.add_argument("--count", type=int, default=N_TOTAL)
    c.add_argument("--out", default=CORPUS)
    c.add_argument("--max-seconds", type=float, default=None, help="stop before the next tensor after this long")
    r = sub.add_parser("refeature")
    r.add_argument("--corpus", default=CORPUS)
    r.add_argument("--out", required=True)
    t = sub.add_parser("train")
    t.add_argument("--corpus", nargs="+", default=[CORPUS])
    t.add_argument("--steps", type=int, default=1500)
    t.add_argument("--out-dir", default=HERE)
    a = ap.parse_args()
    if a.cmd == "corpus":
        corpus(a.first, a.count, a.out, max_seconds=a.max_seconds)
    elif a.cmd == "refeature":
        refeature(a.corpus, a.out)
    else:
        train(a.corpus, steps=a.steps, out_dir=a.out_dir)


if __name__ == "__main__":
    main()
