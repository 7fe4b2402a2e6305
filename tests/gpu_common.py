"""Helpers shared by the GPU parity tests (inputs from synth, expectations from oracle)."""
import numpy as np

import oracle
import synth


def torch():
    import torch as _t
    return _t


def gpu_ok():
    try:
        import torch as _t
        return _t.cuda.is_available()
    except Exception:
        return False


def to_dev(coords, vals):
    t = torch()
    c = t.from_numpy(np.ascontiguousarray(coords).view(np.int32)).cuda()
    v = t.from_numpy(np.ascontiguousarray(vals, np.float32)).cuda()
    return c, v


def factors_dev(fs, dtype="f32"):
    t = torch()
    out = []
    for f in fs:
        x = t.from_numpy(np.ascontiguousarray(f, np.float32)).cuda()
        out.append(x.to(t.bfloat16) if dtype == "bf16" else x)
    return out


def keys_numpy(keys_dev, key_bits):
    k = keys_dev.cpu().numpy()
    if key_bits == 32:
        lo = k.view(np.uint32).astype(np.uint64)
        return lo, np.zeros_like(lo)
    if key_bits == 64:
        return k.view(np.uint64), np.zeros(k.shape, np.uint64)
    k = k.view(np.uint64)
    return np.ascontiguousarray(k[:, 0]), np.ascontiguousarray(k[:, 1])


def oracle_alto(dims, coords, vals):
    """Oracle linearized, ordered and coalesced tensor: ((lo, hi), vals f64, layout)."""
    lay = oracle.layout(dims)
    lo, hi = oracle.encode(lay, coords)
    perm = oracle.sort_perm((lo, hi))
    (ulo, uhi), uv = oracle.coalesce((lo[perm], hi[perm]), np.asarray(vals, np.float64)[perm])
    return (ulo, uhi), uv, lay, perm


def rel_fro(got, ref):
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    den = np.linalg.norm(ref)
    return np.linalg.norm(got - ref) / (den if den > 0 else 1.0)


def small(name, nnz):
    return synth.scaled(synth.WORKLOADS[name], nnz, "_%d" % nnz)
