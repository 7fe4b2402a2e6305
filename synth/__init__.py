"""Seeded synthetic sparse tensors for tests and benchmarks.

This module only draws inputs (coordinates, values, factor matrices); it
contains none of the tensor method's arithmetic.  The draws come from
``gen.c`` (counter-based SplitMix64, so thread count does not change them),
compiled with gcc into ``libsynth.so`` next to this file.

Workloads are described by :class:`Recipe`; ``WORKLOADS`` holds the named
ones used by the tests and the benchmark.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gen.c")
_LIB = os.path.join(_HERE, "libsynth.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile gen.c into libsynth.so (gcc, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c11",
                               _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        u64, i64, c_int = ctypes.c_uint64, ctypes.c_int64, ctypes.c_int
        vp = ctypes.c_void_p
        lib.synth_words.argtypes = [u64, u64, i64, vp]
        lib.synth_mode_coords.argtypes = [u64, c_int, ctypes.c_uint32, ctypes.c_double, i64, vp]
        lib.synth_mode_coords.restype = c_int
        lib.synth_values.argtypes = [u64, c_int, i64, vp]
        lib.synth_factor.argtypes = [u64, c_int, i64, c_int, vp]
        _lib = lib
    return _lib


def words(seed: int, stream: int, n: int) -> np.ndarray:
    out = np.empty(n, dtype=np.uint64)
    _load().synth_words(seed, stream, n, out.ctypes.data)
    return out


def mode_coords(seed: int, mode: int, dim: int, zipf_s: float, m: int) -> np.ndarray:
    out = np.empty(m, dtype=np.uint32)
    if m:
        rc = _load().synth_mode_coords(seed, mode, dim, float(zipf_s), m, out.ctypes.data)
        if rc != 0:
            raise MemoryError("synth_mode_coords failed")
    return out


def values(seed: int, dist: str, m: int) -> np.ndarray:
    out = np.empty(m, dtype=np.float32)
    if m:
        _load().synth_values(seed, {"uniform": 0, "lognormal": 1}[dist], m, out.ctypes.data)
    return out


def factor(seed: int, mode: int, dim: int, rank: int) -> np.ndarray:
    """I x R float32 matrix with entries k/256, k in 1..255 (exact in bf16)."""
    out = np.empty((dim, rank), dtype=np.float32)
    _load().synth_factor(seed, mode, dim, rank, out.ctypes.data)
    return out


def factors(seed: int, dims, rank: int):
    return [factor(seed, n, int(d), rank) for n, d in enumerate(dims)]


@dataclass
class Recipe:
    """A synthetic sparse tensor: shape, nonzero count, per-mode index
    distribution (Zipf exponent, 0 = uniform), value distribution, seed.

    ``unique=True`` removes repeated coordinates and draws again until
    exactly ``nnz`` distinct coordinates remain (small tensors only: the
    check is a NumPy sort of mixed-radix row numbers).  Otherwise repeated
    coordinates are kept as separate COO entries.
    """
    name: str
    dims: tuple
    nnz: int
    zipf: tuple = ()
    values: str = "uniform"
    seed: int = 20210245
    unique: bool = False
    rank: int = 16
    extra: dict = field(default_factory=dict)

    def zipf_of(self, n: int) -> float:
        return float(self.zipf[n]) if self.zipf else 0.0


def coo(rec: Recipe):
    """Return (coords uint32 [N, M], vals float32 [M]) for a recipe."""
    N = len(rec.dims)
    m = int(rec.nnz)
    coords = np.stack([mode_coords(rec.seed, n, int(rec.dims[n]), rec.zipf_of(n), m)
                       for n in range(N)]) if m else np.zeros((N, 0), np.uint32)
    vals = values(rec.seed, rec.values, m)
    if not rec.unique or m == 0:
        return coords, vals
    return _unique_topup(rec, coords, vals)


def _row_numbers(dims, coords):
    lin = np.zeros(coords.shape[1], dtype=object if np.prod([float(d) for d in dims]) >= 2**63 else np.int64)
    for n, d in enumerate(dims):
        lin = lin * int(d) + coords[n].astype(lin.dtype if lin.dtype != object else np.int64)
    return lin


def _unique_topup(rec: Recipe, coords, vals):
    """Keep first occurrences of each coordinate, then append fresh draws
    (from seed + round) until exactly nnz distinct coordinates exist."""
    N = len(rec.dims)
    m = int(rec.nnz)
    prod = 1
    for d in rec.dims:
        prod *= int(d)
    if prod < m:
        raise ValueError("more unique nonzeros requested than coordinates exist")
    if prod >= 2**63:
        raise ValueError("unique=True needs prod(dims) < 2^63")
    for rnd in range(1, 64):
        lin = _row_numbers(rec.dims, coords)
        _, first = np.unique(lin, return_index=True)
        first.sort()
        coords, vals = coords[:, first], vals[first]
        if coords.shape[1] >= m:
            return np.ascontiguousarray(coords[:, :m]), np.ascontiguousarray(vals[:m])
        need = m - coords.shape[1]
        extra = max(need * 2, 1024)
        s2 = rec.seed + 7919 * rnd
        c2 = np.stack([mode_coords(s2, n, int(rec.dims[n]), rec.zipf_of(n), extra) for n in range(N)])
        v2 = values(s2, rec.values, extra)
        coords = np.concatenate([coords, c2], axis=1)
        vals = np.concatenate([vals, v2])
    raise RuntimeError("could not reach the requested unique count")


def planted_cp(dims, rank: int, support, zipf=(), noise: float = 0.1, seed: int = 20210301):
    """A sparse tensor that is a planted sum of ``rank`` rank-1 terms plus noise.

    Term r lives on a small box: ``support[n]`` distinct rows of mode n, drawn
    with the mode's Zipf exponent (so hot rows are shared by many terms and
    the terms overlap), with weights a_n(i, r) in [0.5, 1.5) on a 2^-8 grid.
    Its nonzeros are the box's cells, valued prod_n a_n(i_n, r); cells that
    several terms reach hold the sum.  Every value is then multiplied by
    (1 + noise * z) with z standard normal, so the tensor is exactly rank
    ``rank`` on its support up to a relative noise of ``noise`` and its best
    rank-``rank`` fit is about 1 - noise.

    Returns (coords uint32 [N, M], vals float32 [M], factors) with distinct
    coordinates in row-major order; factors[n] is the dense I_n x rank
    float64 matrix of the planted weights (zero off the boxes).
    """
    N = len(dims)
    rng = np.random.default_rng(seed)
    # one stream of draws per mode (one row permutation, so the hot rows are
    # the same for every term); term r takes the first support[n] distinct
    # rows of its own stretch of that stream
    stretch = [max(64, 16 * int(k)) for k in support]
    draws = []
    for n in range(N):
        if int(support[n]) > dims[n]:
            raise ValueError("support larger than the mode")
        s = float(zipf[n]) if zipf else 0.0
        draws.append(mode_coords(seed, n, int(dims[n]), s, stretch[n] * rank))
    cells = []
    wts = []
    planted = [np.zeros((int(d), rank), np.float64) for d in dims]
    for r in range(rank):
        rows, w = [], []
        for n in range(N):
            k = int(support[n])
            c = draws[n][r * stretch[n]:(r + 1) * stretch[n]]
            _, first = np.unique(c, return_index=True)
            pick = c[np.sort(first)][:k]
            if pick.size < k:  # a very skewed mode: fill with the lowest unused rows
                rest = np.setdiff1d(np.arange(dims[n], dtype=np.uint32), pick)[:k - pick.size]
                pick = np.concatenate([pick, rest])
            rows.append(pick)
            w.append((128 + rng.integers(0, 256, size=k)) / 256.0)
        for n in range(N):
            planted[n][rows[n], r] = w[n]
        grid = np.meshgrid(*rows, indexing="ij")
        val = w[0]
        for n in range(1, N):
            val = np.multiply.outer(val, w[n])
        cells.append(np.stack([g.reshape(-1) for g in grid]))
        wts.append(val.reshape(-1))
    coords = np.concatenate(cells, axis=1)
    vals = np.concatenate(wts)
    lin = _row_numbers(dims, coords)
    uniq, inv = np.unique(lin, return_inverse=True)
    summed = np.zeros(uniq.shape[0], np.float64)
    np.add.at(summed, inv, vals)
    first = np.zeros(uniq.shape[0], np.int64)
    first[inv[::-1]] = np.arange(inv.shape[0])[::-1]
    coords = np.ascontiguousarray(coords[:, first])
    summed *= 1.0 + noise * rng.standard_normal(summed.shape[0])
    return coords, summed.astype(np.float32), planted


def planted_start(planted, jitter: float, seed: int = 20210302):
    """A CP-ALS starting point near planted factors: each entry is
    planted * (1 + jitter * z) + jitter * u (z standard normal, u uniform in
    [0, 1)), clipped to [0, 2) and put on the grid k/128, k in 0..255, so
    that it is exact in bfloat16 and binary32.  Returns float32 matrices."""
    rng = np.random.default_rng(seed)
    out = []
    for f in planted:
        x = f * (1.0 + jitter * rng.standard_normal(f.shape)) + jitter * rng.random(f.shape)
        k = np.clip(np.rint(x * 128.0), 0, 255)
        out.append((k / 128.0).astype(np.float32))
    return out


# Named workloads (shapes and distributions of the benchmark configurations).
WORKLOADS = {
    # 3-mode uniform tensor, exactly 100k distinct coordinates, R=16
    "uniform3_1000x800x600_100k": Recipe(
        "uniform3_1000x800x600_100k", (1000, 800, 600), 100_000, (0, 0, 0), "uniform",
        seed=20210246, unique=True, rank=16),
    # 3-mode skewed tensor, 50M draws, Zipf(1.1) on modes 0-1, R=16 and 64
    "zipf3_2Mx2Mx20k_50M": Recipe(
        "zipf3_2Mx2Mx20k_50M", (2_000_000, 2_000_000, 20_000), 50_000_000, (1.1, 1.1, 0),
        "uniform", seed=20210247, rank=16),
    # 4-mode skewed tensor, 150M draws, Zipf(1.2) on modes 0-1, lognormal values, R=32
    "zipf4_1Mx100kx10kx500_150M": Recipe(
        "zipf4_1Mx100kx10kx500_150M", (1_000_000, 100_000, 10_000, 500), 150_000_000,
        (1.2, 1.2, 0, 0), "lognormal", seed=20210248, rank=32),
    # 5-mode tensor, 200M draws, Zipf(1.0) on every mode, R=32, 128-bit index
    "zipf5_10Mx5Mx2Mx100kx1k_200M": Recipe(
        "zipf5_10Mx5Mx2Mx100kx1k_200M", (10_000_000, 5_000_000, 2_000_000, 100_000, 1_000),
        200_000_000, (1.0, 1.0, 1.0, 1.0, 1.0), "uniform", seed=20210249, rank=32),
}


def scaled(rec: Recipe, nnz: int, name_suffix: str = "") -> Recipe:
    """Same shape and distributions with a different nonzero count."""
    return Recipe(rec.name + name_suffix, rec.dims, nnz, rec.zipf, rec.values,
                  rec.seed, rec.unique, rec.rank, dict(rec.extra))
