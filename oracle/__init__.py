"""FP64 CPU oracle for ALTO sparse MTTKRP and CP-ALS (test infrastructure).

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg
may import this package.  The product (the HIP library and its binding)
never does.  It wraps ``oracle.c`` (plain C, compiled here with gcc into
``liboracle.so``) through ctypes.

Every function restates a definition from "ALTO: Adaptive Linearized
Storage of Sparse Tensors" (Helal et al., ICS 2021):
  layout / encode / decode ....... Section 3.1 (bit groups, Fig. 4, Eq. 1)
  sort_perm / coalesce ........... Section 3.1 (ordering stage)
  partition / intervals .......... Section 3.2 (equal-nonzero line segments,
                                   mode intervals T_{l,n})
  coverage ....................... Algorithm 2, pull-based accumulation
  mttkrp, mttkrp_rows ............ Section 2.2 and Algorithm 1
  mttkrp_par ..................... the same sum on every host core (timing)
  cp_als ......................... Section 2.2 (CPD-ALS; standard ALS)
  heuristic_staging .............. Section 3.3 (reuse > 4 memory operations)
  storage_bits / ratio ........... Eq. 1 and Eq. 2
  transpose ...................... sparse tensor transposition (the sparse
                                   tensor operations of the related work)
  bf16_round ..................... storage rule for bfloat16 factors
  mlp_forward / mlp_backward ..... selector network (two hidden layers)
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

vp = ctypes.c_void_p
i64 = ctypes.c_int64
c_int = ctypes.c_int


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc into liboracle.so."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=gnu11", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        L.oracle_layout.argtypes = [c_int, vp, vp, vp, vp]
        L.oracle_layout.restype = c_int
        L.oracle_encode.argtypes = [c_int, i64, vp, vp, vp, vp, vp]
        L.oracle_decode.argtypes = [c_int, i64, vp, vp, vp, vp, vp]
        L.oracle_sort_perm.argtypes = [i64, vp, vp, vp]
        L.oracle_sort_perm.restype = c_int
        L.oracle_coalesce.argtypes = [i64, vp, vp, vp, vp, vp, vp]
        L.oracle_coalesce.restype = i64
        L.oracle_partition.argtypes = [i64, c_int, vp]
        L.oracle_partition.restype = c_int
        L.oracle_intervals.argtypes = [c_int, c_int, vp, vp, vp, vp, vp, vp]
        L.oracle_coverage.argtypes = [c_int, c_int, vp, c_int, ctypes.c_uint64, vp]
        L.oracle_mttkrp.argtypes = [c_int, i64, vp, vp, vp, vp, c_int, c_int, vp]
        L.oracle_mttkrp_par.argtypes = [c_int, i64, vp, vp, vp, vp, c_int, c_int, vp]
        L.oracle_mttkrp_par.restype = c_int
        L.oracle_mttkrp_rows.argtypes = [c_int, i64, vp, vp, vp, vp, c_int, c_int, i64, vp, vp]
        L.oracle_mttkrp_rows.restype = c_int
        L.oracle_norm2.argtypes = [c_int, i64, vp, vp]
        L.oracle_norm2.restype = ctypes.c_double
        L.oracle_cp_als.argtypes = [c_int, i64, vp, vp, vp, c_int, c_int, vp, vp, vp]
        L.oracle_cp_als.restype = c_int
        L.oracle_bf16_round.argtypes = [i64, vp, vp, vp]
        L.oracle_heuristic_staging.argtypes = [i64, ctypes.c_uint64]
        L.oracle_heuristic_staging.restype = c_int
        for f in (L.oracle_mlp_forward, L.oracle_mlp_backward):
            f.restype = ctypes.c_double
        L.oracle_mlp_forward.argtypes = [c_int] * 4 + [vp] * 10
        L.oracle_mlp_backward.argtypes = [c_int] * 4 + [vp] * 15
        _lib = L
    return _lib


def _ptrs(arrs):
    a = (ctypes.c_void_p * len(arrs))()
    for n, x in enumerate(arrs):
        a[n] = x.ctypes.data
    return a


def _u32_rows(coords):
    coords = np.asarray(coords)
    return [np.ascontiguousarray(coords[n], dtype=np.uint32) for n in range(coords.shape[0])]


def _key_words(keys):
    """Split integer keys (python ints or uint64 arrays) into (lo, hi) uint64."""
    if isinstance(keys, tuple):
        return (np.ascontiguousarray(keys[0], np.uint64), np.ascontiguousarray(keys[1], np.uint64))
    keys = np.asarray(keys)
    if keys.dtype == object:
        lo = np.array([int(k) & (2**64 - 1) for k in keys], dtype=np.uint64)
        hi = np.array([int(k) >> 64 for k in keys], dtype=np.uint64)
        return lo, hi
    return np.ascontiguousarray(keys, np.uint64), np.zeros(keys.shape, np.uint64)


# ---------------------------------------------------------------- layout
class Layout:
    """ALTO bit layout of a shape: per-mode bit counts and masks (ints)."""

    def __init__(self, dims):
        N = len(dims)
        d = np.array(dims, dtype=np.uint64)
        nb = np.zeros(N, dtype=np.int32)
        lo = np.zeros(N, dtype=np.uint64)
        hi = np.zeros(N, dtype=np.uint64)
        B = _load().oracle_layout(N, d.ctypes.data, nb.ctypes.data, lo.ctypes.data, hi.ctypes.data)
        if B == -1:
            raise ValueError("invalid dims")
        if B == -2:
            raise ValueError("linearized index wider than 128 bits")
        self.dims = tuple(int(x) for x in dims)
        self.N = N
        self.nbits = [int(x) for x in nb]
        self.mask_lo, self.mask_hi = lo, hi
        self.masks = [int(lo[n]) | (int(hi[n]) << 64) for n in range(N)]
        self.B = int(B)
        self.W = 32 if self.B <= 32 else (64 if self.B <= 64 else 128)


def layout(dims) -> Layout:
    return Layout(dims)


def encode(lay: Layout, coords):
    """Linearized index of every nonzero, as (lo, hi) uint64 arrays."""
    rows = _u32_rows(coords)
    M = rows[0].shape[0] if rows else 0
    lo = np.zeros(M, np.uint64)
    hi = np.zeros(M, np.uint64)
    _load().oracle_encode(lay.N, M, _ptrs(rows), lay.mask_lo.ctypes.data, lay.mask_hi.ctypes.data,
                          lo.ctypes.data, hi.ctypes.data)
    return lo, hi


def decode(lay: Layout, keys):
    lo, hi = _key_words(keys)
    M = lo.shape[0]
    out = [np.zeros(M, np.uint32) for _ in range(lay.N)]
    _load().oracle_decode(lay.N, M, lo.ctypes.data, hi.ctypes.data, lay.mask_lo.ctypes.data,
                          lay.mask_hi.ctypes.data, _ptrs(out))
    return np.stack(out) if out else np.zeros((0, M), np.uint32)


def sort_perm(keys):
    lo, hi = _key_words(keys)
    perm = np.zeros(lo.shape[0], np.int64)
    if _load().oracle_sort_perm(lo.shape[0], lo.ctypes.data, hi.ctypes.data, perm.ctypes.data):
        raise MemoryError
    return perm


def coalesce(keys_sorted, vals_sorted):
    lo, hi = _key_words(keys_sorted)
    v = np.ascontiguousarray(vals_sorted, np.float64)
    olo, ohi, ov = np.zeros_like(lo), np.zeros_like(hi), np.zeros_like(v)
    u = _load().oracle_coalesce(lo.shape[0], lo.ctypes.data, hi.ctypes.data, v.ctypes.data,
                                olo.ctypes.data, ohi.ctypes.data, ov.ctypes.data)
    return (olo[:u], ohi[:u]), ov[:u]


def partition(M: int, L: int):
    seg = np.zeros(min(L, M) + 1 if M > 0 else 1, np.int64)
    Le = _load().oracle_partition(M, L, seg.ctypes.data)
    if Le < 0:
        raise ValueError("L must be >= 1")
    return seg[:Le + 1]


def intervals(lay: Layout, seg, keys_sorted):
    lo, hi = _key_words(keys_sorted)
    seg = np.ascontiguousarray(seg, np.int64)
    Le = seg.shape[0] - 1
    ivl = np.zeros((max(Le, 0), lay.N, 2), np.uint32)
    _load().oracle_intervals(lay.N, Le, seg.ctypes.data, lo.ctypes.data, hi.ctypes.data,
                             lay.mask_lo.ctypes.data, lay.mask_hi.ctypes.data, ivl.ctypes.data)
    return ivl


def coverage(ivl, mode: int, dim: int):
    ivl = np.ascontiguousarray(ivl, np.uint32)
    Le, N = ivl.shape[0], ivl.shape[1]
    cov = np.zeros(dim, np.uint32)
    _load().oracle_coverage(N, Le, ivl.ctypes.data, mode, dim, cov.ctypes.data)
    return cov


# ---------------------------------------------------------------- MTTKRP
def _f64_rows(factors):
    return [np.ascontiguousarray(f, np.float64) for f in factors]


def mttkrp(dims, coords, vals, factors, mode: int):
    """Mode-`mode` MTTKRP in FP64 over the COO list (Algorithm 1)."""
    rows = _u32_rows(coords)
    v = np.ascontiguousarray(vals, np.float64)
    fs = _f64_rows(factors)
    R = fs[0].shape[1]
    d = np.array(dims, np.uint64)
    out = np.zeros((int(dims[mode]), R), np.float64)
    _load().oracle_mttkrp(len(dims), v.shape[0], _ptrs(rows), v.ctypes.data, d.ctypes.data,
                          _ptrs(fs), R, mode, out.ctypes.data)
    return out


def mttkrp_par(dims, coords, vals, factors, mode: int):
    """The same MTTKRP on every host core (OpenMP, thread-private outputs
    added at the end).  Returns (out, threads used)."""
    rows = _u32_rows(coords)
    v = np.ascontiguousarray(vals, np.float64)
    fs = _f64_rows(factors)
    R = fs[0].shape[1]
    d = np.array(dims, np.uint64)
    out = np.zeros((int(dims[mode]), R), np.float64)
    used = _load().oracle_mttkrp_par(len(dims), v.shape[0], _ptrs(rows), v.ctypes.data, d.ctypes.data,
                                     _ptrs(fs), R, mode, out.ctypes.data)
    if used < 0:
        raise MemoryError
    return out, used


def mttkrp_rows(dims, coords, vals, factors, mode: int, rows_sel):
    rows = _u32_rows(coords)
    v = np.ascontiguousarray(vals, np.float64)
    fs = _f64_rows(factors)
    R = fs[0].shape[1]
    d = np.array(dims, np.uint64)
    sel = np.ascontiguousarray(rows_sel, np.uint32)
    out = np.zeros((sel.shape[0], R), np.float64)
    if _load().oracle_mttkrp_rows(len(dims), v.shape[0], _ptrs(rows), v.ctypes.data, d.ctypes.data,
                                  _ptrs(fs), R, mode, sel.shape[0], sel.ctypes.data, out.ctypes.data):
        raise MemoryError
    return out


def norm2(coords, vals):
    rows = _u32_rows(coords)
    v = np.ascontiguousarray(vals, np.float64)
    return _load().oracle_norm2(len(rows), v.shape[0], _ptrs(rows), v.ctypes.data)


def cp_als(dims, coords, vals, init_factors, iters: int):
    """FP64 CP-ALS from the given initial factors.  Returns (factors, lambda, fit[iters])."""
    rows = _u32_rows(coords)
    v = np.ascontiguousarray(vals, np.float64)
    fs = [np.array(f, dtype=np.float64, copy=True, order="C") for f in init_factors]
    R = fs[0].shape[1]
    d = np.array(dims, np.uint64)
    lam = np.zeros(R, np.float64)
    fit = np.zeros(iters, np.float64)
    rc = _load().oracle_cp_als(len(dims), v.shape[0], _ptrs(rows), v.ctypes.data, d.ctypes.data, R,
                               iters, _ptrs(fs), lam.ctypes.data, fit.ctypes.data)
    if rc == -1:
        raise np.linalg.LinAlgError("normal equations not positive definite")
    if rc:
        raise MemoryError
    return fs, lam, fit


# ---------------------------------------------------------------- transposition
def transpose(coords, vals, perm):
    """The nonzeros of a COO tensor (repeated coordinates summed in FP64, in
    input order) listed in lexicographic order of their coordinates taken in
    the mode order perm[0], perm[1], ... (perm[0] most significant).
    Returns (coords uint32 [N, M'] with row j the coordinates along mode
    perm[j], vals float64 [M'])."""
    c = np.asarray(coords, np.uint32)
    v = np.asarray(vals, np.float64)
    N = c.shape[0]
    pc = c[list(perm)]
    if c.shape[1] == 0:
        return pc, v
    # np.lexsort sorts by its last key first: pass the least significant first
    order = np.lexsort(tuple(pc[j] for j in range(N - 1, -1, -1)))
    pc, v = pc[:, order], v[order]
    new = np.ones(pc.shape[1], bool)
    new[1:] = np.any(pc[:, 1:] != pc[:, :-1], axis=0)
    starts = np.nonzero(new)[0]
    return np.ascontiguousarray(pc[:, starts]), np.add.reduceat(v, starts)


# ---------------------------------------------------------------- misc
def bf16_round(x):
    """(bits uint16, values float64) of the bfloat16 rounding of x."""
    x = np.ascontiguousarray(x, np.float64)
    bits = np.zeros(x.shape, np.uint16)
    out = np.zeros(x.shape, np.float64)
    _load().oracle_bf16_round(x.size, x.ctypes.data, bits.ctypes.data, out.ctypes.data)
    return bits, out


def heuristic_staging(M: int, dim: int) -> bool:
    """Section 3.3: local staging when the fiber reuse M/I_n exceeds 4."""
    return bool(_load().oracle_heuristic_staging(M, dim))


def storage_bits(dims, M: int) -> int:
    """Eq. 1 with ceil(log2 I_n) bits per mode: M * sum_n b_n."""
    return M * sum(max(0, math.ceil(math.log2(d))) if d > 1 else 0 for d in dims)


def compression_ratio(dims, word_bits: int) -> float:
    """Eq. 2: sum_n ceil(b_n / W_b) / ceil(sum_n b_n / W_b)."""
    b = [math.ceil(math.log2(d)) if d > 1 else 0 for d in dims]
    return sum(math.ceil(x / word_bits) for x in b) / math.ceil(sum(b) / word_bits)


def sfc_bits(dims, M: int) -> int:
    """Eq. 3: a Z-Morton index needs M * N * max_n b_n bits."""
    return M * len(dims) * max(math.ceil(math.log2(d)) if d > 1 else 0 for d in dims)


class MLP:
    """Parameter container for the selector network oracle (FP64)."""

    def __init__(self, W1, b1, W2, b2, W3, b3):
        self.p = [np.ascontiguousarray(a, np.float64) for a in (W1, b1, W2, b2, W3, b3)]
        self.H, self.F = self.p[0].shape
        self.K = self.p[4].shape[0]

    def forward(self, x, t=None, mask=None):
        x = np.ascontiguousarray(x, np.float64)
        B = x.shape[0]
        y = np.zeros((B, self.K), np.float64)
        tt = np.ascontiguousarray(t, np.float64) if t is not None else None
        mm = np.ascontiguousarray(mask, np.float64) if mask is not None else None
        loss = _load().oracle_mlp_forward(B, self.F, self.H, self.K, *[a.ctypes.data for a in self.p],
                                          x.ctypes.data, tt.ctypes.data if tt is not None else None,
                                          mm.ctypes.data if mm is not None else None, y.ctypes.data)
        return y, loss

    def backward(self, x, t, mask):
        x = np.ascontiguousarray(x, np.float64)
        t = np.ascontiguousarray(t, np.float64)
        mask = np.ascontiguousarray(mask, np.float64)
        grads = [np.zeros_like(a) for a in self.p]
        loss = _load().oracle_mlp_backward(x.shape[0], self.F, self.H, self.K,
                                           *[a.ctypes.data for a in self.p], x.ctypes.data,
                                           t.ctypes.data, mask.ctypes.data,
                                           *[g.ctypes.data for g in grads])
        return grads, loss
