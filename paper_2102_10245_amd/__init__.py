"""Python binding of libalto: ALTO sparse tensors, MTTKRP and CP-ALS on MI355X.

Argument marshalling only: every step runs in the HIP library
(``libalto.so``, built by ``paper_2102_10245_amd.build``) through its C ABI
(``include/alto.h``).  PyTorch supplies device memory and the current
stream; no tensor arithmetic happens here.  Importing works without a GPU,
but every call that needs the library raises if ``libalto.so`` is missing.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libalto.so")

MAX_MODES = 8

OK, E_INVAL, E_TOO_WIDE, E_RANGE, E_NOMEM, E_HIP, E_NOTSPD, E_STATE = range(8)
PREC = {"f32": 0, "bf16": 1}
STRATEGY = {"auto": 0, "atomic": 1, "staged": 2, "sorted": 3}
STRATEGY_NAME = {v: k for k, v in STRATEGY.items()}

# Names the C ABI exports (include/alto.h).
EXPORTS = (
    "alto_build", "alto_info", "alto_partition", "alto_mttkrp", "alto_mttkrp_noalloc", "cp_als", "alto_select",
    "alto_selector_load", "alto_selector_features", "alto_mlp_forward", "alto_mlp_backward",
    "alto_mlp_adam", "alto_export_keys", "alto_export_mode_order", "alto_export_partition", "alto_export_coverage",
    "alto_round_bf16", "alto_transpose", "alto_append", "alto_export_flags", "alto_free", "alto_last_error", "alto_device_compute_units", "alto_layout",
    "alto_timing_enable", "alto_timing_read",
)


class AltoError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libalto error {code}: {msg}")
        self.code = code


class _Opts(ctypes.Structure):
    _fields_ = [("key_bits", ctypes.c_int), ("num_segments", ctypes.c_int), ("validate", ctypes.c_int)]


class _Exec(ctypes.Structure):
    _fields_ = [("strategy", ctypes.c_int), ("num_segments", ctypes.c_int)]


class _Info(ctypes.Structure):
    _fields_ = [
        ("N", ctypes.c_int), ("index_bits", ctypes.c_int), ("key_bits", ctypes.c_int),
        ("num_segments", ctypes.c_int), ("nnz_in", ctypes.c_int64), ("nnz", ctypes.c_int64),
        ("dims", ctypes.c_uint64 * MAX_MODES), ("mode_bits", ctypes.c_int * MAX_MODES),
        ("mask_lo", ctypes.c_uint64 * MAX_MODES), ("mask_hi", ctypes.c_uint64 * MAX_MODES),
        ("fiber_reuse", ctypes.c_double * MAX_MODES), ("index_bytes", ctypes.c_double),
        ("coo_index_bytes", ctypes.c_double), ("norm2", ctypes.c_double),
        ("tensor_bytes", ctypes.c_double), ("partition_bytes", ctypes.c_double),
        ("order_bytes", ctypes.c_double), ("scratch_bytes", ctypes.c_double),
        ("flag_bit", ctypes.c_int * MAX_MODES),
    ]


_lib = None


def lib_available() -> bool:
    return os.path.exists(LIB_PATH)


def lib():
    """Load libalto.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: run `python -m paper_2102_10245_amd.build` first")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64
    L.alto_build.argtypes = [vp, vp, i64, vp, i32, vp, ctypes.POINTER(vp), vp]
    L.alto_info.argtypes = [vp, ctypes.POINTER(_Info)]
    L.alto_layout.argtypes = [vp, i32, i32, ctypes.POINTER(_Info)]
    L.alto_partition.argtypes = [vp, i32, vp]
    L.alto_mttkrp.argtypes = [vp, vp, i32, i32, i32, vp, vp, vp]
    L.alto_mttkrp_noalloc.argtypes = [vp, vp, i32, i32, i32, vp, vp]
    L.cp_als.argtypes = [vp, i32, i32, i32, vp, vp, vp, vp, vp]
    L.alto_select.argtypes = [vp, i32, i32, i32, ctypes.POINTER(_Exec)]
    L.alto_selector_load.argtypes = [vp, ctypes.c_size_t]
    L.alto_selector_features.argtypes = [vp, i32, i32, i32, vp]
    L.alto_mlp_forward.argtypes = [i32, i32, i32, i32, vp, vp, vp, vp, vp, vp, vp]
    L.alto_mlp_backward.argtypes = [i32, i32, i32, i32, vp, vp, vp, vp, vp, vp, vp]
    L.alto_mlp_adam.argtypes = [i64, vp, vp, vp, vp, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                ctypes.c_float, i32, vp]
    L.alto_export_keys.argtypes = [vp, vp, vp, vp]
    L.alto_export_mode_order.argtypes = [vp, i32, vp, vp, vp]
    L.alto_export_partition.argtypes = [vp, vp, vp, vp]
    L.alto_export_coverage.argtypes = [vp, i32, vp, vp]
    L.alto_round_bf16.argtypes = [vp, vp, i64, vp]
    L.alto_transpose.argtypes = [vp, vp, vp, vp, vp]
    L.alto_append.argtypes = [vp, vp, vp, i64, vp]
    L.alto_export_flags.argtypes = [vp, i32, vp, ctypes.POINTER(ctypes.c_int), vp]
    L.alto_free.argtypes = [vp]
    L.alto_free.restype = None
    L.alto_last_error.restype = ctypes.c_char_p
    L.alto_device_compute_units.restype = i32
    L.alto_timing_enable.argtypes = [i32]
    L.alto_timing_read.argtypes = [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]
    _lib = L
    return L


def _check(rc: int):
    if rc != OK:
        raise AltoError(rc, lib().alto_last_error().decode())


def _torch():
    import torch
    return torch


def _stream(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _ptr_array(ts):
    a = (ctypes.c_void_p * len(ts))()
    for n, t in enumerate(ts):
        a[n] = t.data_ptr() if t is not None else None
    return a


def _prec_of(factors):
    torch = _torch()
    dts = {f.dtype for f in factors if f is not None}
    if dts == {torch.float32}:
        return PREC["f32"]
    if dts == {torch.bfloat16}:
        return PREC["bf16"]
    raise ValueError("factors must all be float32 or all bfloat16")


def _check_factor(f, dim, R):
    torch = _torch()
    if not f.is_cuda or not f.is_contiguous() or tuple(f.shape) != (int(dim), R):
        raise ValueError(f"factor must be a contiguous CUDA tensor of shape ({dim}, {R})")
    if f.dtype not in (torch.float32, torch.bfloat16):
        raise ValueError("factor dtype must be float32 or bfloat16")


class AltoTensor:
    """A sparse tensor in ALTO form on the current GPU (owns device memory)."""

    def __init__(self, handle: ctypes.c_void_p):
        self._h = handle
        self._lib = lib()

    # -------------------------------------------------------------- build
    @classmethod
    def build(cls, coords, vals, dims, key_bits: int = 0, num_segments: int = 0, stream=None):
        """coords: CUDA int32 tensor [N, M] (read as uint32); vals: CUDA float32 [M]."""
        torch = _torch()
        N = len(dims)
        if coords.dim() != 2 or coords.shape[0] != N:
            raise ValueError("coords must have shape [N, M]")
        if coords.dtype != torch.int32 or vals.dtype != torch.float32:
            raise ValueError("coords must be int32 (uint32 bit pattern) and vals float32")
        if not coords.is_cuda or not vals.is_cuda:
            raise ValueError("coords and vals must be CUDA tensors")
        coords = coords.contiguous()
        vals = vals.contiguous()
        M = int(coords.shape[1])
        if vals.shape != (M,):
            raise ValueError("vals must have shape [M]")
        rows = _ptr_array([coords[n] for n in range(N)])
        d = (ctypes.c_uint64 * N)(*[int(x) for x in dims])
        opts = _Opts(key_bits, num_segments, 1)
        h = ctypes.c_void_p()
        _check(lib().alto_build(rows, _ptr(vals), M, d, N, ctypes.byref(opts), ctypes.byref(h), _stream(stream)))
        return cls(h)

    def append(self, coords, vals, stream=None):
        """alto_append: add a batch (CUDA int32 coords [N, M], float32 vals [M])."""
        torch = _torch()
        N = self.info()["N"]
        if coords.dim() != 2 or coords.shape[0] != N or coords.dtype != torch.int32 or not coords.is_cuda:
            raise ValueError("coords must be a CUDA int32 tensor of shape [N, M]")
        if vals.dtype != torch.float32 or not vals.is_cuda or vals.shape != (coords.shape[1],):
            raise ValueError("vals must be a CUDA float32 tensor of shape [M]")
        coords = coords.contiguous()
        vals = vals.contiguous()
        rows = _ptr_array([coords[n] for n in range(N)])
        _check(self._lib.alto_append(self._h, rows, _ptr(vals), int(coords.shape[1]), _stream(stream)))

    def close(self):
        if self._h:
            self._lib.alto_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -------------------------------------------------------------- info
    def info(self) -> dict:
        inf = _Info()
        _check(self._lib.alto_info(self._h, ctypes.byref(inf)))
        N = inf.N
        return {
            "N": N, "index_bits": inf.index_bits, "key_bits": inf.key_bits,
            "num_segments": inf.num_segments, "nnz_in": inf.nnz_in, "nnz": inf.nnz,
            "dims": [int(inf.dims[n]) for n in range(N)],
            "mode_bits": [int(inf.mode_bits[n]) for n in range(N)],
            "masks": [int(inf.mask_lo[n]) | (int(inf.mask_hi[n]) << 64) for n in range(N)],
            "fiber_reuse": [float(inf.fiber_reuse[n]) for n in range(N)],
            "index_bytes": inf.index_bytes, "coo_index_bytes": inf.coo_index_bytes, "norm2": inf.norm2,
            "tensor_bytes": inf.tensor_bytes, "partition_bytes": inf.partition_bytes,
            "order_bytes": inf.order_bytes, "scratch_bytes": inf.scratch_bytes,
            "flag_bit": [int(inf.flag_bit[n]) for n in range(N)],
        }

    @property
    def N(self):
        return self.info()["N"]

    def partition(self, num_segments: int, stream=None):
        _check(self._lib.alto_partition(self._h, num_segments, _stream(stream)))

    # -------------------------------------------------------------- MTTKRP
    def mttkrp(self, factors, mode: int, out=None, strategy: str = "auto", num_segments: int = 0, stream=None):
        """factors: list of N CUDA tensors [I_n, R] (float32 or bfloat16; entry `mode` may be None)."""
        torch = _torch()
        inf = self.info()
        if not 0 <= mode < inf["N"] or len(factors) != inf["N"]:
            raise ValueError("mode out of range or wrong number of factors")
        R = next(f.shape[1] for f in factors if f is not None)
        for n, f in enumerate(factors):
            if n != mode:
                _check_factor(f, inf["dims"][n], R)
        prec = _prec_of([f for n, f in enumerate(factors) if n != mode])
        if out is None:
            out = torch.empty((inf["dims"][mode], R), dtype=torch.float32, device=factors[(mode + 1) % len(factors)].device)
        elif out.dtype != torch.float32 or tuple(out.shape) != (inf["dims"][mode], R) or not out.is_contiguous():
            raise ValueError("out must be a contiguous float32 tensor of shape (I_mode, R)")
        ex = _Exec(STRATEGY[strategy], num_segments)
        fp = _ptr_array([f if n != mode else None for n, f in enumerate(factors)])
        _check(self._lib.alto_mttkrp(self._h, fp, R, prec, mode, _ptr(out), ctypes.byref(ex), _stream(stream)))
        return out

    def mttkrp_noalloc(self, factors, mode: int, out, stream=None):
        """alto_mttkrp_noalloc: atomic-update MTTKRP on the current partition with
        no device allocation; `out` (float32 CUDA tensor [I_mode, R]) is required."""
        torch = _torch()
        inf = self.info()
        if not 0 <= mode < inf["N"] or len(factors) != inf["N"]:
            raise ValueError("mode out of range or wrong number of factors")
        R = next(f.shape[1] for f in factors if f is not None)
        for n, f in enumerate(factors):
            if n != mode:
                _check_factor(f, inf["dims"][n], R)
        prec = _prec_of([f for n, f in enumerate(factors) if n != mode])
        if out.dtype != torch.float32 or tuple(out.shape) != (inf["dims"][mode], R) or not out.is_contiguous():
            raise ValueError("out must be a contiguous float32 tensor of shape (I_mode, R)")
        fp = _ptr_array([f if n != mode else None for n, f in enumerate(factors)])
        _check(self._lib.alto_mttkrp_noalloc(self._h, fp, R, prec, mode, _ptr(out), _stream(stream)))
        return out

    def cp_als(self, factors, iters: int, strategy: str = "auto", num_segments: int = 0, stream=None):
        """In-place CP-ALS on `factors` (float32 or bfloat16 CUDA tensors).  Returns (lambda, fit)."""
        torch = _torch()
        inf = self.info()
        R = factors[0].shape[1]
        for n, f in enumerate(factors):
            _check_factor(f, inf["dims"][n], R)
        prec = _prec_of(factors)
        lam = torch.empty(R, dtype=torch.float64, device=factors[0].device)
        fit = (ctypes.c_double * max(1, iters))()
        ex = _Exec(STRATEGY[strategy], num_segments)
        _check(self._lib.cp_als(self._h, R, iters, prec, _ptr_array(factors), _ptr(lam), fit, ctypes.byref(ex),
                                _stream(stream)))
        return lam, np.array(fit[:iters], dtype=np.float64)

    def transpose(self, perm, stream=None):
        """alto_transpose: (coords int32 CUDA tensor [N, nnz] whose row j holds
        the coordinates along mode perm[j], vals float32 [nnz]) in
        lexicographic order of (perm[0], perm[1], ...)."""
        torch = _torch()
        inf = self.info()
        N, M = inf["N"], inf["nnz"]
        if sorted(perm) != list(range(N)):
            raise ValueError("perm must be a permutation of 0..N-1")
        dev = torch.device("cuda", torch.cuda.current_device())
        coords = torch.empty((N, M), dtype=torch.int32, device=dev)
        vals = torch.empty(M, dtype=torch.float32, device=dev)
        p = (ctypes.c_int * N)(*perm)
        _check(self._lib.alto_transpose(self._h, p, _ptr_array([coords[j] for j in range(N)]), _ptr(vals),
                                        _stream(stream)))
        return coords, vals

    def export_flags(self, mode: int, stream=None):
        """alto_export_flags: (flags uint8 CUDA tensor [nnz], lane groups per segment)."""
        torch = _torch()
        M = self.info()["nnz"]
        out = torch.empty(M, dtype=torch.uint8, device=torch.device("cuda", torch.cuda.current_device()))
        g = ctypes.c_int(0)
        _check(self._lib.alto_export_flags(self._h, mode, _ptr(out), ctypes.byref(g), _stream(stream)))
        return out, g.value

    def select(self, mode: int, R: int, prec: str = "f32"):
        ex = _Exec()
        _check(self._lib.alto_select(self._h, mode, R, PREC[prec], ctypes.byref(ex)))
        return STRATEGY_NAME[ex.strategy], ex.num_segments

    def selector_features(self, mode: int, R: int, prec: str = "f32") -> np.ndarray:
        f = np.zeros(15, np.float32)
        _check(self._lib.alto_selector_features(self._h, mode, R, PREC[prec], f.ctypes.data))
        return f

    # -------------------------------------------------------------- inspection
    def export_keys(self, stream=None):
        """(keys, vals): keys int32 [M] / int64 [M] / int64 [M, 2] (lo, hi) by key width."""
        torch = _torch()
        inf = self.info()
        M, kb = inf["nnz"], inf["key_bits"]
        dev = torch.device("cuda", torch.cuda.current_device())
        if kb == 32:
            keys = torch.empty(M, dtype=torch.int32, device=dev)
        elif kb == 64:
            keys = torch.empty(M, dtype=torch.int64, device=dev)
        else:
            keys = torch.empty((M, 2), dtype=torch.int64, device=dev)
        vals = torch.empty(M, dtype=torch.float32, device=dev)
        _check(self._lib.alto_export_keys(self._h, _ptr(keys), _ptr(vals), _stream(stream)))
        return keys, vals

    def export_mode_order(self, mode: int, stream=None):
        """(keys, vals) of the segment-local order by `mode` (layout as export_keys)."""
        torch = _torch()
        inf = self.info()
        if not 0 <= mode < inf["N"]:
            raise ValueError("mode out of range")
        M, kb = inf["nnz"], inf["key_bits"]
        dev = torch.device("cuda", torch.cuda.current_device())
        shape = (M, 2) if kb == 128 else (M,)
        keys = torch.empty(shape, dtype=torch.int32 if kb == 32 else torch.int64, device=dev)
        vals = torch.empty(M, dtype=torch.float32, device=dev)
        _check(self._lib.alto_export_mode_order(self._h, mode, _ptr(keys), _ptr(vals), _stream(stream)))
        return keys, vals

    def export_partition(self, stream=None):
        torch = _torch()
        inf = self.info()
        L, N = inf["num_segments"], inf["N"]
        dev = torch.device("cuda", torch.cuda.current_device())
        seg = torch.empty(L + 1, dtype=torch.int64, device=dev)
        ivl = torch.empty((max(L, 0), N, 2), dtype=torch.int32, device=dev)
        _check(self._lib.alto_export_partition(self._h, _ptr(seg), _ptr(ivl) if L > 0 else None, _stream(stream)))
        return seg, ivl

    def export_coverage(self, mode: int, stream=None):
        torch = _torch()
        inf = self.info()
        cov = torch.empty(inf["dims"][mode], dtype=torch.int32, device=torch.device("cuda", torch.cuda.current_device()))
        _check(self._lib.alto_export_coverage(self._h, mode, _ptr(cov), _stream(stream)))
        return cov


def layout(dims, key_bits: int = 0) -> dict:
    """The library's bit layout for these mode lengths (host only)."""
    N = len(dims)
    d = (ctypes.c_uint64 * N)(*[int(x) for x in dims])
    inf = _Info()
    _check(lib().alto_layout(d, N, key_bits, ctypes.byref(inf)))
    return {"N": N, "index_bits": inf.index_bits, "key_bits": inf.key_bits,
            "mode_bits": [int(inf.mode_bits[n]) for n in range(N)],
            "masks": [int(inf.mask_lo[n]) | (int(inf.mask_hi[n]) << 64) for n in range(N)]}


def build_tensor(coords, vals, dims, **kw) -> AltoTensor:
    return AltoTensor.build(coords, vals, dims, **kw)


def round_bf16(x, stream=None):
    """bfloat16 storage rounding of a CUDA float64 tensor (returns int16 bit patterns)."""
    torch = _torch()
    if x.dtype != torch.float64 or not x.is_cuda:
        raise ValueError("x must be a CUDA float64 tensor")
    x = x.contiguous()
    out = torch.empty(x.shape, dtype=torch.int16, device=x.device)
    _check(lib().alto_round_bf16(_ptr(x), _ptr(out), x.numel(), _stream(stream)))
    return out


def selector_load(weights: np.ndarray | None):
    if weights is None:
        _check(lib().alto_selector_load(None, 0))
        return
    w = np.ascontiguousarray(weights, dtype=np.float32)
    _check(lib().alto_selector_load(w.ctypes.data, w.size))


DEFAULT_SELECTOR = os.path.join(_HERE, "selector_weights.f32")


def load_default_selector() -> bool:
    """Install the trained selector weights shipped with the package, if present."""
    if not os.path.exists(DEFAULT_SELECTOR):
        return False
    selector_load(np.fromfile(DEFAULT_SELECTOR, dtype=np.float32))
    return True


def compute_units() -> int:
    return int(lib().alto_device_compute_units())


def timing_enable(enable: bool = True):
    """Start (or stop) recording an event pair around the MTTKRP kernels of
    every MTTKRP the library runs (measurement only)."""
    _check(lib().alto_timing_enable(1 if enable else 0))


def timing_read():
    """(total milliseconds, number of MTTKRPs) recorded since the last read."""
    ms = ctypes.c_double(0.0)
    n = ctypes.c_int64(0)
    _check(lib().alto_timing_read(ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


# ------------------------------------------------------------------ selector network kernels
def mlp_param_count(F: int, H: int, K: int) -> int:
    return H * F + H + H * H + H + K * H + K


def mlp_forward(params, x, F: int, H: int, K: int, t=None, mask=None, stream=None):
    torch = _torch()
    B = int(x.shape[0])
    y = torch.empty((B, K), dtype=torch.float32, device=x.device)
    loss = torch.empty(1, dtype=torch.float32, device=x.device) if t is not None else None
    _check(lib().alto_mlp_forward(B, F, H, K, _ptr(params), _ptr(x), _ptr(t), _ptr(mask), _ptr(y), _ptr(loss),
                                  _stream(stream)))
    return y, loss


def mlp_backward(params, x, t, mask, F: int, H: int, K: int, stream=None):
    torch = _torch()
    B = int(x.shape[0])
    g = torch.empty_like(params)
    loss = torch.empty(1, dtype=torch.float32, device=x.device)
    _check(lib().alto_mlp_backward(B, F, H, K, _ptr(params), _ptr(x), _ptr(t), _ptr(mask), _ptr(g), _ptr(loss),
                                   _stream(stream)))
    return g, loss


def mlp_adam(params, grads, m, v, lr: float, step: int, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    _check(lib().alto_mlp_adam(params.numel(), _ptr(params), _ptr(grads), _ptr(m), _ptr(v), lr, beta1, beta2, eps,
                               step, _stream(stream)))
