"""The C-ABI library loads and exports every entry point include/alto.h
declares; argument errors come back as exact codes without touching a GPU."""
import ctypes
import os
import re

import pytest

import paper_2102_10245_amd as alto

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "alto.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|void|const char \*)\s*\**\s*(\w+)\s*\(", src, flags=re.M)))


def test_header_declares_expected_calls():
    names = _declared()
    for n in ("alto_build", "alto_mttkrp", "cp_als", "alto_select", "alto_free", "alto_last_error"):
        assert n in names
    assert set(names) == set(alto.EXPORTS)


@pytest.mark.skipif(not alto.lib_available(), reason="libalto.so not built")
def test_library_exports_every_declared_symbol():
    L = ctypes.CDLL(alto.LIB_PATH)
    for n in _declared():
        assert hasattr(L, n), n


@pytest.mark.skipif(not alto.lib_available(), reason="libalto.so not built")
def test_argument_errors_without_device_work():
    L = alto.lib()
    h = ctypes.c_void_p()
    dims = (ctypes.c_uint64 * 3)(4, 8, 2)
    # N outside 2..8
    assert L.alto_build(None, None, 0, dims, 1, None, ctypes.byref(h), None) == alto.E_INVAL
    assert L.alto_build(None, None, 0, dims, 9, None, ctypes.byref(h), None) == alto.E_INVAL
    # a zero dimension and one above 2^32
    bad = (ctypes.c_uint64 * 3)(4, 0, 2)
    assert L.alto_build(None, None, 0, bad, 3, None, ctypes.byref(h), None) == alto.E_INVAL
    big = (ctypes.c_uint64 * 3)(4, 2 ** 32 + 1, 2)
    assert L.alto_build(None, None, 0, big, 3, None, ctypes.byref(h), None) == alto.E_INVAL
    assert b"dims" in L.alto_last_error()
    # null coordinates with nnz > 0
    assert L.alto_build(None, None, 5, dims, 3, None, ctypes.byref(h), None) == alto.E_INVAL
    # null handles
    assert L.alto_mttkrp(None, None, 16, 0, 0, None, None, None) == alto.E_INVAL
    assert L.cp_als(None, 16, 1, 0, None, None, None, None, None) == alto.E_INVAL
    assert L.alto_partition(None, 4, None) == alto.E_INVAL
    assert L.alto_info(None, None) == alto.E_INVAL
    ex = alto._Exec()
    assert L.alto_select(None, 0, 16, 0, ctypes.byref(ex)) == alto.E_INVAL
    # selector weights with a bad header
    import numpy as np
    w = np.zeros(10, np.float32)
    assert L.alto_selector_load(w.ctypes.data, w.size) == alto.E_INVAL
    assert L.alto_selector_load(None, 0) == alto.OK
    # MLP size checks
    assert L.alto_mlp_forward(0, 1, 1, 1, None, None, None, None, None, None, None) == alto.E_INVAL
    assert L.alto_mlp_adam(0, None, None, None, None, 0.1, 0.9, 0.99, 1e-8, 1, None) == alto.E_INVAL
    assert L.alto_round_bf16(None, None, -1, None) == alto.E_INVAL
    L.alto_free(None)
    # kernel timing: null outputs; an empty record reads as nothing
    assert L.alto_timing_read(None, None) == alto.E_INVAL
    assert alto.timing_read() == (0.0, 0)


@pytest.mark.skipif(not alto.lib_available(), reason="libalto.so not built")
@pytest.mark.parametrize("dims", [(4, 8, 2), (1000, 800, 600), (2_000_000, 2_000_000, 20_000),
                                  (1_000_000, 100_000, 10_000, 500), (10_000_000, 5_000_000, 2_000_000, 100_000, 1_000),
                                  (1, 7, 1), (2 ** 32, 2 ** 32, 2 ** 20), (3, 3, 3, 3, 3, 3, 3, 3), (5, 5), (17, 16, 17)])
def test_library_layout_matches_oracle(dims):
    """The host half of alto_build (bit layout, Section 3.1) against the oracle."""
    import oracle
    got = alto.layout(dims)
    ref = oracle.layout(dims)
    assert got["index_bits"] == ref.B and got["mode_bits"] == ref.nbits and got["masks"] == ref.masks
    assert got["key_bits"] == ref.W


@pytest.mark.skipif(not alto.lib_available(), reason="libalto.so not built")
def test_library_layout_errors():
    with pytest.raises(alto.AltoError) as e:
        alto.layout((2 ** 32,) * 5)
    assert e.value.code == alto.E_TOO_WIDE
    with pytest.raises(alto.AltoError) as e:
        alto.layout((2 ** 20,) * 3, key_bits=32)
    assert e.value.code == alto.E_TOO_WIDE
    with pytest.raises(alto.AltoError) as e:
        alto.layout((4, 0, 2))
    assert e.value.code == alto.E_INVAL
    assert alto.layout((1000, 800, 600), key_bits=128)["key_bits"] == 128


def _table1_dims():
    import json
    with open(os.path.join(ROOT, "tests", "golden", "table1_tensors.json")) as f:
        return [(name, tuple(int(round(d)) for d in dims)) for name, dims, _, _ in json.load(f)["tensors"]]


@pytest.mark.skipif(not alto.lib_available(), reason="libalto.so not built")
@pytest.mark.parametrize("name,dims", [(n, tuple(r.dims)) for n, r in __import__("synth").WORKLOADS.items()]
                         + _table1_dims())
def test_library_storage_matches_eq1_eq2(name, dims):
    """Format storage (Section 3.1, Eq. 1 and Eq. 2) as the library lays it
    out: the index bits per nonzero are Eq. 1's sum of ceil(log2 I_n); the
    stored word is the smallest of 32, 64 and 128 bits that holds them; and
    the COO-to-ALTO index ratio in stored words is Eq. 2's ratio with 32-bit
    words when the ALTO index takes 1, 2 or 4 such words (otherwise the
    stored word rounds up to the next power of two and the ratio is lower)."""
    import math

    import oracle
    got = alto.layout(dims)
    N = len(dims)
    B = got["index_bits"]
    assert B == oracle.storage_bits(dims, 1)
    W = got["key_bits"]
    assert W == min(w for w in (32, 64, 128) if w >= B)
    words = math.ceil(B / 32)
    eq2 = oracle.compression_ratio(dims, 32)
    assert eq2 == pytest.approx(N / words)
    stored = N * 32 / W
    if words in (1, 2, 4):
        assert stored == pytest.approx(eq2)
    else:
        assert stored < eq2
