"""GPU format generation vs the oracle, bit for bit: linearized indices,
their order, coalescing, segment bounds, mode intervals and coverage."""
import ctypes

import numpy as np
import pytest

import oracle
import paper_2102_10245_amd as alto
import synth
from gpu_common import gpu_ok, keys_numpy, oracle_alto, small, to_dev

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_ok(), reason="needs a GPU")]

CASES = [
    # (recipe, key_bits override, L)
    (synth.WORKLOADS["uniform3_1000x800x600_100k"], 0, 2048),
    (small("zipf3_2Mx2Mx20k_50M", 200_000), 0, 1024),
    (small("zipf4_1Mx100kx10kx500_150M", 300_000), 0, 2048),
    (small("zipf5_10Mx5Mx2Mx100kx1k_200M", 150_000), 0, 512),
    (synth.Recipe("wide_key_short_index", (1000, 800, 600), 50_001, (0.8, 0, 1.3), seed=3), 128, 97),
    (synth.Recipe("pow2_dims", (1024, 2, 4096, 1, 64), 70_000, (0, 0, 1.1, 0, 0), seed=4), 64, 300),
    (synth.Recipe("order2", (5000, 3000), 40_000, (1.0, 0), seed=5), 0, 64),
    (synth.Recipe("order6", (40, 30, 20, 10, 7, 3), 60_000, (0.5,) * 6, seed=6), 0, 333),
    (synth.Recipe("order8", (9, 8, 7, 6, 5, 4, 3, 2), 30_000, (), seed=7), 0, 40),
    # 120-bit index whose deposit tables (18 coordinate bytes x 256 x 16 B)
    # exceed the LDS budget of the table encoder: the bit-run encoder runs
    (synth.Recipe("order6_wide", (1 << 20,) * 6, 50_000, (0.7, 0, 0, 0, 0, 0), seed=8), 0, 128),
]


@pytest.mark.parametrize("rec,kb,L", CASES, ids=[c[0].name for c in CASES])
def test_build_bit_exact(rec, kb, L):
    print("case", rec.name, rec.dims, rec.nnz, kb, L, flush=True)
    coords, vals = synth.coo(rec)
    c, v = to_dev(coords, vals)
    t = alto.AltoTensor.build(c, v, rec.dims, key_bits=kb, num_segments=L)
    info = t.info()
    (olo, ohi), ov, lay, _ = oracle_alto(rec.dims, coords, vals)
    assert info["index_bits"] == lay.B
    assert info["masks"] == lay.masks
    assert info["key_bits"] == (kb or lay.W)
    assert info["nnz_in"] == rec.nnz and info["nnz"] == len(olo)
    # storage (Eq. 1 in stored words) and the device bytes of the tensor proper
    M, N = info["nnz"], len(rec.dims)
    assert info["index_bytes"] == M * info["key_bits"] / 8
    assert info["coo_index_bytes"] == M * N * 4
    assert info["tensor_bytes"] >= M * (info["key_bits"] / 8 + 4)
    assert info["order_bytes"] == 0
    keys, gv = t.export_keys()
    glo, ghi = keys_numpy(keys, info["key_bits"])
    assert np.array_equal(glo, olo) and np.array_equal(ghi, ohi)
    gv = gv.cpu().numpy().astype(np.float64)
    if info["nnz"] == rec.nnz:
        assert np.array_equal(gv, ov)  # a permutation of the inputs, bit for bit
    else:
        assert np.allclose(gv, ov, rtol=2e-6, atol=0)  # FP32 sums of repeated coordinates
    assert info["norm2"] == pytest.approx(float(np.sum(ov * ov)), rel=1e-6)
    seg, ivl = t.export_partition()
    oseg = oracle.partition(len(olo), L)
    assert np.array_equal(seg.cpu().numpy(), oseg)
    oivl = oracle.intervals(lay, oseg, (olo, ohi))
    assert np.array_equal(ivl.cpu().numpy().view(np.uint32), oivl)
    for n in range(len(rec.dims)):
        if rec.dims[n] * len(oseg) > 2e8:
            continue  # the brute-force coverage would take too long
        cov = t.export_coverage(n).cpu().numpy().view(np.uint32)
        assert np.array_equal(cov, oracle.coverage(oivl, n, rec.dims[n])), n
    t.close()


def test_duplicates_coalesced_in_input_order():
    torch = pytest.importorskip("torch")
    dims = (7, 5, 3)
    coords = np.array([[1, 1, 6, 1, 0, 1], [2, 2, 4, 2, 0, 2], [0, 0, 2, 0, 0, 0]], np.uint32)
    vals = np.array([1.0, 2.0, 3.0, 1e-8, 5.0, 4.0], np.float32)
    c, v = to_dev(coords, vals)
    t = alto.AltoTensor.build(c, v, dims, num_segments=2)
    assert t.info()["nnz"] == 3
    _, gv = t.export_keys()
    (olo, _), ov, _, _ = oracle_alto(dims, coords, vals)
    # the repeated coordinate (1,2,0) is summed in FP32 in input order: ((1+2)+1e-8)+4
    expect = np.float32(np.float32(np.float32(1.0) + np.float32(2.0)) + np.float32(1e-8)) + np.float32(4.0)
    got = dict(zip(olo.tolist(), gv.cpu().numpy().tolist()))
    lay = oracle.layout(dims)
    k = int(oracle.encode(lay, np.array([[1], [2], [0]], np.uint32))[0][0])
    assert got[k] == expect
    t.close()


@pytest.mark.parametrize("M,L", [(0, 16), (1, 16), (5, 16), (4097, 4096)])
def test_tiny_and_empty(M, L):
    rec = synth.Recipe("tiny", (30, 20, 10), M, (), seed=11)
    coords, vals = synth.coo(rec)
    torch = pytest.importorskip("torch")
    if M == 0:
        c = torch.zeros((3, 0), dtype=torch.int32, device="cuda")
        v = torch.zeros(0, dtype=torch.float32, device="cuda")
    else:
        c, v = to_dev(coords, vals)
    t = alto.AltoTensor.build(c, v, rec.dims, num_segments=L)
    info = t.info()
    (olo, ohi), ov, lay, _ = oracle_alto(rec.dims, coords, vals)
    assert info["nnz"] == len(olo) and info["num_segments"] == min(L, len(olo))
    if M:
        keys, _ = t.export_keys()
        glo, _ = keys_numpy(keys, info["key_bits"])
        assert np.array_equal(glo, olo)
        seg, ivl = t.export_partition()
        oseg = oracle.partition(len(olo), L)
        assert np.array_equal(seg.cpu().numpy(), oseg)
        assert np.array_equal(ivl.cpu().numpy().view(np.uint32), oracle.intervals(lay, oseg, (olo, ohi)))
    t.close()


def test_out_of_range_coordinate_is_reported():
    coords = np.array([[0, 3], [0, 1], [0, 1]], np.uint32)  # 3 is not below dim 3
    c, v = to_dev(coords, np.ones(2, np.float32))
    with pytest.raises(alto.AltoError) as e:
        alto.AltoTensor.build(c, v, (3, 2, 2))
    assert e.value.code == alto.E_RANGE


def test_too_wide_index_rejected():
    c, v = to_dev(np.zeros((5, 1), np.uint32), np.ones(1, np.float32))
    with pytest.raises(alto.AltoError) as e:
        alto.AltoTensor.build(c, v, (2 ** 32,) * 5)
    assert e.value.code == alto.E_TOO_WIDE
    with pytest.raises(alto.AltoError) as e:
        alto.AltoTensor.build(c[:3], v, (2 ** 20,) * 3, key_bits=32)
    assert e.value.code == alto.E_TOO_WIDE


def test_bf16_rounding_bits_match_oracle():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(8)
    x = np.concatenate([rng.standard_normal(100000) * 10.0 ** rng.integers(-20, 20, 100000),
                        [0.0, -0.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, np.inf, -np.inf, np.nan, 3.4e38, 1e-45]])
    got = alto.round_bf16(torch.from_numpy(x).cuda()).cpu().numpy().view(np.uint16)
    ref, _ = oracle.bf16_round(x)
    assert np.array_equal(got, ref)


# segment-local mode orders (the `sorted` strategy's input): every key width,
# an order-5 tensor with one-row modes, and segments longer than one
# workgroup tile of 4096 nonzeros
ORDER_CASES = [CASES[2], CASES[4], CASES[5], CASES[6],
               (synth.Recipe("long_segments", (3000, 700, 90), 120_000, (1.1, 0.6, 0), seed=8), 0, 7)]


@pytest.mark.parametrize("rec,kb,L", ORDER_CASES, ids=[c[0].name for c in ORDER_CASES])
def test_mode_order_bit_exact(rec, kb, L):
    print("case", rec.name, rec.dims, rec.nnz, kb, L, flush=True)
    coords, vals = synth.coo(rec)
    c, v = to_dev(coords, vals)
    t = alto.AltoTensor.build(c, v, rec.dims, key_bits=kb, num_segments=L)
    info = t.info()
    (olo, ohi), ov, lay, _ = oracle_alto(rec.dims, coords, vals)
    M = len(olo)
    oseg = oracle.partition(M, L)
    segid = np.repeat(np.arange(len(oseg) - 1), np.diff(oseg))
    oc = oracle.decode(lay, (olo, ohi))
    for n in range(len(rec.dims)):
        # stable by (segment, coordinate along n): ties keep the linearized order
        perm = np.lexsort((np.arange(M), oc[n], segid))
        keys, gv = t.export_mode_order(n)
        glo, ghi = keys_numpy(keys, info["key_bits"])
        assert np.array_equal(glo, olo[perm]) and np.array_equal(ghi, ohi[perm]), n
        gv = gv.cpu().numpy().astype(np.float64)
        if info["nnz"] == rec.nnz:
            assert np.array_equal(gv, ov[perm]), n
        else:
            assert np.allclose(gv, ov[perm], rtol=2e-6, atol=0), n
    # one reordered copy of index and values per mode, on the current partition
    info = t.info()
    assert info["order_bytes"] == len(rec.dims) * M * (info["key_bits"] / 8 + 4)
    t.close()


def test_largest_dimension_bit_exact():
    # a mode of 2^32 rows (32 index bits, a full-width coordinate field in the
    # compact form), with both extreme coordinates present
    dims = (2 ** 32, 5, 3)
    rng = np.random.default_rng(41)
    M = 60_000
    coords = np.stack([rng.integers(0, 2 ** 32, M, dtype=np.uint64).astype(np.uint32),
                       rng.integers(0, 5, M).astype(np.uint32), rng.integers(0, 3, M).astype(np.uint32)])
    coords[:, 0] = (0, 0, 0)
    coords[:, 1] = (2 ** 32 - 1, 4, 2)
    vals = rng.random(M).astype(np.float32)
    c, v = to_dev(coords, vals)
    L = 16
    t = alto.AltoTensor.build(c, v, dims, num_segments=L)
    info = t.info()
    (olo, ohi), ov, lay, _ = oracle_alto(dims, coords, vals)
    assert info["index_bits"] == lay.B == 37 and info["key_bits"] == 64
    keys, _ = t.export_keys()
    glo, ghi = keys_numpy(keys, info["key_bits"])
    assert np.array_equal(glo, olo) and np.array_equal(ghi, ohi)
    oseg = oracle.partition(len(olo), L)
    seg, ivl = t.export_partition()
    assert np.array_equal(seg.cpu().numpy(), oseg)
    assert np.array_equal(ivl.cpu().numpy().view(np.uint32), oracle.intervals(lay, oseg, (olo, ohi)))
    segid = np.repeat(np.arange(len(oseg) - 1), np.diff(oseg))
    oc = oracle.decode(lay, (olo, ohi))
    for n in range(3):
        perm = np.lexsort((np.arange(len(olo)), oc[n], segid))
        k, _ = t.export_mode_order(n)
        klo, khi = keys_numpy(k, info["key_bits"])
        assert np.array_equal(klo, olo[perm]) and np.array_equal(khi, ohi[perm]), n
    # an MTTKRP (or CP-ALS) whose output mode has 2^32 rows is refused: row
    # 2^32-1 would alias the kernels' no-row marker (nothing is launched, so
    # the small placeholder buffers are never touched)
    import torch
    L_ = alto.lib()
    R = 4
    small_f = [torch.ones((d, R), dtype=torch.float32, device="cuda") for d in dims[1:]]
    dummy = torch.zeros(64, dtype=torch.float32, device="cuda")
    fp = alto._ptr_array([None] + small_f)
    assert L_.alto_mttkrp(t._h, fp, R, 0, 0, dummy.data_ptr(), None, None) == alto.E_INVAL
    assert b"2^32" in L_.alto_last_error()
    assert L_.alto_mttkrp_noalloc(t._h, fp, R, 0, 0, dummy.data_ptr(), None) == alto.E_INVAL
    lam = torch.zeros(R, dtype=torch.float64, device="cuda")
    fit = (ctypes.c_double * 1)()
    fp_all = alto._ptr_array([dummy] + small_f)
    assert L_.cp_als(t._h, R, 1, 0, fp_all, lam.data_ptr(), fit, None, None) == alto.E_INVAL
    assert b"2^32" in L_.alto_last_error()
    t.close()


ROW_FEATURE_CASES = [
    small("zipf4_1Mx100kx10kx500_150M", 300_000),                                  # 64-bit index
    small("zipf5_10Mx5Mx2Mx100kx1k_200M", 150_000),                                # 128-bit index
    synth.Recipe("tall_mode", (1 << 25, 100, 50), 60_000, (1.2, 0, 0.5), seed=11),  # 2^25 rows: hashed buckets
    synth.Recipe("many", (600, 400, 100), 3_000_000, (1.0, 0.3, 0), seed=12),       # over 2^20 nonzeros: a spaced sample
]


@pytest.mark.parametrize("rec", ROW_FEATURE_CASES, ids=[r.name for r in ROW_FEATURE_CASES])
def test_row_skew_features_match_a_host_count(rec):
    """The selector's two skew features (alto_selector_features 12 and 13):
    row counts of the nonzeros floor(k * M / S), k < S = min(M, 2^20), of the
    ordered tensor, modes over 2^24 rows folded onto 2^24 buckets by
    the multiplicative hash; counted here on the host from the oracle's
    ordered tensor."""
    coords, vals = synth.coo(rec)
    c, v = to_dev(coords, vals)
    t = alto.AltoTensor.build(c, v, rec.dims)
    (lo, hi), _, lay, _ = oracle_alto(rec.dims, coords, vals)
    M = len(lo)
    assert t.info()["nnz"] == M
    S = min(M, 1 << 20)
    idx = np.arange(S, dtype=np.int64) * M // S
    rows = oracle.decode(lay, (lo[idx], hi[idx]))
    for mode, I in enumerate(rec.dims):
        nb = min(I, 1 << 24)
        r = rows[mode].astype(np.uint64)
        b = r if nb == I else (((r * np.uint64(2654435769)) & np.uint64(0xffffffff)) * np.uint64(nb)) >> np.uint64(32)
        cnt = np.bincount(b.astype(np.int64), minlength=1)
        hot = np.log2(max(1, cnt.max()) * I / S)
        distinct = np.log2(max(1, np.count_nonzero(cnt)) / min(S, nb))
        f = t.selector_features(mode, 16, "f32")
        print(rec.name, mode, f[12], hot, f[13], distinct, flush=True)
        assert f[12] == pytest.approx(hot, rel=1e-6, abs=1e-6)
        assert f[13] == pytest.approx(distinct, rel=1e-6, abs=1e-6)
    t.close()
