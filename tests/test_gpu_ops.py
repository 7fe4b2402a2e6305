"""Operations on the format beyond MTTKRP, through the C ABI, against the
oracle: sparse tensor transposition (lexicographic order of permuted
coordinates, bit for bit), incremental format generation (append) and
streaming CP-ALS on a growing tensor."""
import numpy as np
import pytest

import oracle
import paper_2102_10245_amd as alto
import synth
from gpu_common import factors_dev, gpu_ok, keys_numpy, oracle_alto, rel_fro, small, to_dev

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_ok(), reason="needs a GPU")]

TRANSPOSE_CASES = [
    # (recipe, permutations)
    (synth.WORKLOADS["uniform3_1000x800x600_100k"], [(0, 1, 2), (2, 1, 0), (1, 2, 0)]),            # 32-bit index
    (small("zipf4_1Mx100kx10kx500_150M", 300_000), [(3, 2, 1, 0), (1, 0, 3, 2)]),                  # 64-bit
    (small("zipf5_10Mx5Mx2Mx100kx1k_200M", 200_000), [(4, 3, 2, 1, 0), (2, 0, 4, 1, 3)]),          # 95 of 128 bits
    (synth.Recipe("order2", (5000, 3000), 40_000, (1.0, 0), seed=5), [(1, 0)]),
    (synth.Recipe("unit_modes", (1, 700, 1, 90), 30_000, (0, 1.1, 0, 0), seed=26), [(3, 0, 2, 1)]),  # repeats
]


@pytest.mark.parametrize("rec,perms", TRANSPOSE_CASES, ids=[c[0].name for c in TRANSPOSE_CASES])
def test_transpose_matches_oracle(rec, perms):
    coords, vals = synth.coo(rec)
    c, v = to_dev(coords, vals)
    t = alto.AltoTensor.build(c, v, rec.dims)
    M = t.info()["nnz"]
    for perm in perms:
        print("transpose", rec.name, perm, flush=True)
        gc, gv = t.transpose(perm)
        oc, ov = oracle.transpose(coords, vals, perm)
        assert gc.shape[1] == M == oc.shape[1]
        assert np.array_equal(gc.cpu().numpy().view(np.uint32), oc), perm
        gv = gv.cpu().numpy().astype(np.float64)
        if M == rec.nnz:
            assert np.array_equal(gv, ov)  # a permutation of the inputs, bit for bit
        else:
            assert np.allclose(gv, ov, rtol=2e-6, atol=0)  # FP32 sums of repeated coordinates
    t.close()


def test_transpose_errors_and_empty():
    import torch
    rec = synth.Recipe("small", (30, 20, 10), 500, (), seed=3)
    coords, vals = synth.coo(rec)
    c, v = to_dev(coords, vals)
    t = alto.AltoTensor.build(c, v, rec.dims)
    with pytest.raises(ValueError):
        t.transpose((0, 0, 1))
    import ctypes
    L = alto.lib()
    bad = (ctypes.c_int * 3)(0, 3, 1)
    out = [torch.empty(500, dtype=torch.int32, device="cuda") for _ in range(3)]
    vo = torch.empty(500, dtype=torch.float32, device="cuda")
    assert L.alto_transpose(t._h, bad, alto._ptr_array(out), alto._ptr(vo), None) == alto.E_INVAL
    t.close()
    e = alto.AltoTensor.build(torch.zeros((3, 0), dtype=torch.int32, device="cuda"),
                              torch.zeros(0, dtype=torch.float32, device="cuda"), (4, 5, 6))
    gc, gv = e.transpose((2, 0, 1))
    assert gc.shape == (3, 0) and gv.shape == (0,)
    e.close()


APPEND_CASES = [
    # (recipe, number of batches, requested L)
    (small("zipf4_1Mx100kx10kx500_150M", 200_000), 4, 1024),
    (small("zipf5_10Mx5Mx2Mx100kx1k_200M", 100_000), 3, 0),        # 128-bit index
    (synth.Recipe("repeats", (50, 40, 30), 60_000, (1.1, 0.5, 0), seed=9), 3, 64),  # many repeated coordinates
]


@pytest.mark.parametrize("rec,nb,L", APPEND_CASES, ids=[c[0].name for c in APPEND_CASES])
def test_append_equals_build_of_concatenation(rec, nb, L):
    """Building from the first part and appending the rest, batch by batch,
    gives the tensor alto_build makes from the whole COO list, bit for bit:
    index, values, norm, segments, intervals, coverage and the selector's
    features."""
    import torch
    coords, vals = synth.coo(rec)
    M = coords.shape[1]
    cuts = [0] + [M * (k + 1) // (nb + 1) for k in range(nb)] + [M]
    c, v = to_dev(coords[:, :cuts[1]], vals[:cuts[1]])
    t = alto.AltoTensor.build(c, v, rec.dims, num_segments=L)
    for k in range(1, nb + 1):
        c, v = to_dev(coords[:, cuts[k]:cuts[k + 1]], vals[cuts[k]:cuts[k + 1]])
        t.append(c, v)
    ca, va = to_dev(coords, vals)
    ref = alto.AltoTensor.build(ca, va, rec.dims, num_segments=L)
    gi, ri = t.info(), ref.info()
    for k in ("nnz", "nnz_in", "num_segments", "index_bits", "key_bits"):
        assert gi[k] == ri[k], k
    assert gi["norm2"] == ri["norm2"]
    gk, gv = t.export_keys()
    rk, rv = ref.export_keys()
    assert torch.equal(gk, rk) and torch.equal(gv, rv)
    gs, gl = t.export_partition()
    rs, rl = ref.export_partition()
    assert torch.equal(gs, rs) and torch.equal(gl, rl)
    for n in range(len(rec.dims)):
        assert torch.equal(t.export_coverage(n), ref.export_coverage(n))
        # the selector's features, the row-count ones included
        assert np.array_equal(t.selector_features(n, 16, "f32"), ref.selector_features(n, 16, "f32"))
    # and the keys are the oracle's
    (olo, ohi), _, lay, _ = oracle_alto(rec.dims, coords, vals)
    glo, ghi = keys_numpy(gk, gi["key_bits"])
    assert np.array_equal(glo, olo) and np.array_equal(ghi, ohi)
    t.close()
    ref.close()


def test_streaming_cp_als_tracks_the_oracle():
    """Streaming decomposition in its simplest form: the tensor grows by
    batches (alto_append) and after each batch CP-ALS is warm-started from
    the previous factors; every refit matches the FP64 oracle run on the
    COO list seen so far from the same starting factors."""
    rec = small("zipf4_1Mx100kx10kx500_150M", 120_000)
    coords, vals = synth.coo(rec)
    M = coords.shape[1]
    R, iters = 8, 3
    fs = synth.factors(rec.seed + 1, rec.dims, R)
    cuts = [0, M // 3, 2 * M // 3, M]
    t = None
    fd = factors_dev(fs, "f32")
    for k in range(3):
        c, v = to_dev(coords[:, cuts[k]:cuts[k + 1]], vals[cuts[k]:cuts[k + 1]])
        if t is None:
            t = alto.AltoTensor.build(c, v, rec.dims)
        else:
            t.append(c, v)
        seen = cuts[k + 1]
        # the oracle starts from the factors the GPU holds now (FP32 values)
        start = [f.cpu().numpy().astype(np.float64) for f in fd]
        oA, olam, ofit = oracle.cp_als(rec.dims, coords[:, :seen], vals[:seen], start, iters)
        lam, fit = t.cp_als(fd, iters)
        print("batch", k, "fit", fit, "oracle", ofit, flush=True)
        assert np.all(np.abs(fit - ofit) <= 1e-5)
        assert np.allclose(lam.cpu().numpy(), olam, rtol=1e-3)
        for f, a in zip(fd, oA):
            assert rel_fro(f.cpu().numpy(), a) <= 1e-3
    t.close()
