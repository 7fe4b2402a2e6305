"""Helper flags (Section 3.3): the spare index bits that mark a nonzero as
internal along a mode of limited fiber reuse, so that the atomic strategy
writes its row without atomics.  Through the C ABI against the definition
computed from the oracle's ordered tensor and partition: a nonzero is
internal iff every nonzero of its row lies in the same lane-group range of
the launch (bit for bit); MTTKRP parity with the flags in use; modes of
higher reuse get no flags."""
import os

import numpy as np
import pytest

import oracle
import paper_2102_10245_amd as alto
import synth
from gpu_common import factors_dev, gpu_ok, keys_numpy, oracle_alto, rel_fro, small, to_dev

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_ok(), reason="needs a GPU")]

FLAG_CASES = [
    # a limited-reuse tensor of darpa's shape (Table 1): 22.5K x 22.5K x 23.8M
    (synth.Recipe("darpa_shape", (22_500, 22_500, 23_800_000), 400_000, (1.0, 1.0, 0.5), seed=31), 8, 256),
    (small("zipf3_2Mx2Mx20k_50M", 300_000), 16, 512),
    (small("zipf5_10Mx5Mx2Mx100kx1k_200M", 200_000), 32, 1024),  # 128-bit index
    (synth.Recipe("generic_rank_r24", (400_000, 300_000, 2000), 150_000, (0.8, 0, 0), seed=32), 24, 100),
    # segments of ~15 nonzeros cut into many lane groups, most of them empty
    (synth.Recipe("tiny_segments", (100_000, 80_000, 600), 30_000, (0, 0, 0), seed=33), 32, 2048),
]


def flag_definition(dims, coords, vals, L, G, mode):
    """Internal flag of every nonzero (tensor order): all nonzeros of its row
    lie in one lane-group range (segment l's offsets o with
    floor(S*g/G) <= o < floor(S*(g+1)/G))."""
    (lo, hi), _, lay, _ = oracle_alto(dims, coords, vals)
    M = len(lo)
    seg = oracle.partition(M, L)
    chunk = np.empty(M, np.int64)
    for l in range(len(seg) - 1):
        S = int(seg[l + 1] - seg[l])
        o = np.arange(S, dtype=np.int64)
        g = np.searchsorted((S * np.arange(1, G + 1, dtype=np.int64)) // G, o, side="right")
        chunk[seg[l]:seg[l + 1]] = l * G + g
    rows = oracle.decode(lay, (lo, hi))[mode].astype(np.int64)
    lo_c = np.full(dims[mode], np.iinfo(np.int64).max)
    hi_c = np.full(dims[mode], -1)
    np.minimum.at(lo_c, rows, chunk)
    np.maximum.at(hi_c, rows, chunk)
    return lo_c[rows] == hi_c[rows]


@pytest.mark.parametrize("rec,R,L", FLAG_CASES, ids=[c[0].name for c in FLAG_CASES])
def test_helper_flags_match_definition_and_mttkrp_parity(rec, R, L):
    coords, vals = synth.coo(rec)
    c, v = to_dev(coords, vals)
    t = alto.AltoTensor.build(c, v, rec.dims, num_segments=L)
    info = t.info()
    fs = synth.factors(rec.seed + 1, rec.dims, R)
    flagged_modes = 0
    for prec in ("f32", "bf16"):
        fd = factors_dev(fs, prec)
        for mode in range(len(rec.dims)):
            print("flags", rec.name, prec, "mode", mode, flush=True)
            out = t.mttkrp(fd, mode, strategy="atomic").cpu().numpy()
            ref = oracle.mttkrp(rec.dims, coords, vals, fs, mode)
            assert rel_fro(out, ref) <= 1e-5, (mode, prec)
            limited = info["nnz"] <= 4 * rec.dims[mode]
            if info["flag_bit"][mode] < 0 or not limited:
                with pytest.raises(alto.AltoError) as e:
                    t.export_flags(mode)
                assert e.value.code == alto.E_STATE
                continue
            flags, G = t.export_flags(mode)
            flags = flags.cpu().numpy().astype(bool)
            exp = flag_definition(rec.dims, coords, vals, L, G, mode)
            assert np.array_equal(flags, exp), (mode, prec)
            flagged_modes += 1
            print(f"  {flags.mean():.3f} of the nonzeros internal ({G} lane groups per segment)", flush=True)
    assert flagged_modes > 0
    # the index and its exports are unchanged by the flags
    keys, _ = t.export_keys()
    (olo, ohi), _, _, _ = oracle_alto(rec.dims, coords, vals)
    glo, ghi = keys_numpy(keys, info["key_bits"])
    assert np.array_equal(glo, olo) and np.array_equal(ghi, ohi)
    t.close()


def test_helper_flags_off_gives_the_same_result():
    rec = FLAG_CASES[0][0]
    coords, vals = synth.coo(rec)
    c, v = to_dev(coords, vals)
    t = alto.AltoTensor.build(c, v, rec.dims, num_segments=256)
    fd = factors_dev(synth.factors(5, rec.dims, 16))
    on = t.mttkrp(fd, 2, strategy="atomic").cpu().numpy()
    os.environ["ALTO_HELPER_FLAGS"] = "0"
    try:
        off = t.mttkrp(fd, 2, strategy="atomic").cpu().numpy()
    finally:
        del os.environ["ALTO_HELPER_FLAGS"]
    assert rel_fro(on, off) <= 1e-6
    # a re-partition computes the flags again for the new lane-group ranges
    t.partition(1000)
    again = t.mttkrp(fd, 2, strategy="atomic").cpu().numpy()
    assert rel_fro(again, on) <= 1e-6
    t.close()
