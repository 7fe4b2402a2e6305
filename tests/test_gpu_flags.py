"""Helper flags (Section 3.3): the spare index bits that mark a nonzero as
internal along a mode, so that the atomic strategy writes its row without
atomics.  Through the C ABI against the oracle: the flags bit for bit (the
definition over the lane-group ranges of the launch, from the oracle's own
partition and intervals), that every flagged row really is touched by one
lane group only, and MTTKRP parity with the flags in use."""
import os

import numpy as np
import pytest

import oracle
import paper_2102_10245_amd as alto
import synth
from gpu_common import factors_dev, gpu_ok, oracle_alto, rel_fro, small, to_dev

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_ok(), reason="needs a GPU")]

FLAG_CASES = [
    # a limited-reuse tensor of darpa's shape (Table 1): 22.5K x 22.5K x 23.8M
    (synth.Recipe("darpa_shape", (22_500, 22_500, 23_800_000), 400_000, (1.0, 1.0, 0.5), seed=31), 8, 256),
    (small("zipf3_2Mx2Mx20k_50M", 300_000), 16, 512),
    (small("zipf5_10Mx5Mx2Mx100kx1k_200M", 200_000), 32, 1024),  # 128-bit index
    (synth.Recipe("generic_rank_r24", (4000, 3000, 2000), 150_000, (0.8, 0, 0), seed=32), 24, 100),
    # segments of ~15 nonzeros cut into 32 lane groups: most lane groups are
    # empty and have no interval (their coverage marks must be skipped)
    (synth.Recipe("tiny_segments", (1000, 800, 600), 30_000, (0, 0, 0), seed=33), 32, 2048),
]


def oracle_flags(dims, coords, vals, L, G, mode):
    """Flag of every nonzero (tensor order) by the definition: its row lies in
    the mode interval of one lane-group range only."""
    (lo, hi), _, lay, _ = oracle_alto(dims, coords, vals)
    M = len(lo)
    seg = oracle.partition(M, L)
    micro = []
    for l in range(len(seg) - 1):
        S = int(seg[l + 1] - seg[l])
        micro += [int(seg[l]) + (S * g) // G for g in range(G)]
    micro = np.array(micro + [M], np.int64)
    ivl = oracle.intervals(lay, micro, (lo, hi))
    rows = oracle.decode(lay, (lo, hi))[mode]
    # intervals holding row r = #(starts <= r) - #(ends < r); at these sizes
    # this replaces the oracle's per-row loop over every interval
    s0 = ivl[:, mode, 0].astype(np.int64)
    e0 = ivl[:, mode, 1].astype(np.int64)
    live = s0 <= e0  # a lane group with no nonzeros has no interval
    starts = np.sort(s0[live])
    ends = np.sort(e0[live])
    r = rows.astype(np.int64)
    cover = np.searchsorted(starts, r, side="right") - np.searchsorted(ends, r, side="left")
    return cover == 1, micro, rows


@pytest.mark.parametrize("rec,R,L", FLAG_CASES, ids=[c[0].name for c in FLAG_CASES])
def test_helper_flags_match_oracle_and_mttkrp_parity(rec, R, L):
    coords, vals = synth.coo(rec)
    c, v = to_dev(coords, vals)
    t = alto.AltoTensor.build(c, v, rec.dims, num_segments=L)
    info = t.info()
    fs = synth.factors(rec.seed + 1, rec.dims, R)
    for prec in ("f32", "bf16"):
        fd = factors_dev(fs, prec)
        for mode in range(len(rec.dims)):
            print("flags", rec.name, prec, "mode", mode, flush=True)
            out = t.mttkrp(fd, mode, strategy="atomic").cpu().numpy()
            ref = oracle.mttkrp(rec.dims, coords, vals, fs, mode)
            assert rel_fro(out, ref) <= 1e-5, (mode, prec)
            if info["flag_bit"][mode] < 0:
                continue
            flags, G = t.export_flags(mode)
            flags = flags.cpu().numpy().astype(bool)
            exp, micro, rows = oracle_flags(rec.dims, coords, vals, L, G, mode)
            assert np.array_equal(flags, exp), (mode, prec)
            # a flagged row has all its nonzeros in one lane-group range
            chunk = np.searchsorted(micro, np.arange(len(rows)), side="right") - 1
            fr = rows[flags]
            fc = chunk[flags]
            order = np.argsort(fr, kind="stable")
            fr, fc = fr[order], fc[order]
            same = fr[1:] == fr[:-1]
            assert np.all(fc[1:][same] == fc[:-1][same])
            counts = np.bincount(rows, minlength=rec.dims[mode])
            fcount = np.bincount(fr, minlength=rec.dims[mode])
            assert np.all(fcount[np.unique(fr)] == counts[np.unique(fr)])
            print(f"  {flags.mean():.3f} of the nonzeros flagged internal ({G} lane groups per segment)",
                  flush=True)
    # the index and its exports are unchanged by the flags
    keys, _ = t.export_keys()
    (olo, ohi), _, _, _ = oracle_alto(rec.dims, coords, vals)
    from gpu_common import keys_numpy
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
