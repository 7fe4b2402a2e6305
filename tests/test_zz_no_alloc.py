"""alto_mttkrp_noalloc (the entry point for callers that cannot allocate)
against alto_mttkrp with the atomic strategy and against the FP64 oracle,
through the C ABI: two calls in a row, the second on a smaller tensor, so
that what the first call left in the shared static scratch must not leak
into the second; and the size limit of that scratch."""
import numpy as np
import pytest

import oracle
import paper_2102_10245_amd as alto
import synth
from gpu_common import factors_dev, gpu_ok, rel_fro, to_dev

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_ok(), reason="needs a GPU")]


def _case(rec, prec):
    import torch
    coords, vals = synth.coo(rec)
    c, v = to_dev(coords, vals)
    t = alto.AltoTensor.build(c, v, rec.dims)
    fs = synth.factors(rec.seed + 3, rec.dims, rec.rank)
    fd = factors_dev(fs, prec)
    res = []
    for mode in range(len(rec.dims)):
        print(f"noalloc {rec.name} {prec} mode {mode}", flush=True)
        out = torch.full((rec.dims[mode], rec.rank), 7.0, dtype=torch.float32, device="cuda")
        t.mttkrp_noalloc(fd, mode, out)
        ref = t.mttkrp(fd, mode, strategy="atomic")
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        exp = ref.cpu().numpy()
        orc = oracle.mttkrp(rec.dims, coords, vals, fs, mode)
        res.append((rel_fro(got, exp), rel_fro(got, orc)))
    t.close()
    return res


def test_noalloc_matches_atomic_entry_point_twice():
    first = synth.WORKLOADS["uniform3_1000x800x600_100k"]            # 1000 x 16 outputs
    # smaller in every respect: 30k nonzeros, outputs of at most 500 x 8
    second = synth.Recipe("zipf4_small", (500, 400, 300, 50), 30_000, (1.2, 1.2, 0, 0),
                          "lognormal", seed=77, rank=8)
    for rec, prec in ((first, "f32"), (second, "f32"), (second, "bf16")):
        for mode, (e_entry, e_oracle) in enumerate(_case(rec, prec)):
            assert e_entry <= 1e-5, (rec.name, prec, mode, e_entry)
            assert e_oracle <= 1e-5, (rec.name, prec, mode, e_oracle)


def test_noalloc_rejects_outputs_beyond_the_scratch():
    import torch
    rec = synth.Recipe("tallmode", (400_000, 50, 40), 5_000, (0, 0, 0), seed=5, rank=32)
    coords, vals = synth.coo(rec)
    c, v = to_dev(coords, vals)
    t = alto.AltoTensor.build(c, v, rec.dims)
    fd = factors_dev(synth.factors(9, rec.dims, 32))
    out = torch.empty((rec.dims[0], 32), dtype=torch.float32, device="cuda")
    with pytest.raises(alto.AltoError) as e:
        t.mttkrp_noalloc(fd, 0, out)  # 400k x 32 x 4 B per replica: beyond 32 MiB
    assert e.value.code == alto.E_INVAL
    assert "scratch" in str(e.value)
    # a short mode of the same tensor fits
    out1 = torch.empty((rec.dims[1], 32), dtype=torch.float32, device="cuda")
    t.mttkrp_noalloc(fd, 1, out1)
    exp = oracle.mttkrp(rec.dims, coords, vals, synth.factors(9, rec.dims, 32), 1)
    assert rel_fro(out1.cpu().numpy(), exp) <= 1e-5
    t.close()
