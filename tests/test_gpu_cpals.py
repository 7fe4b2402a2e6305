"""GPU CP-ALS vs the FP64 oracle: fit within 1e-3 (FP32 and BF16 factors),
exact-rank recovery, and the normalization invariants."""
import numpy as np
import pytest

import oracle
import paper_2102_10245_amd as alto
import synth
from gpu_common import factors_dev, gpu_ok, rel_fro, to_dev

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_ok(), reason="needs a GPU")]


@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_cp_als_fit_matches_oracle(prec):
    rec = synth.WORKLOADS["uniform3_1000x800x600_100k"]
    coords, vals = synth.coo(rec)
    c, v = to_dev(coords, vals)
    t = alto.AltoTensor.build(c, v, rec.dims)
    init = synth.factors(rec.seed + 1, rec.dims, rec.rank)
    _, olam, ofit = oracle.cp_als(rec.dims, coords, vals, init, 5)
    fd = factors_dev(init, prec)
    lam, fit = t.cp_als(fd, 5)
    print("fit", prec, fit, "oracle", ofit, flush=True)
    assert np.all(np.abs(fit - ofit) <= 1e-3)
    if prec == "f32":
        assert np.all(np.abs(fit - ofit) <= 1e-5)
        assert np.allclose(lam.cpu().numpy(), olam, rtol=1e-3)
    for f in fd:
        norms = f.float().norm(dim=0).cpu().numpy()
        assert np.allclose(norms, 1.0, atol=1e-2 if prec == "bf16" else 1e-5)
    t.close()


def test_cp_als_four_modes_skewed():
    rec = small_rec = synth.scaled(synth.WORKLOADS["zipf4_1Mx100kx10kx500_150M"], 400_000)
    coords, vals = synth.coo(rec)
    c, v = to_dev(coords, vals)
    t = alto.AltoTensor.build(c, v, rec.dims)
    init = synth.factors(rec.seed + 1, rec.dims, 8)
    _, _, ofit = oracle.cp_als(rec.dims, coords, vals, init, 3)
    for prec in ("f32", "bf16"):
        lam, fit = t.cp_als(factors_dev(init, prec), 3)
        assert np.all(np.abs(fit - ofit) <= 1e-3), (prec, fit, ofit)
    t.close()


def test_cp_als_exact_rank_recovery():
    rng = np.random.default_rng(21)
    dims = (12, 10, 8)
    R = 3
    fs = [rng.standard_normal((d, R)) for d in dims]
    X = np.einsum("ir,jr,kr->ijk", *fs)
    idx = np.nonzero(np.ones(dims))
    coords = np.stack(idx).astype(np.uint32)
    vals = X[idx].astype(np.float32)
    c, v = to_dev(coords, vals)
    t = alto.AltoTensor.build(c, v, dims, num_segments=16)
    init = [rng.random((d, R)).astype(np.float32) for d in dims]
    fd = factors_dev(init)
    lam, fit = t.cp_als(fd, 100)
    # the fit formula resolves about sqrt(2 * 1e-7) near 1 with FP32 MTTKRP outputs
    assert fit[-1] >= 1 - 1e-3
    # the direct residual of the reconstruction is the sharper check
    A = [f.cpu().numpy().astype(np.float64) for f in fd]
    Xhat = np.einsum("r,ir,jr,kr->ijk", lam.cpu().numpy(), *A)
    assert np.linalg.norm(Xhat - X) / np.linalg.norm(X) <= 1e-4
    t.close()


def test_cp_als_zero_iterations_and_errors():
    rec = synth.Recipe("z", (20, 10, 5), 200, (), seed=2)
    coords, vals = synth.coo(rec)
    c, v = to_dev(coords, vals)
    t = alto.AltoTensor.build(c, v, rec.dims)
    fd = factors_dev(synth.factors(3, rec.dims, 4))
    lam, fit = t.cp_als(fd, 0)
    assert fit.shape == (0,)
    t.close()


@pytest.mark.parametrize("R", [5, 8, 16, 32, 64, 96, 160])
def test_cp_als_ranks_match_oracle(R):
    # ranks with a specialized update (8, 16, 32, 64) and the generic one, with
    # the normal equations in LDS (R <= 128) and in device memory (160)
    rec = synth.scaled(synth.WORKLOADS["uniform3_1000x800x600_100k"], 30_000)
    coords, vals = synth.coo(rec)
    c, v = to_dev(coords, vals)
    t = alto.AltoTensor.build(c, v, rec.dims)
    init = synth.factors(rec.seed + 7, rec.dims, R)
    oA, olam, ofit = oracle.cp_als(rec.dims, coords, vals, init, 3)
    fd = factors_dev(init)
    lam, fit = t.cp_als(fd, 3)
    print("R", R, "fit", fit, "oracle", ofit, flush=True)
    assert np.all(np.abs(fit - ofit) <= 1e-5)
    assert np.allclose(lam.cpu().numpy(), olam, rtol=1e-3)
    for f, a in zip(fd, oA):
        assert rel_fro(f.cpu().numpy(), a) <= 1e-3
    t.close()


@pytest.mark.parametrize("R,rows", [(16, 330_001), (32, 200_003), (64, 60_001)])
def test_cp_als_tall_mode_matches_oracle(R, rows):
    # a tall mode: the blocks of the row-solve passes stream more tiles than
    # the loads they keep in flight (on a 256-CU GPU), with a ragged last tile
    rec = synth.Recipe("tall", (rows, 300, 200), 150_000, (0.8, 0, 0), seed=11)
    coords, vals = synth.coo(rec)
    c, v = to_dev(coords, vals)
    t = alto.AltoTensor.build(c, v, rec.dims)
    init = synth.factors(rec.seed + 1, rec.dims, R)
    oA, olam, ofit = oracle.cp_als(rec.dims, coords, vals, init, 2)
    fd = factors_dev(init)
    lam, fit = t.cp_als(fd, 2)
    print("tall R", R, "fit", fit, "oracle", ofit, flush=True)
    assert np.all(np.abs(fit - ofit) <= 1e-5)
    assert np.allclose(lam.cpu().numpy(), olam, rtol=1e-3)
    for f, a in zip(fd, oA):
        assert rel_fro(f.cpu().numpy(), a) <= 1e-3
    t.close()


def test_cp_als_singular_normal_equations():
    # all-zero factors: every Gram is zero, so is the ridge, and the normal
    # equations stay singular -> ALTO_E_NOTSPD
    rec = synth.Recipe("z", (30, 20, 10), 500, (), seed=4)
    coords, vals = synth.coo(rec)
    c, v = to_dev(coords, vals)
    t = alto.AltoTensor.build(c, v, rec.dims)
    for R in (4, 32):
        fd = factors_dev([np.zeros((d, R), np.float32) for d in rec.dims])
        with pytest.raises(alto.AltoError) as e:
            t.cp_als(fd, 2)
        assert e.value.code == alto.E_NOTSPD
    t.close()
