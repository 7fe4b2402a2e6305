"""GPU CP-ALS vs the FP64 oracle: per-iteration fit, lambda and factors with
FP32 and BF16 factors (a planted rank-32 tensor of the headline shape),
exact-rank recovery, and the normalization invariants."""
import numpy as np
import pytest

import oracle
import paper_2102_10245_amd as alto
import synth
from gpu_common import factors_dev, gpu_ok, rel_fro, to_dev

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_ok(), reason="needs a GPU")]


def test_cp_als_fit_matches_oracle():
    rec = synth.WORKLOADS["uniform3_1000x800x600_100k"]
    coords, vals = synth.coo(rec)
    c, v = to_dev(coords, vals)
    t = alto.AltoTensor.build(c, v, rec.dims)
    init = synth.factors(rec.seed + 1, rec.dims, rec.rank)
    oA, olam, ofit = oracle.cp_als(rec.dims, coords, vals, init, 5)
    fd = factors_dev(init, "f32")
    lam, fit = t.cp_als(fd, 5)
    print("fit", fit, "oracle", ofit, flush=True)
    assert np.all(np.abs(fit - ofit) <= 1e-5)
    assert np.allclose(lam.cpu().numpy(), olam, rtol=1e-3)
    for f, a in zip(fd, oA):
        assert rel_fro(f.cpu().numpy(), a) <= 1e-3
        assert np.allclose(f.norm(dim=0).cpu().numpy(), 1.0, atol=1e-5)
    t.close()


def test_cp_als_four_modes_skewed():
    rec = synth.scaled(synth.WORKLOADS["zipf4_1Mx100kx10kx500_150M"], 400_000)
    coords, vals = synth.coo(rec)
    c, v = to_dev(coords, vals)
    t = alto.AltoTensor.build(c, v, rec.dims)
    init = synth.factors(rec.seed + 1, rec.dims, 8)
    oA, olam, ofit = oracle.cp_als(rec.dims, coords, vals, init, 3)
    fd = factors_dev(init, "f32")
    lam, fit = t.cp_als(fd, 3)
    print("fit", fit, "oracle", ofit, flush=True)
    assert np.all(np.abs(fit - ofit) <= 1e-5)
    assert np.allclose(lam.cpu().numpy(), olam, rtol=1e-3)
    for f, a in zip(fd, oA):
        assert rel_fro(f.cpu().numpy(), a) <= 1e-3
    t.close()


# The headline shape (1M x 100k x 10k x 500, Zipf(1.2) coordinates on modes 0
# and 1, R = 32, 20 iterations) with values that have rank-32 structure: a
# planted sum of 32 sparse rank-1 terms (50 x 25 x 10 x 5 boxes of rows drawn
# from the modes' distributions, so the terms share hot rows) times a 10%
# relative noise, 2M nonzeros.  CP-ALS starts from the planted factors with
# a jitter as large as the weights themselves (fit 0.40 after the first
# iteration, 0.83 after the second) and converges to fit 0.9007, the noise
# floor.  From random starts the iteration on this tensor is chaotic: a
# 1e-7 relative change of the start moves the fit by 1e-5 and lambda by
# 3e-4 (measured with the oracle), so there FP32 rounding alone would exceed
# any useful tolerance.  Emulating FP32 and BF16 factor storage on the
# oracle's iteration from this start gives fit differences of 4e-8 / 9e-5,
# lambda 3e-8 / 1.4e-3 and factors 4e-8 / 1.7e-3 relative.
PLANTED_DIMS = (1_000_000, 100_000, 10_000, 500)
PLANTED_R = 32
PLANTED_ITERS = 20


@pytest.fixture(scope="module")
def planted():
    coords, vals, truth = synth.planted_cp(PLANTED_DIMS, PLANTED_R, (50, 25, 10, 5), (1.2, 1.2, 0, 0),
                                           noise=0.1)
    init = synth.planted_start(truth, 1.0)
    print("planted tensor:", coords.shape[1], "nonzeros; FP64 oracle CP-ALS ...", flush=True)
    oA, olam, ofit = oracle.cp_als(PLANTED_DIMS, coords, vals, init, PLANTED_ITERS)
    print("oracle fit", ofit, flush=True)
    return coords, vals, init, oA, olam, ofit


# tolerances against the FP64 oracle: FP32 factors (FP32 MTTKRP accumulation,
# FP32 storage) and BF16 factors (8-bit mantissa storage, FP32 accumulation)
PLANTED_TOL = {"f32": {"fit": 1e-5, "lam": 1e-4, "fac": 1e-4},
               "bf16": {"fit": 1e-3, "lam": 1e-2, "fac": 1e-2}}


@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_cp_als_planted_headline_shape(planted, prec):
    coords, vals, init, oA, olam, ofit = planted
    assert ofit[-1] >= 0.85 and ofit[0] <= 0.5  # a real trajectory to a meaningful fit
    c, v = to_dev(coords, vals)
    t = alto.AltoTensor.build(c, v, PLANTED_DIMS)
    fd = factors_dev(init, prec)
    lam, fit = t.cp_als(fd, PLANTED_ITERS)
    lam = lam.cpu().numpy()
    dfit = np.abs(fit - ofit)
    dlam = np.abs(lam - olam) / np.abs(olam)
    dfac = [rel_fro(f.float().cpu().numpy(), a) for f, a in zip(fd, oA)]
    print(f"planted {prec}: fit {fit[-1]:.6f} (oracle {ofit[-1]:.6f}); max |dfit| {dfit.max():.2e} "
          f"at iteration {int(dfit.argmax())}; max lambda rel {dlam.max():.2e}; factor rel fro "
          + " ".join(f"{e:.2e}" for e in dfac), flush=True)
    tol = PLANTED_TOL[prec]
    assert dfit.max() <= tol["fit"], (prec, fit, ofit)
    assert dlam.max() <= tol["lam"], (prec, lam, olam)
    assert max(dfac) <= tol["fac"], (prec, dfac)
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


@pytest.mark.parametrize("R", [8, 32, 64])
def test_cp_als_ridge_retry_matches_oracle(R):
    """Column 3 of the start is zero in modes 1 and 2, so every normal-equation
    matrix of the sweeps has a zero row and column: each update takes the
    ridge retry (1e-10 tr(V)/R on the diagonal), on the GPU (Gauss-Jordan,
    pivot <= 0) as in the oracle (Cholesky).  Column 3 stays zero with
    lambda 0; the other columns, fit and lambda match the oracle.  R = 8 and
    32 solve in one wave, R = 64 in a workgroup over LDS."""
    rec = synth.scaled(synth.WORKLOADS["uniform3_1000x800x600_100k"], 30_000)
    coords, vals = synth.coo(rec)
    c, v = to_dev(coords, vals)
    t = alto.AltoTensor.build(c, v, rec.dims)
    init = synth.factors(rec.seed + 3, rec.dims, R)
    init[1][:, 3] = 0.0
    init[2][:, 3] = 0.0
    oA, olam, ofit = oracle.cp_als(rec.dims, coords, vals, init, 2)
    fd = factors_dev(init)
    lam, fit = t.cp_als(fd, 2)
    lam = lam.cpu().numpy()
    print("ridge R", R, "fit", fit, "oracle", ofit, "lambda_3", lam[3], olam[3], flush=True)
    assert np.all(np.abs(fit - ofit) <= 1e-5)
    assert olam[3] == 0.0 and lam[3] == 0.0
    keep = np.arange(R) != 3
    assert np.allclose(lam[keep], olam[keep], rtol=1e-3)
    for f, a in zip(fd, oA):
        f = f.cpu().numpy()
        assert np.all(f[:, 3] == 0.0) and np.all(a[:, 3] == 0.0)
        assert rel_fro(f, a) <= 1e-3
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
