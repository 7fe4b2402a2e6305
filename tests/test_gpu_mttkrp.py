"""GPU MTTKRP vs the FP64 oracle (relative Frobenius error <= 1e-5 for the
FP32 path; the BF16 path reads factors that are exact in bfloat16, so the
same bound applies to it against the oracle on those factors)."""
import numpy as np
import pytest

import oracle
import paper_2102_10245_amd as alto
import synth
from gpu_common import factors_dev, gpu_ok, rel_fro, small, to_dev

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_ok(), reason="needs a GPU")]

TOL = 1e-5

CASES = [
    (synth.WORKLOADS["uniform3_1000x800x600_100k"], 16, 0),
    (small("zipf3_2Mx2Mx20k_50M", 400_000), 16, 0),
    (small("zipf3_2Mx2Mx20k_50M", 300_000), 64, 0),
    (small("zipf4_1Mx100kx10kx500_150M", 600_000), 32, 0),
    (small("zipf5_10Mx5Mx2Mx100kx1k_200M", 300_000), 32, 0),
    (synth.Recipe("r8_order3", (300, 200, 100), 80_000, (1.0, 0, 0.5), seed=21), 8, 100),
    (synth.Recipe("generic_r24", (500, 400, 30), 50_000, (0.9, 0.3, 0), seed=22), 24, 0),
    (synth.Recipe("generic_r5_order2", (3000, 2000), 60_000, (1.2, 0), seed=23), 5, 64),
    (synth.Recipe("generic_r100_order6", (20, 18, 16, 14, 12, 10), 40_000, (0.7,) * 6, seed=24), 100, 77),
    (synth.Recipe("r256", (400, 300, 20), 20_000, (0, 0.8, 0), seed=25), 256, 0),
    (synth.Recipe("unit_modes", (1, 700, 1, 90), 30_000, (0, 1.1, 0, 0), seed=26), 16, 0),
    # segments of at least 64K nonzeros: factor matrices of 500 rows (R = 32)
    # and of 600 rows (R = 16) are gathered from LDS in 1024-thread workgroups
    (small("zipf4_1Mx100kx10kx500_150M", 400_000), 32, 3),
    (synth.Recipe("uniform3_staged_r16", (1000, 800, 600), 300_000, (), seed=27), 16, 4),
    (synth.Recipe("staged_r64", (3000, 2000, 200), 200_000, (1.1, 0.5, 0), seed=28), 64, 2),
]


def _run_case(rec, R, L, strategies=("atomic", "staged", "sorted", "auto"), precs=("f32", "bf16")):
    coords, vals = synth.coo(rec)
    c, v = to_dev(coords, vals)
    t = alto.AltoTensor.build(c, v, rec.dims, num_segments=L)
    fs = synth.factors(rec.seed + 1, rec.dims, R)
    for mode in range(len(rec.dims)):
        ref = oracle.mttkrp(rec.dims, coords, vals, fs, mode)
        for prec in precs:
            fd = factors_dev(fs, prec)
            for st in strategies:
                print("case", rec.name, "R", R, "mode", mode, prec, st, flush=True)
                out = t.mttkrp(fd, mode, strategy=st).cpu().numpy()
                err = rel_fro(out, ref)
                assert err <= TOL, (rec.name, mode, prec, st, err)
    t.close()


@pytest.mark.parametrize("rec,R,L", CASES, ids=[c[0].name + "_R%d" % c[1] for c in CASES])
def test_mttkrp_parity(rec, R, L):
    _run_case(rec, R, L)


@pytest.mark.parametrize("L", [1, 3, 1000, 100_000])
def test_mttkrp_partition_extremes(L):
    """One segment, a few, many, and more segments than nonzeros."""
    rec = small("zipf4_1Mx100kx10kx500_150M", 20_000)
    _run_case(rec, 16, L, precs=("f32",))


def test_repartition_through_exec():
    rec = small("zipf3_2Mx2Mx20k_50M", 100_000)
    coords, vals = synth.coo(rec)
    c, v = to_dev(coords, vals)
    t = alto.AltoTensor.build(c, v, rec.dims)
    fs = synth.factors(5, rec.dims, 16)
    fd = factors_dev(fs)
    ref = oracle.mttkrp(rec.dims, coords, vals, fs, 1)
    for L in (128, 4096, 7):
        for st in ("staged", "sorted"):
            out = t.mttkrp(fd, 1, strategy=st, num_segments=L).cpu().numpy()
            assert t.info()["num_segments"] == L
            assert rel_fro(out, ref) <= TOL
    t.close()


def test_kernel_timing_records_every_call():
    """alto_timing_enable / alto_timing_read: one event pair per MTTKRP while
    enabled, none otherwise; the kernels take no longer than the whole calls
    (torch events around them on the same stream)."""
    import torch
    rec = small("zipf4_1Mx100kx10kx500_150M", 200_000)
    coords, vals = synth.coo(rec)
    c, v = to_dev(coords, vals)
    t = alto.AltoTensor.build(c, v, rec.dims)
    fd = factors_dev(synth.factors(3, rec.dims, 32))
    for st in ("sorted", "atomic", "staged"):
        out = t.mttkrp(fd, 3, strategy=st)  # plans, orders and flags first
        alto.timing_read()
        alto.timing_enable(True)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(4):
            t.mttkrp(fd, 3, out=out, strategy=st)
        e1.record()
        alto.timing_enable(False)
        t.mttkrp(fd, 3, out=out, strategy=st)  # not recorded
        torch.cuda.synchronize()
        ms, n = alto.timing_read()
        print(st, "kernels", ms, "calls", e0.elapsed_time(e1), flush=True)
        assert n == 4
        assert 0.0 < ms <= e0.elapsed_time(e1) * 1.001
        assert alto.timing_read() == (0.0, 0)
    t.close()


def test_empty_tensor_gives_zero_output():
    torch = pytest.importorskip("torch")
    c = torch.zeros((3, 0), dtype=torch.int32, device="cuda")
    v = torch.zeros(0, dtype=torch.float32, device="cuda")
    t = alto.AltoTensor.build(c, v, (10, 20, 30))
    fd = factors_dev(synth.factors(1, (10, 20, 30), 16))
    out = torch.full((20, 16), 7.0, device="cuda")
    t.mttkrp(fd, 1, out=out)
    assert float(out.abs().max()) == 0.0
    t.close()


def test_invalid_calls():
    rec = synth.Recipe("inv", (10, 20, 30), 100, (), seed=1)
    coords, vals = synth.coo(rec)
    c, v = to_dev(coords, vals)
    t = alto.AltoTensor.build(c, v, rec.dims)
    fd = factors_dev(synth.factors(1, rec.dims, 16))
    with pytest.raises(ValueError):
        t.mttkrp(fd, 3)
    import ctypes
    import torch
    out = torch.zeros((30, 16), device="cuda")
    fp = alto._ptr_array(fd)
    L = alto.lib()
    s = alto._stream()
    assert L.alto_mttkrp(t._h, fp, 16, 0, 3, alto._ptr(out), None, s) == alto.E_INVAL   # mode >= N
    assert L.alto_mttkrp(t._h, fp, 0, 0, 2, alto._ptr(out), None, s) == alto.E_INVAL   # R = 0
    assert L.alto_mttkrp(t._h, fp, 257, 0, 2, alto._ptr(out), None, s) == alto.E_INVAL  # R > 256
    assert L.alto_mttkrp(t._h, fp, 16, 7, 2, alto._ptr(out), None, s) == alto.E_INVAL   # precision
    bad = alto._Exec(9, 0)
    assert L.alto_mttkrp(t._h, fp, 16, 0, 2, alto._ptr(out), ctypes.byref(bad), s) == alto.E_INVAL
    mis = ctypes.c_void_p(out.data_ptr() + 4)
    assert L.alto_mttkrp(t._h, fp, 16, 0, 2, mis, None, s) == alto.E_INVAL             # misaligned output
    t.close()


def _hot_rows(col, dim, k):
    cnt = np.bincount(col, minlength=dim)
    return np.argsort(cnt)[::-1][:k]


FULL_SIZE = [
    # (workload, rank, factor kind, strategies)
    ("zipf4_1Mx100kx10kx500_150M", 32, "grid", ("auto", "atomic", "staged", "sorted")),
    ("zipf5_10Mx5Mx2Mx100kx1k_200M", 32, "grid", ("auto", "atomic", "staged", "sorted")),
    ("zipf3_2Mx2Mx20k_50M", 64, "gauss", ("auto", "atomic", "staged", "sorted")),
]


@pytest.mark.slow
@pytest.mark.parametrize("name,R,kind,strategies", FULL_SIZE, ids=[f"{c[0]}_R{c[1]}_{c[2]}" for c in FULL_SIZE])
def test_full_size_sampled_rows(name, R, kind, strategies):
    """A benchmark tensor at full size with the default partition (the
    benchmark's launch configuration) for every strategy: sampled output rows
    (the hottest rows, which take up to tens of millions of contributions,
    plus random ones) against the oracle computed row by row.  The error of a
    row is measured against the row of sums of absolute terms (the FP32
    summation error bound), which for positive inputs is the row itself;
    with signed Gaussian factors that keeps cancelling rows meaningful."""
    torch = pytest.importorskip("torch")
    rec = synth.WORKLOADS[name]
    coords, vals = synth.coo(rec)
    c, v = to_dev(coords, vals)
    t = alto.AltoTensor.build(c, v, rec.dims)
    del c, v
    N = len(rec.dims)
    if kind == "grid":
        fs = synth.factors(rec.seed + 1, rec.dims, R)
        precs = ("f32", "bf16")
    else:
        rng = np.random.default_rng(rec.seed + 5)
        fs = [rng.standard_normal((d, R)).astype(np.float32) for d in rec.dims]
        precs = ("f32",)
    fabs = [np.abs(f) for f in fs]
    vabs = np.abs(vals)
    rng = np.random.default_rng(0)
    worst = {}
    # The strategies of Algorithm 2 visit the nonzeros in linearized order, so
    # the hottest rows (up to 16M contributions on the 5-mode tensor) reach
    # the output as millions of short runs; the library adds those with FP64
    # atomics (FP32 atomics measured up to 8e-4 here, a random walk of
    # roundings of the running sum).  The segment-local order sums every
    # (segment, row) run in registers before one FP32
    # atomic per run.  Measured worst rows: 7e-8 and 1.5e-6.
    tol = {"atomic": TOL, "staged": TOL, "sorted": TOL}
    for mode in range(N):
        rows = np.unique(np.concatenate([_hot_rows(coords[mode], rec.dims[mode], 8),
                                         rng.integers(0, rec.dims[mode], 24)])).astype(np.uint32)
        ref = oracle.mttkrp_rows(rec.dims, coords, vals, fs, mode, rows)
        bound = np.linalg.norm(oracle.mttkrp_rows(rec.dims, coords, vabs, fabs, mode, rows), axis=1)
        bound[bound == 0] = 1.0
        for prec in precs:
            fd = factors_dev(fs, prec)
            for st in strategies:
                print("full-size", name, "mode", mode, prec, st, flush=True)
                out = t.mttkrp(fd, mode, strategy=st)
                got = out[torch.from_numpy(rows.astype(np.int64)).cuda()].cpu().numpy().astype(np.float64)
                del out
                err = np.linalg.norm(got - ref, axis=1) / bound
                key = (prec, st)
                worst[key] = max(worst.get(key, 0.0), float(err.max()))
                resolved = t.select(mode, R, prec)[0] if st == "auto" else st
                assert err.max() <= tol[resolved], (mode, prec, st, resolved, int(rows[err.argmax()]),
                                                    float(err.max()))
    for (prec, st), e in sorted(worst.items()):
        print(f"worst sampled-row error {name} R={R} {kind} {prec} {st}: {e:.2e}", flush=True)
    t.close()


@pytest.mark.parametrize("name,nnz,R", [("zipf4_1Mx100kx10kx500_150M", 600_000, 32),
                                        ("uniform3_1000x800x600_100k", 0, 16)])
def test_bf16_factor_error_budget(name, nnz, R):
    """Factors that are not exact in bfloat16 (Gaussian FP32): the BF16 path
    (factors rounded to bfloat16, FP32 accumulation) stays within 1e-2
    relative Frobenius error of the FP64 oracle on the FP32 factors, and the
    FP32 path within 1e-5; the errors of every strategy are printed."""
    torch = pytest.importorskip("torch")
    rec = small(name, nnz) if nnz else synth.WORKLOADS[name]
    coords, vals = synth.coo(rec)
    c, v = to_dev(coords, vals)
    t = alto.AltoTensor.build(c, v, rec.dims)
    rng = np.random.default_rng(rec.seed + 99)
    fs = [rng.standard_normal((d, R)).astype(np.float32) for d in rec.dims]
    f32 = factors_dev(fs, "f32")
    bf16 = [f.to(torch.bfloat16) for f in f32]
    for mode in range(len(rec.dims)):
        ref = oracle.mttkrp(rec.dims, coords, vals, fs, mode)
        for st in ("atomic", "staged", "sorted"):
            e32 = rel_fro(t.mttkrp(f32, mode, strategy=st).cpu().numpy(), ref)
            e16 = rel_fro(t.mttkrp(bf16, mode, strategy=st).cpu().numpy(), ref)
            print(f"error {rec.name} mode {mode} {st}: fp32 {e32:.2e} bf16 {e16:.2e}", flush=True)
            assert e32 <= TOL and e16 <= 1e-2, (mode, st, e32, e16)
    t.close()
