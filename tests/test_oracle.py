"""Pins for the FP64 CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: the
paper's printed worked example, closed forms, library routines (NumPy
GEMM/lstsq, torch's bfloat16 conversion), brute force on tiny inputs, or
invariants that any correct implementation satisfies.
"""
import itertools
import json
import math
import os

import numpy as np
import pytest

import oracle

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _load(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


# ------------------------------------------------------------ layout / encode
def test_layout_worked_example_subspaces():
    """Section 3.1: the prefixes [0-31], [0-15], [0-7] of the 6-bit line of a
    4x8x2 tensor are 4x4x2, 4x2x2 and 2x2x2 subspaces."""
    g = _load("alto_example_4x8x2.json")
    lay = oracle.layout(g["dims"])
    assert lay.B == g["index_bits"] and 2 ** lay.B == g["line_length"]
    for (lo, hi), shape in g["subspaces"]:
        keys = np.arange(lo, hi + 1, dtype=np.uint64)
        c = oracle.decode(lay, keys)
        ext = [int(c[n].max()) - int(c[n].min()) + 1 for n in range(3)]
        assert ext == shape
        assert [int(c[n].min()) for n in range(3)] == [0, 0, 0]
        # the prefix is exactly the product set (every point once)
        assert len({tuple(x) for x in c.T}) == math.prod(shape) == hi - lo + 1
    # the masks this forces (MSB..LSB = j2 j1 i1 j0 i0 k0)
    assert lay.masks == [0b001010, 0b110100, 0b000001]


def test_layout_alternative_rejected():
    """A longest-mode-lowest layout would give 2x4x2 for [0-15], not 4x2x2:
    the pin above is able to fail."""
    # layout with k0 j0 i0 order reversed inside a level: masks by hand
    alt = {0: 0b000100 | 0b010000, 1: 0b000001 | 0b001000 | 0b100000, 2: 0b000010}
    pts = []
    for p in range(16):
        c = []
        for n in range(3):
            m, k, v = alt[n], 0, 0
            for b in range(6):
                if (m >> b) & 1:
                    v |= ((p >> b) & 1) << k
                    k += 1
            c.append(v)
        pts.append(c)
    ext = [max(q[n] for q in pts) + 1 for n in range(3)]
    assert ext != [4, 2, 2]


def test_partition_worked_example():
    """Section 3.2: two equal-nonzero segments [2-20] and [25-51] with the
    printed mode intervals."""
    g = _load("alto_example_4x8x2.json")
    lay = oracle.layout(g["dims"])
    keys = np.array(g["positions"], np.uint64)
    seg = oracle.partition(len(keys), 2)
    assert list(seg) == [0, 3, 6]
    for l, (a, b) in enumerate(g["segments"]):
        assert int(keys[seg[l]]) == a and int(keys[seg[l + 1] - 1]) == b
    ivl = oracle.intervals(lay, seg, keys)
    assert ivl.tolist() == g["intervals"]
    # the printed end points decode to fixed coordinates under the layout
    c = oracle.decode(lay, np.array([2, 20, 25, 51], np.uint64)).T.tolist()
    assert c == [[1, 0, 0], [0, 3, 0], [2, 2, 1], [1, 6, 1]]


def test_partition_example_all_consistent_middles():
    """Every choice of middle nonzeros that reproduces the printed intervals
    exists and the interval rule is min/max over the segment's nonzeros (the
    bounding box of the key range [25,51] would give i in [0,3], not [1,3])."""
    g = _load("alto_example_4x8x2.json")
    lay = oracle.layout(g["dims"])
    ok = 0
    for m0 in range(3, 20):
        for m1 in range(26, 51):
            keys = np.array([2, m0, 20, 25, m1, 51], np.uint64)
            ivl = oracle.intervals(lay, np.array([0, 3, 6]), keys)
            if ivl.tolist() == g["intervals"]:
                ok += 1
    assert ok > 0
    box = oracle.decode(lay, np.arange(25, 52, dtype=np.uint64))
    assert int(box[0].min()) == 0  # the key-range box would contradict [1-3]


def test_eq2_eq3_examples():
    g = _load("alto_example_4x8x2.json")
    assert oracle.compression_ratio(g["dims"], 8) == g["compression_ratio_wb8"]
    lay = oracle.layout(g["dims"])
    assert math.ceil(lay.B / 8) == g["alto_bytes_per_nnz"]
    assert sum(math.ceil(b / 8) for b in lay.nbits) == g["coo_bytes_per_nnz"]
    # Eq. 3: Z-Morton needs N * max b_n bits: 9 vs 6 bits -> line 8x longer
    assert 2 ** (oracle.sfc_bits(g["dims"], 1) - oracle.storage_bits(g["dims"], 1)) == g["sfc_line_ratio"]


def test_table1_index_widths_and_reuse_classes():
    g = _load("table1_tensors.json")
    widths = {}
    for name, dims, nnz, cls in g["tensors"]:
        lay = oracle.layout([int(round(d)) for d in dims])
        widths[name] = 8 * math.ceil(lay.B / 8)
        reuse = min(nnz / d for d in dims)
        got = "High" if reuse > 8 else ("Medium" if reuse >= 5 else "Limited")
        if name != "deli":
            assert got == cls, (name, reuse)
    assert (min(widths.values()), max(widths.values())) == tuple(g["index_bits_byte_rounded_range"])
    assert widths["amazon"] == g["amazon_index_bits_byte_rounded"]
    # Section 4.4: darpa mode 3 (limited reuse) uses atomics, mode 1 staging
    _, dims, nnz, _ = [t for t in g["tensors"] if t[0] == "darpa"][0]
    assert not oracle.heuristic_staging(int(nnz), int(dims[2]))
    assert oracle.heuristic_staging(int(nnz), int(dims[0]))


def test_heuristic_threshold_is_strict():
    """Section 3.3: staging only when reuse is MORE than four memory operations."""
    assert not oracle.heuristic_staging(400, 100)
    assert oracle.heuristic_staging(401, 100)


@pytest.mark.parametrize("dims", [(3, 5, 2), (7, 1, 4, 3), (2, 2, 2, 2, 2), (1, 1), (9, 17), (16, 4, 8),
                                  (5, 6, 7, 3), (33,)])
def test_encode_decode_exhaustive(dims):
    """Every coordinate tuple of a tiny shape round-trips and gets a distinct
    key below 2^B; with power-of-two dims the keys are exactly 0..2^B-1."""
    lay = oracle.layout(dims)
    assert lay.B == sum(lay.nbits) == sum(math.ceil(math.log2(d)) if d > 1 else 0 for d in dims)
    for n in range(len(dims)):
        assert bin(lay.masks[n]).count("1") == lay.nbits[n]
        for m in range(n):
            assert lay.masks[n] & lay.masks[m] == 0
    pts = np.array(list(itertools.product(*[range(d) for d in dims])), np.uint32).T
    lo, hi = oracle.encode(lay, pts)
    assert np.all(hi == 0)
    assert len(np.unique(lo)) == pts.shape[1]
    assert int(lo.max()) < 2 ** lay.B
    assert np.array_equal(oracle.decode(lay, (lo, hi)), pts)
    if all(d & (d - 1) == 0 for d in dims):
        assert sorted(lo.tolist()) == list(range(2 ** lay.B))


def test_longest_mode_owns_top_bits():
    """The most significant bits belong to the longest mode and, inside a
    level, the shorter mode takes the lower bit (Section 3.1)."""
    lay = oracle.layout((500, 1_000_000, 10_000, 100_000))
    top = lay.B - 1
    assert (lay.masks[1] >> top) & 1
    # level 0: modes ordered 0 (500) < 2 (10k) < 3 (100k) < 1 (1M)
    assert [(lay.masks[n] & 0xF).bit_length() - 1 for n in (0, 2, 3, 1)] == [0, 1, 2, 3]


@pytest.mark.parametrize("dims,B", [((1000, 800, 600), 30), ((2_000_000, 2_000_000, 20_000), 57),
                                    ((1_000_000, 100_000, 10_000, 500), 60),
                                    ((10_000_000, 5_000_000, 2_000_000, 100_000, 1_000), 95),
                                    ((4_800_000, 1_800_000, 1_800_000), 65)])
def test_wide_layouts_roundtrip(dims, B):
    lay = oracle.layout(dims)
    assert lay.B == B
    rng = np.random.default_rng(1)
    pts = np.stack([rng.integers(0, d, 5000) for d in dims]).astype(np.uint32)
    edge = np.array([[d - 1 for d in dims], [0] * len(dims)], np.uint32).T
    pts = np.concatenate([pts, edge], axis=1)
    lo, hi = oracle.encode(lay, pts)
    assert np.array_equal(oracle.decode(lay, (lo, hi)), pts)
    if B > 64:
        assert hi.max() > 0
    # Python big-int cross-check of the deposit definition for a few points
    for x in range(0, pts.shape[1], 997):
        key = 0
        for n in range(len(dims)):
            k = 0
            for p in range(128):
                if (lay.masks[n] >> p) & 1:
                    key |= ((int(pts[n, x]) >> k) & 1) << p
                    k += 1
        assert key == int(lo[x]) | (int(hi[x]) << 64)


def test_layout_rejects_too_wide():
    with pytest.raises(ValueError):
        oracle.layout([2 ** 32] * 5)  # 160 bits


# ------------------------------------------------------------ sort / partition
def test_sort_perm_matches_numpy_stable():
    rng = np.random.default_rng(3)
    lo = rng.integers(0, 50, 4000).astype(np.uint64)
    hi = rng.integers(0, 3, 4000).astype(np.uint64)
    perm = oracle.sort_perm((lo, hi))
    ref = np.lexsort((np.arange(4000), lo, hi))
    assert np.array_equal(perm, ref)


def test_coalesce_sums_runs():
    lo = np.array([1, 1, 2, 5, 5, 5], np.uint64)
    (ulo, _), v = oracle.coalesce((lo, np.zeros(6, np.uint64)), [1.0, 2.0, 3.0, 4.0, 5.0, 6.0])
    assert ulo.tolist() == [1, 2, 5] and v.tolist() == [3.0, 3.0, 15.0]


@pytest.mark.parametrize("M,L", [(10, 3), (7, 7), (5, 9), (1000, 64), (1, 1), (123457, 4096)])
def test_partition_invariants(M, L):
    seg = oracle.partition(M, L)
    Le = min(L, M)
    assert len(seg) == Le + 1 and seg[0] == 0 and seg[-1] == M
    sizes = np.diff(seg)
    assert sizes.min() >= 1 and sizes.max() - sizes.min() <= 1
    assert sizes.sum() == M


def test_intervals_and_coverage_brute_force():
    rng = np.random.default_rng(5)
    dims = (37, 12, 5, 64)
    pts = np.stack([rng.integers(0, d, 3000) for d in dims]).astype(np.uint32)
    lay = oracle.layout(dims)
    lo, hi = oracle.encode(lay, pts)
    perm = oracle.sort_perm((lo, hi))
    lo = lo[perm]
    seg = oracle.partition(len(lo), 17)
    ivl = oracle.intervals(lay, seg, (lo, hi[perm]))
    c = oracle.decode(lay, (lo, hi[perm]))
    for l in range(len(seg) - 1):
        for n in range(4):
            part = c[n, seg[l]:seg[l + 1]]
            assert ivl[l, n, 0] == part.min() and ivl[l, n, 1] == part.max()
    for n in range(4):
        cov = oracle.coverage(ivl, n, dims[n])
        brute = np.zeros(dims[n], np.int64)
        for l in range(len(seg) - 1):
            brute[ivl[l, n, 0]:ivl[l, n, 1] + 1] += 1
        assert np.array_equal(cov, brute)
        assert cov.sum() == sum(int(ivl[l, n, 1]) - int(ivl[l, n, 0]) + 1 for l in range(len(seg) - 1))


# ------------------------------------------------------------ MTTKRP
def _dense(dims, coords, vals):
    X = np.zeros(dims)
    np.add.at(X, tuple(coords.astype(np.int64)), vals)
    return X


def _mttkrp_bruteforce(dims, coords, vals, factors, mode):
    """Materialize, unfold (row-major: remaining modes in order, last fastest),
    explicit Khatri-Rao product of the remaining factors, GEMM."""
    X = _dense(dims, coords, vals)
    Xn = np.moveaxis(X, mode, 0).reshape(dims[mode], -1)
    R = factors[0].shape[1]
    KR = np.ones((1, R))
    for m in range(len(dims)):
        if m != mode:
            KR = (KR[:, None, :] * factors[m][None, :, :]).reshape(-1, R)
    return Xn @ KR


@pytest.mark.parametrize("dims", [(6, 5), (4, 7, 3), (3, 1, 5, 2), (2, 3, 2, 3, 2), (1, 9, 4)])
def test_mttkrp_matches_dense_khatri_rao(dims):
    rng = np.random.default_rng(sum(dims))
    M = 40
    coords = np.stack([rng.integers(0, d, M) for d in dims]).astype(np.uint32)
    vals = rng.standard_normal(M)
    R = 5
    fs = [rng.standard_normal((d, R)) for d in dims]
    for mode in range(len(dims)):
        got = oracle.mttkrp(dims, coords, vals, fs, mode)
        ref = _mttkrp_bruteforce(dims, coords, vals, fs, mode)
        assert np.abs(got - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max())


def test_mttkrp_order2_is_sparse_matrix_product():
    rng = np.random.default_rng(11)
    I, J, M, R = 30, 20, 90, 4
    c = np.stack([rng.integers(0, I, M), rng.integers(0, J, M)]).astype(np.uint32)
    v = rng.random(M)
    B = rng.random((J, R))
    A = rng.random((I, R))
    X = np.zeros((I, J))
    np.add.at(X, (c[0].astype(int), c[1].astype(int)), v)
    assert np.allclose(oracle.mttkrp((I, J), c, v, [A, B], 0), X @ B, rtol=1e-13, atol=0)
    assert np.allclose(oracle.mttkrp((I, J), c, v, [A, B], 1), X.T @ A, rtol=1e-13, atol=0)


def test_mttkrp_rank1_ones_is_slice_sum():
    rng = np.random.default_rng(12)
    dims = (50, 40, 30)
    M = 2000
    c = np.stack([rng.integers(0, d, M) for d in dims]).astype(np.uint32)
    v = rng.random(M)
    fs = [np.ones((d, 1)) for d in dims]
    for n in range(3):
        got = oracle.mttkrp(dims, c, v, fs, n)[:, 0]
        assert np.allclose(got, np.bincount(c[n], weights=v, minlength=dims[n]), rtol=1e-13, atol=0)


def test_mttkrp_linearity_and_order_invariance():
    rng = np.random.default_rng(13)
    dims = (20, 30, 10, 5)
    M = 500
    c = np.stack([rng.integers(0, d, M) for d in dims]).astype(np.uint32)
    v1, v2 = rng.random(M), rng.random(M)
    fs = [rng.random((d, 3)) for d in dims]
    a = oracle.mttkrp(dims, c, v1, fs, 2)
    b = oracle.mttkrp(dims, c, v2, fs, 2)
    assert np.allclose(oracle.mttkrp(dims, c, 2 * v1 + 3 * v2, fs, 2), 2 * a + 3 * b, rtol=1e-12)
    p = rng.permutation(M)
    assert np.allclose(oracle.mttkrp(dims, c[:, p], v1[p], fs, 2), a, rtol=1e-12)


def test_mttkrp_par_matches_serial():
    """The all-core variant differs from the serial loop only in the order of
    the sums (thread-private outputs added at the end)."""
    rng = np.random.default_rng(19)
    dims = (300, 200, 100, 7)
    M = 50_000
    c = np.stack([rng.integers(0, d, M) for d in dims]).astype(np.uint32)
    v = rng.standard_normal(M)
    fs = [rng.standard_normal((d, 5)) for d in dims]
    for mode in range(4):
        ref = oracle.mttkrp(dims, c, v, fs, mode)
        got, used = oracle.mttkrp_par(dims, c, v, fs, mode)
        assert used >= 1
        assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


def test_mttkrp_rows_subset():
    rng = np.random.default_rng(14)
    dims = (100, 30, 10)
    M = 3000
    c = np.stack([rng.integers(0, d, M) for d in dims]).astype(np.uint32)
    v = rng.random(M)
    fs = [rng.random((d, 8)) for d in dims]
    full = oracle.mttkrp(dims, c, v, fs, 0)
    sel = np.array([99, 0, 17, 53], np.uint32)
    assert np.array_equal(oracle.mttkrp_rows(dims, c, v, fs, 0, sel), full[sel])


def test_norm2_with_repeats():
    c = np.array([[0, 0, 1, 0], [1, 1, 2, 1]], np.uint32)
    v = np.array([1.0, 2.0, 4.0, 0.5])
    assert oracle.norm2(c, v) == pytest.approx(3.5 ** 2 + 4.0 ** 2, rel=1e-15)


# ------------------------------------------------------------ CP-ALS
def _rank_r_dense_coo(dims, R, rng):
    fs = [rng.standard_normal((d, R)) for d in dims]
    X = np.einsum("ir,jr,kr->ijk", *fs)
    idx = np.nonzero(np.ones(dims))
    return np.stack(idx).astype(np.uint32), X[idx]


def test_cp_als_recovers_exact_rank():
    rng = np.random.default_rng(21)
    dims = (8, 7, 6)
    c, v = _rank_r_dense_coo(dims, 3, rng)
    init = [rng.random((d, 3)) for d in dims]
    _, lam, fit = oracle.cp_als(dims, c, v, init, 100)
    assert fit[-1] >= 1 - 1e-6


def test_cp_als_disjoint_blocks_exact_rank():
    """Sum of R rank-1 blocks on disjoint index ranges: sparse, exact rank R."""
    rng = np.random.default_rng(22)
    R = 3
    blocks = [(3, 4, 2), (2, 2, 3), (4, 3, 3)]
    dims = tuple(sum(b[n] for b in blocks) for n in range(3))
    cs, vs, off = [], [], [0, 0, 0]
    for b in blocks:
        u = [rng.random(b[n]) + 0.5 for n in range(3)]
        for i, j, k in itertools.product(*[range(x) for x in b]):
            cs.append((off[0] + i, off[1] + j, off[2] + k))
            vs.append(u[0][i] * u[1][j] * u[2][k])
        off = [off[n] + b[n] for n in range(3)]
    c = np.array(cs, np.uint32).T
    v = np.array(vs)
    init = [rng.random((d, R)) + 0.05 for d in dims]
    _, _, fit = oracle.cp_als(dims, c, v, init, 300)
    assert fit[-1] >= 1 - 1e-6


def test_cp_als_fit_monotone_and_normal_equations():
    rng = np.random.default_rng(23)
    dims = (9, 8, 7, 6)
    M = 300
    c = np.stack([rng.integers(0, d, M) for d in dims]).astype(np.uint32)
    v = rng.random(M)
    R = 4
    init = [rng.random((d, R)) for d in dims]
    fs, lam, fit = oracle.cp_als(dims, c, v, init, 12)
    assert np.all(np.diff(fit) >= -1e-10)
    # the last mode solved the normal equations with the final other factors
    n = len(dims) - 1
    Mn = oracle.mttkrp(dims, c, v, fs, n)
    V = np.ones((R, R))
    for m in range(n):
        V *= fs[m].T @ fs[m]
    lhs = (fs[n] * lam) @ V
    assert np.abs(lhs - Mn).max() <= 1e-9 * np.abs(Mn).max()
    # ... which is the least-squares solution of the unfolded problem
    X = _dense(dims, c, v)
    Xn = np.moveaxis(X, n, 0).reshape(dims[n], -1)
    KR = np.ones((1, R))
    for m in range(n):
        KR = (KR[:, None, :] * fs[m][None, :, :]).reshape(-1, R)
    sol = np.linalg.lstsq(KR, Xn.T, rcond=None)[0].T
    assert np.abs(sol - fs[n] * lam).max() <= 1e-8 * np.abs(sol).max()
    # and the reported fit is 1 - ||X - Xhat|| / ||X||
    Xhat = np.einsum("r,ir,jr,kr,lr->ijkl", lam, *fs)
    ref = 1 - np.linalg.norm(X - Xhat) / np.linalg.norm(X)
    assert fit[-1] == pytest.approx(ref, abs=1e-9)


def test_cp_als_unit_columns():
    rng = np.random.default_rng(24)
    dims = (10, 9, 8)
    c = np.stack([rng.integers(0, d, 200) for d in dims]).astype(np.uint32)
    fs, lam, _ = oracle.cp_als(dims, c, rng.random(200), [rng.random((d, 3)) for d in dims], 3)
    for f in fs:
        assert np.allclose(np.linalg.norm(f, axis=0), 1.0, rtol=1e-12)


def _als_sweep_with_ridge(dims, X, init, eps):
    """One ALS sweep in NumPy from the dense tensor X, adding the ridge
    eps * trace(V) / R to the diagonal of V whenever V has no Cholesky
    factor.  Returns (factors, lambda, number of ridged updates)."""
    fs = [np.array(f, np.float64) for f in init]
    R = fs[0].shape[1]
    lam = np.ones(R)
    ridged = 0
    for n in range(len(dims)):
        Xn = np.moveaxis(X, n, 0).reshape(dims[n], -1)
        KR = np.ones((1, R))
        for m in range(len(dims)):
            if m != n:
                KR = (KR[:, None, :] * fs[m][None, :, :]).reshape(-1, R)
        Mn = Xn @ KR
        V = np.ones((R, R))
        for m in range(len(dims)):
            if m != n:
                V *= fs[m].T @ fs[m]
        try:
            np.linalg.cholesky(V)
        except np.linalg.LinAlgError:
            V = V + eps * np.trace(V) / R * np.eye(R)
            ridged += 1
        A = np.linalg.solve(V, Mn.T).T
        lam = np.linalg.norm(A, axis=0)
        A[:, lam > 0] /= lam[lam > 0]
        fs[n] = A
    return fs, lam, ridged


def test_cp_als_ridge_retry():
    """A singular normal-equation matrix takes the ridge reading (one retry
    with 1e-10 * trace(V) / R on the diagonal).  Column 3 is zero in modes 1
    and 2, so every V of the sweep has a zero row; columns 1 and 2 are nearly
    parallel in every mode, so V is ill-conditioned on the rest and the size
    of the ridge shows in the solution (a scale off by 2x, or the trace not
    divided by R, moves it far beyond the tolerance)."""
    rng = np.random.default_rng(31)
    dims = (12, 10, 8)
    R = 4
    X = rng.random(dims)
    c = np.stack(np.nonzero(np.ones(dims))).astype(np.uint32)
    v = X[tuple(c)]
    init = [rng.random((d, R)) for d in dims]
    for f in init:
        f[:, 2] = f[:, 1] + 1e-4 * rng.standard_normal(f.shape[0])
    init[1][:, 3] = 0.0
    init[2][:, 3] = 0.0
    fs, lam, _ = oracle.cp_als(dims, c, v, init, 1)
    ref, rlam, ridged = _als_sweep_with_ridge(dims, X, init, 1e-10)
    assert ridged == 3  # every update needed the ridge
    err = max(np.abs(a - b).max() for a, b in zip(fs, ref))
    assert err <= 1e-9, err
    assert np.allclose(lam, rlam, rtol=1e-7)
    assert np.all(fs[1][:, 3] == 0.0) and np.all(fs[2][:, 3] == 0.0)
    # the test can tell a wrong ridge from the right one
    for wrong in (2e-10, 5e-11, 4e-10):
        alt, _, _ = _als_sweep_with_ridge(dims, X, init, wrong)
        assert max(np.abs(a - b).max() for a, b in zip(fs, alt)) > 1e3 * 1e-9, wrong
    # no retry beyond the one: zero factors keep V zero even with the ridge
    with pytest.raises(np.linalg.LinAlgError):
        oracle.cp_als(dims, c, v, [np.zeros((d, R)) for d in dims], 1)


@pytest.mark.parametrize("dims,perm", [((4, 8, 2), (1, 0, 2)), ((5, 3, 4, 2), (3, 1, 0, 2)),
                                       ((6, 7), (1, 0)), ((3, 4, 5), (0, 1, 2))])
def test_transpose_matches_dense_transpose(dims, perm):
    """Transposition: the nonzeros of np.transpose(X, perm) in row-major
    (C) order are exactly the lexicographic order of the permuted coordinates;
    repeated COO entries are summed."""
    rng = np.random.default_rng(41)
    M = 40
    c = np.stack([rng.integers(0, d, M) for d in dims]).astype(np.uint32)
    v = rng.random(M) + 0.5
    X = _dense(dims, c, v)
    Y = np.transpose(X, perm)
    ref_idx = np.nonzero(Y)
    got_c, got_v = oracle.transpose(c, v, perm)
    assert all(np.array_equal(got_c[j], ref_idx[j]) for j in range(len(dims)))
    assert np.allclose(got_v, Y[ref_idx], rtol=1e-15)


# ------------------------------------------------------------ BF16# ------------------------------------------------------------ BF16
def test_bf16_matches_torch_rne():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(31)
    x = np.concatenate([rng.standard_normal(20000) * 10.0 ** rng.integers(-30, 30, 20000),
                        [0.0, -0.0, 1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, 3.0e38, 1e-40, np.inf, -np.inf]])
    bits, vals = oracle.bf16_round(x)
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16)
    assert np.array_equal(bits, ref.view(torch.int16).numpy().view(np.uint16))
    assert np.array_equal(vals, ref.to(torch.float64).numpy())
    # ties go to even: 1 + 2^-8 is halfway between 1 and 1 + 2^-7
    assert vals[-6] == 1.0 and vals[-5] == 1.0 + 2 ** -7


def test_bf16_nan_quiet():
    bits, vals = oracle.bf16_round(np.array([np.nan]))
    assert np.isnan(vals[0]) and (bits[0] & 0x7F80) == 0x7F80 and (bits[0] & 0x7F)


# ------------------------------------------------------------ MLP
def test_mlp_gradients_central_differences():
    rng = np.random.default_rng(41)
    F, H, K, B = 7, 6, 5, 9
    p = [rng.standard_normal((H, F)) * 0.5, rng.standard_normal(H) * 0.1,
         rng.standard_normal((H, H)) * 0.5, rng.standard_normal(H) * 0.1,
         rng.standard_normal((K, H)) * 0.5, rng.standard_normal(K) * 0.1]
    x = rng.standard_normal((B, F))
    t = rng.standard_normal((B, K))
    mask = (rng.random((B, K)) > 0.3).astype(float)
    net = oracle.MLP(*p)
    grads, loss = net.backward(x, t, mask)
    _, loss_f = net.forward(x, t, mask)
    assert loss == pytest.approx(loss_f, rel=1e-14)
    h = 1e-6
    for a, g in zip(net.p, grads):
        flat, gf = a.reshape(-1), g.reshape(-1)
        for q in range(flat.size):
            old = flat[q]
            flat[q] = old + h
            lp = net.forward(x, t, mask)[1]
            flat[q] = old - h
            lm = net.forward(x, t, mask)[1]
            flat[q] = old
            fd = (lp - lm) / (2 * h)
            assert abs(fd - gf[q]) <= 1e-6 * max(1.0, abs(fd)), (q, fd, gf[q])


def test_mlp_forward_matches_numpy():
    rng = np.random.default_rng(42)
    F, H, K, B = 4, 8, 3, 5
    p = [rng.standard_normal(s) for s in [(H, F), (H,), (H, H), (H,), (K, H), (K,)]]
    x = rng.standard_normal((B, F))
    y, _ = oracle.MLP(*p).forward(x)
    h1 = np.maximum(x @ p[0].T + p[1], 0)
    h2 = np.maximum(h1 @ p[2].T + p[3], 0)
    assert np.allclose(y, h2 @ p[4].T + p[5], rtol=1e-13)
