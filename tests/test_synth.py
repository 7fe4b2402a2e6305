"""The seeded input generator: determinism, thread independence, distributions."""
import os
import subprocess
import sys

import numpy as np

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_splitmix64_published_sequence():
    """SplitMix64 with state 0: the first outputs of the published generator
    (state += 0x9E3779B97F4A7C15, then the two xor-shift-multiply rounds)."""
    def ref(state, n):
        out = []
        for _ in range(n):
            state = (state + 0x9E3779B97F4A7C15) % 2**64
            z = state
            z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) % 2**64
            z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) % 2**64
            out.append(z ^ (z >> 31))
        return out
    # stream k starts from mix(seed + (k+1)*gamma): compare against the
    # pure-Python reference started from that state
    seed, k = 12345, 3
    z = (seed + (k + 1) * 0x9E3779B97F4A7C15) % 2**64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) % 2**64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) % 2**64
    st = z ^ (z >> 31)
    assert synth.words(seed, k, 6).tolist() == ref(st, 6)
    # a well-known value: the first output of SplitMix64 seeded with 0
    assert ref(0, 1)[0] == 0xE220A8397B1DCDAF


def test_deterministic_and_thread_independent():
    code = ("import synth,hashlib;c,v=synth.coo(synth.scaled(synth.WORKLOADS['zipf4_1Mx100kx10kx500_150M'],200000));"
            "print(hashlib.sha1(c.tobytes()+v.tobytes()).hexdigest())")
    outs = []
    for t in ("1", "3"):
        env = dict(os.environ, OMP_NUM_THREADS=t, PYTHONPATH=ROOT)
        outs.append(subprocess.check_output([sys.executable, "-c", code], env=env, cwd=ROOT).strip())
    assert outs[0] == outs[1]


def test_zipf_head_probability():
    I, s, M = 1000, 1.2, 400000
    x = synth.mode_coords(7, 0, I, s, M)
    assert x.max() < I
    w = np.arange(1, I + 1, dtype=float) ** -s
    p1 = w[0] / w.sum()
    cnt = np.bincount(x, minlength=I)
    # the hottest index is rank 1 (mapped through the permutation)
    assert abs(cnt.max() / M - p1) < 5 * np.sqrt(p1 * (1 - p1) / M)
    # sorted frequencies follow the power law on the head
    top = np.sort(cnt)[::-1][:5] / M
    assert np.allclose(top, w[:5] / w.sum(), rtol=0.05)


def test_uniform_range_and_values():
    x = synth.mode_coords(9, 1, 777, 0.0, 100000)
    assert x.min() == 0 and x.max() == 776
    v = synth.values(9, "uniform", 100000)
    assert v.min() >= 0 and v.max() < 1 and abs(v.mean() - 0.5) < 0.01
    ln = synth.values(9, "lognormal", 200000).astype(np.float64)
    assert abs(np.log(ln).mean()) < 0.01 and abs(np.log(ln).std() - 1) < 0.01


def test_factor_entries_exact_in_bf16():
    f = synth.factor(3, 0, 1000, 32)
    k = f * 256
    assert np.array_equal(k, np.round(k)) and k.min() >= 1 and k.max() <= 255


def test_unique_topup_exact_count():
    rec = synth.Recipe("t", (20, 10, 5), 800, (0, 0, 0), seed=5, unique=True)
    c, v = synth.coo(rec)
    assert c.shape == (3, 800) and v.shape == (800,)
    lin = (c[0].astype(int) * 10 + c[1]) * 5 + c[2]
    assert len(np.unique(lin)) == 800


def test_planted_cp_is_the_sum_of_its_terms():
    """With no noise the planted tensor's values are the rank-R model
    sum_r prod_n A_n(i_n, r) at its (distinct) coordinates."""
    dims = (300, 200, 50, 9)
    c, v, P = synth.planted_cp(dims, 6, (7, 5, 4, 3), (1.2, 1.2, 0, 0), noise=0.0, seed=3)
    lin = ((c[0].astype(np.int64) * dims[1] + c[1]) * dims[2] + c[2]) * dims[3] + c[3]
    assert np.unique(lin).size == c.shape[1]
    model = np.ones((c.shape[1], 6))
    for n in range(4):
        model *= P[n][c[n]]
    assert np.allclose(v, model.sum(axis=1), rtol=1e-6)
    # every term contributes its whole box
    assert c.shape[1] <= 6 * 7 * 5 * 4 * 3
    start = synth.planted_start(P, 0.5)
    for f in start:
        assert f.dtype == np.float32 and np.all(f * 128 == np.rint(f * 128)) and f.max() < 2
