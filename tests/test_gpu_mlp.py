"""Selector network kernels (forward, backward, Adam) vs the FP64 oracle."""
import numpy as np
import pytest

import oracle
import paper_2102_10245_amd as alto
from gpu_common import gpu_ok

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_ok(), reason="needs a GPU")]


def _params(rng, F, H, K):
    shapes = [(H, F), (H,), (H, H), (H,), (K, H), (K,)]
    return [rng.standard_normal(s) * (0.5 if len(s) == 2 else 0.1) for s in shapes]


@pytest.mark.parametrize("B,F,H,K", [(37, 12, 64, 14), (5, 3, 7, 2), (300, 12, 64, 14), (64, 12, 200, 40)])
def test_forward_backward_match_oracle(B, F, H, K):
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(B + H)
    p = _params(rng, F, H, K)
    x = rng.standard_normal((B, F))
    t = rng.standard_normal((B, K))
    mask = (rng.random((B, K)) > 0.2).astype(np.float64)
    net = oracle.MLP(*p)
    y_ref, loss_ref = net.forward(x, t, mask)
    g_ref, _ = net.backward(x, t, mask)
    flat = np.concatenate([a.reshape(-1) for a in p]).astype(np.float32)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()
    P = dev(flat)
    y, loss = alto.mlp_forward(P, dev(x), F, H, K, dev(t), dev(mask))
    assert np.allclose(y.cpu().numpy(), y_ref, rtol=1e-4, atol=1e-4)
    assert float(loss.cpu()) == pytest.approx(loss_ref, rel=1e-4)
    g, loss2 = alto.mlp_backward(P, dev(x), dev(t), dev(mask), F, H, K)
    gr = np.concatenate([a.reshape(-1) for a in g_ref])
    gg = g.cpu().numpy()
    assert np.linalg.norm(gg - gr) <= 1e-4 * max(1e-12, np.linalg.norm(gr))
    assert float(loss2.cpu()) == pytest.approx(loss_ref, rel=1e-4)


def test_adam_step_matches_formula():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(3)
    n = 1000
    w = rng.standard_normal(n).astype(np.float32)
    g = rng.standard_normal(n).astype(np.float32)
    m = rng.standard_normal(n).astype(np.float32) * 0.1
    v = rng.random(n).astype(np.float32) * 0.1
    W, G, Mm, V = (torch.from_numpy(a.copy()).cuda() for a in (w, g, m, v))
    alto.mlp_adam(W, G, Mm, V, lr=1e-2, step=3)
    b1, b2, eps, lr = 0.9, 0.999, 1e-8, 1e-2
    m2 = b1 * m.astype(np.float64) + (1 - b1) * g
    v2 = b2 * v.astype(np.float64) + (1 - b2) * g.astype(np.float64) ** 2
    w2 = w - lr * (m2 / (1 - b1 ** 3)) / (np.sqrt(v2 / (1 - b2 ** 3)) + eps)
    assert np.allclose(W.cpu().numpy(), w2, rtol=1e-5, atol=1e-6)
    assert np.allclose(Mm.cpu().numpy(), m2, rtol=1e-6, atol=1e-7)
