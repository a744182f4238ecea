"""Pins of the CPU MLP reference: gradients against float64 central
differences, GELU identities, the cross-entropy against scipy's logsumexp,
Adam's closed-form first step, and bfloat16 rounding against torch."""
import numpy as np
import pytest
import scipy.special

import labs_inputs as li
from oracle import mlp


def _small(seed=0, n=6, d_in=10, h=7, d_out=5):
    P = {k: v.astype(np.float64) for k, v in li.mlp_init(seed, d_in, h, d_out).items()}
    g = li.rng(seed + 1)
    P["b1"] = g.normal(size=h) * 0.1
    P["b2"] = g.normal(size=h) * 0.1
    P["b3"] = g.normal(size=d_out) * 0.1
    X = g.normal(size=(n, d_in))
    mask = g.random((n, d_out)) < 0.7
    mask[:, 0] = True
    labels = np.array([np.flatnonzero(mask[r])[g.integers(0, mask[r].sum())] for r in range(n)])
    return P, X, mask, labels


def test_gradients_match_central_differences():
    P, X, mask, labels = _small()
    loss, G = mlp.loss_and_grads(P, X, mask, labels, exact=True)
    eps = 1e-6
    for key, w in P.items():
        num = np.zeros_like(w)
        for idx in np.ndindex(w.shape):
            old = w[idx]
            w[idx] = old + eps
            lp, _ = mlp.loss_and_grads(P, X, mask, labels, exact=True)
            w[idx] = old - eps
            lm, _ = mlp.loss_and_grads(P, X, mask, labels, exact=True)
            w[idx] = old
            num[idx] = (lp - lm) / (2 * eps)
        err = np.abs(num - G[key]).max() / max(1e-12, np.abs(num).max())
        assert err < 1e-6, key


def test_gelu_identities():
    x = np.linspace(-6, 6, 101)
    assert mlp.gelu(np.array(0.0)) == 0.0
    np.testing.assert_allclose(mlp.gelu(x) - mlp.gelu(-x), x, atol=1e-12)
    h = 1e-6
    np.testing.assert_allclose(mlp.gelu_grad(x), (mlp.gelu(x + h) - mlp.gelu(x - h)) / (2 * h),
                               rtol=1e-6, atol=1e-9)
    # the tanh form is within 2e-3 of the exact x * Phi(x)
    exact = x * 0.5 * (1 + scipy.special.erf(x / np.sqrt(2)))
    assert np.abs(mlp.gelu(x) - exact).max() < 2e-3


def test_masked_ce_matches_logsumexp():
    g = li.rng(4)
    z = g.normal(size=(5, 9)) * 3
    mask = g.random((5, 9)) < 0.6
    mask[:, 2] = True
    labels = np.array([2] * 5)
    loss, dz = mlp.masked_ce(z, mask, labels)
    ref = np.mean([scipy.special.logsumexp(z[r][mask[r]]) - z[r, 2] for r in range(5)])
    assert abs(loss - ref) < 1e-12
    assert np.all(dz[~mask] == 0)
    np.testing.assert_allclose(dz.sum(axis=1), 0, atol=1e-12)


def test_adam_first_step_closed_form():
    P = {"w": np.array([1.0, -2.0, 0.5], np.float32)}
    G = {"w": np.array([0.3, -1e-3, 0.0], np.float32)}
    M = {"w": np.zeros(3, np.float32)}
    V = {"w": np.zeros(3, np.float32)}
    mlp.adam(P, G, M, V, 1, lr=1e-3)
    g = G["w"].astype(np.float64)
    want = np.array([1.0, -2.0, 0.5]) - 1e-3 * g / (np.abs(g) + 1e-8)
    np.testing.assert_allclose(P["w"], want, rtol=1e-6)


def test_bf16_rounding_matches_torch():
    torch = pytest.importorskip("torch")
    vals = np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, -3.14159, 1e-30, 65504.0, 0.1, -0.0],
                    np.float32)
    g = li.rng(2)
    vals = np.concatenate([vals, g.normal(size=1000).astype(np.float32) * 10])
    ours = mlp.bf16_round(vals)
    ref = torch.from_numpy(vals).to(torch.bfloat16).float().numpy()
    assert np.array_equal(ours.view(np.uint32), ref.view(np.uint32))
    assert mlp.bf16_round(np.float32(1 + 2 ** -8)) == 1.0          # tie to even
    assert mlp.bf16_round(np.float32(1 + 3 * 2 ** -8)) == 1 + 2 ** -6


def test_rounded_forward_close_to_exact():
    P, X, mask, labels = _small(seed=3, n=20, d_in=40, h=16, d_out=12)
    z1, _ = mlp.forward(P, X, exact=True)
    z2, _ = mlp.forward(P, X, exact=False)
    assert np.abs(z1 - z2).max() < 0.05 * max(1.0, np.abs(z1).max())


def test_features_layout(orc):
    L = 13
    s = li.random_skew(3, 2, L)
    C = np.stack([orc.energy(x, with_c=True)[1][1::2] for x in s])
    X = mlp.features(s, C)
    assert X.shape == (2, L + 6)
    assert np.array_equal(X[:, :L], s)
    for m in range(1, 7):
        np.testing.assert_allclose(X[:, L + m - 1], C[:, m - 1] / (L - 2 * m))
