"""CPU reference of the learned flip proposal (test infrastructure only).

A small MLP scores the free positions of a skew-symmetric walker state:
  input  x = (s_1..s_L as +1/-1, C_{2m}/(L-2m) for m = 1..k), L + k values;
  h1 = GELU(W1 x + b1), h2 = GELU(W2 h1 + b2), z = W3 h2 + b3,
  one logit per position 1..k+1 (prefix and tabu positions are masked out).
GELU is the tanh form 0.5 x (1 + tanh(sqrt(2/pi) (x + 0.044715 x^3)))
(Hendrycks and Gimpel, 2016).  Training minimises the softmax cross-entropy
over the admissible positions against the plain walker's chosen flip, with
Adam (Kingma and Ba, 2015).  The paper has no learned component: these are
readings of the configuration, listed with the others.

Precision: weights live in FP32 (masters) and enter every product rounded to
bfloat16 (round to nearest even); activations are rounded to bfloat16 at every
product's input; sums are FP32.  ``exact=True`` turns every rounding off and
computes in float64 -- that form is what the finite-difference pins check.
"""
from __future__ import annotations

import numpy as np

SQRT_2_OVER_PI = np.sqrt(2.0 / np.pi)
GELU_C = 0.044715


def bf16_round(x: np.ndarray) -> np.ndarray:
    """Round float32 values to the nearest bfloat16 (ties to even), as float32."""
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = a.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) & 0xFFFF0000).astype(np.uint32)
    return r.view(np.float32).reshape(a.shape)


def gelu(x):
    return 0.5 * x * (1.0 + np.tanh(SQRT_2_OVER_PI * (x + GELU_C * x ** 3)))


def gelu_grad(x):
    u = SQRT_2_OVER_PI * (x + GELU_C * x ** 3)
    t = np.tanh(u)
    du = SQRT_2_OVER_PI * (1.0 + 3.0 * GELU_C * x ** 2)
    return 0.5 * (1.0 + t) + 0.5 * x * (1.0 - t * t) * du


def features(seqs: np.ndarray, C_even: np.ndarray) -> np.ndarray:
    """x per walker state: the +1/-1 sequence then C_{2m}/(L-2m), m = 1..k.
    seqs [n, L] int8; C_even [n, k] the even-lag autocorrelations."""
    n, L = seqs.shape
    k = (L - 1) // 2
    den = (L - 2 * np.arange(1, k + 1)).astype(np.float64)
    return np.concatenate([seqs.astype(np.float64), C_even.astype(np.float64) / den[None, :]],
                          axis=1)


def _q(a, exact):
    return np.asarray(a, dtype=np.float64) if exact else bf16_round(a).astype(np.float64)


def _mm(a, b, exact):
    """Product of two already-rounded operands: float64 when exact, else the
    float64 sum rounded to float32 (FP32 accumulation)."""
    r = a @ b
    return r if exact else r.astype(np.float32).astype(np.float64)


def forward(P: dict, X: np.ndarray, exact: bool = False):
    """Logits [n, d_out] and the cache for backward.  P holds W1 [h, d_in], b1 [h],
    W2 [h, h], b2 [h], W3 [d_out, h], b3 [d_out]."""
    f = (lambda a: np.asarray(a, dtype=np.float64)) if exact else \
        (lambda a: np.asarray(a, dtype=np.float32).astype(np.float64))
    x = _q(X, exact)
    a1 = _mm(x, _q(P["W1"], exact).T, exact) + f(P["b1"])
    if not exact:
        a1 = a1.astype(np.float32).astype(np.float64)
    h1 = gelu(a1)
    h1q = _q(h1, exact)
    a2 = _mm(h1q, _q(P["W2"], exact).T, exact) + f(P["b2"])
    if not exact:
        a2 = a2.astype(np.float32).astype(np.float64)
    h2 = gelu(a2)
    h2q = _q(h2, exact)
    z = _mm(h2q, _q(P["W3"], exact).T, exact) + f(P["b3"])
    if not exact:
        z = z.astype(np.float32).astype(np.float64)
    return z, dict(x=x, a1=a1, h1q=h1q, a2=a2, h2q=h2q)


def masked_ce(z: np.ndarray, mask: np.ndarray, labels: np.ndarray):
    """Mean softmax cross-entropy over the admissible entries (mask True) and its
    gradient with respect to z."""
    n = z.shape[0]
    zm = np.where(mask, z, -np.inf)
    mx = zm.max(axis=1, keepdims=True)
    e = np.where(mask, np.exp(zm - mx), 0.0)
    ssum = e.sum(axis=1, keepdims=True)
    logp = zm - mx - np.log(ssum)
    loss = -logp[np.arange(n), labels].mean()
    p = e / ssum
    dz = p.copy()
    dz[np.arange(n), labels] -= 1.0
    return float(loss), dz / n


def backward(P: dict, cache: dict, dz: np.ndarray, exact: bool = False, operands: dict = None) -> dict:
    """Gradients of the loss for every parameter; the products use the same
    rounded operands as the forward pass (and a rounded upstream gradient).
    When `operands` is a dict, it receives, per parameter, the two factors whose
    products over the batch rows the gradient sums ((upstream, input) for a
    weight, (upstream, None) for a bias)."""
    q = (lambda a: _q(a, exact))
    dzq = q(dz)
    g = {}
    g["W3"] = _mm(dzq.T, cache["h2q"], exact)
    g["b3"] = dz.sum(axis=0)
    dh2 = _mm(dzq, q(P["W3"]), exact)
    da2 = dh2 * gelu_grad(cache["a2"])
    da2q = q(da2)
    g["W2"] = _mm(da2q.T, cache["h1q"], exact)
    g["b2"] = da2.sum(axis=0)
    dh1 = _mm(da2q, q(P["W2"]), exact)
    da1 = dh1 * gelu_grad(cache["a1"])
    da1q = q(da1)
    g["W1"] = _mm(da1q.T, cache["x"], exact)
    g["b1"] = da1.sum(axis=0)
    if operands is not None:
        operands.update(W3=(dzq, cache["h2q"]), b3=(dz, None), W2=(da2q, cache["h1q"]), b2=(da2, None),
                        W1=(da1q, cache["x"]), b1=(da1, None))
    return g


def loss_and_grads(P, X, mask, labels, exact=False, operands=None):
    z, cache = forward(P, X, exact)
    loss, dz = masked_ce(z, mask, labels)
    return loss, backward(P, cache, dz, exact, operands)


def term_norms(operands: dict) -> dict:
    """Per gradient element, the 2-norm over batch rows of the products the
    element sums: sqrt(sum_n (u_nj v_ni)^2) for a weight, sqrt(sum_n u_nj^2) for a
    bias.  It scales the rounding a batch sum of bf16 products can carry."""
    out = {}
    for key, (u, v) in operands.items():
        u2 = np.asarray(u, dtype=np.float64) ** 2
        out[key] = np.sqrt(u2.sum(axis=0) if v is None else u2.T @ (np.asarray(v, dtype=np.float64) ** 2))
    return out


def adam(P: dict, G: dict, M: dict, V: dict, t: int, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (FP32 masters) in place; t counts from 1."""
    for key in P:
        g = np.asarray(G[key], dtype=np.float32)
        M[key] = (b1 * M[key] + (1 - b1) * g).astype(np.float32)
        V[key] = (b2 * V[key] + (1 - b2) * g * g).astype(np.float32)
        mh = M[key] / (1 - b1 ** t)
        vh = V[key] / (1 - b2 ** t)
        P[key] = (P[key] - lr * mh / (np.sqrt(vh) + eps)).astype(np.float32)


def top_m(z: np.ndarray, mask: np.ndarray, m: int) -> np.ndarray:
    """Indices of the m largest admissible logits per row (ties: lower index)."""
    out = np.full((z.shape[0], m), -1, dtype=np.int64)
    for r in range(z.shape[0]):
        idx = [j for j in range(z.shape[1]) if mask[r, j]]
        idx.sort(key=lambda j: (-z[r, j], j))
        out[r, :min(m, len(idx))] = idx[:m]
    return out
