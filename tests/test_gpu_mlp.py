"""GPU parity of the learned-proposal network through the C ABI against the
CPU reference (oracle/mlp.py): features bit for bit, logits within 1e-2
relative, every gradient element within a tolerance of its own (relative to
the element, with a floor from the products it sums), Adam bit for bit."""
import numpy as np
import pytest

import labs_inputs as li
from oracle import mlp as omlp

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lb():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2409_07222_amd import labs
    labs.lib()
    return labs


def _dev_i32(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a).view(np.int32)).cuda()


def _c_even(orc, S):
    return np.stack([orc.energy(x, with_c=True)[1][1::2] for x in S])


def _params(lb, L, hidden, seed):
    import torch
    lay = lb.mlp_layout(L, hidden)
    P = li.mlp_init(seed, lay.d_in, hidden, lay.d_out)
    g = li.rng(seed + 7)
    for b in ("b1", "b2", "b3"):
        P[b] = (g.normal(size=P[b].shape) * 0.05).astype(np.float32)
    blob = torch.from_numpy(lb.mlp_blob_from_dict(lay, P)).cuda()
    pb = torch.empty(lay.n_params, dtype=torch.bfloat16, device="cuda")
    lb.mlp_cast(lay, blob, pb)
    return lay, P, blob, pb


def _mask_labels(seed, n, d_out):
    g = li.rng(seed)
    adm = g.random((n, d_out)) < 0.6
    labels = np.array([g.choice(np.flatnonzero(r)) if r.any() else 0 for r in adm], np.int32)
    adm[np.arange(n), labels] = True
    mw = (d_out + 31) // 32
    words = np.zeros((n, mw), np.uint32)
    for j in range(d_out):
        words[:, j // 32] |= adm[:, j].astype(np.uint32) << np.uint32(j % 32)
    return adm, labels, words


@pytest.mark.parametrize("L", [5, 37, 101, 501, 1023])
def test_features_bit_exact(lb, orc, L):
    S = li.random_skew(300 + L, 67, L, 0)
    X = lb.mlp_features(L, _dev_i32(li.pack(S)))
    lay = lb.mlp_layout(L, 64)
    want = omlp.bf16_round(omlp.features(S, _c_even(orc, S)).astype(np.float32))
    got = X.float().cpu().numpy()
    assert np.array_equal(got[:, :lay.d_in].view(np.uint32), want.view(np.uint32))
    assert np.all(got[:, lay.d_in:] == 0)


@pytest.mark.parametrize("L,hidden,n", [(37, 64, 1), (101, 128, 300), (501, 256, 257), (501, 256, 1000), (101, 64, 700)])
def test_forward_logits(lb, orc, L, hidden, n):
    lay, P, blob, pb = _params(lb, L, hidden, 55)
    S = li.random_skew(11 * L, n, L, 0)
    X = lb.mlp_features(L, _dev_i32(li.pack(S)))
    z = lb.mlp_forward(lay, blob, pb, X).cpu().numpy()[:, :lay.d_out]
    zr, _ = omlp.forward(P, omlp.features(S, _c_even(orc, S)), exact=False)
    err = np.abs(z - zr) / np.maximum(np.abs(zr), 1.0)
    assert err.max() <= 1e-2, err.max()


def test_forward_logits_128_tiles(lb, orc):
    """33,000 rows at L = 501, hidden 256: the grid of 128 x 128 tiles holds 516
    workgroups, so the forward runs the 128-tile kernel; its last row tile is
    ragged (104 rows).  The oracle scores sampled rows one by one: the first and
    last tiles whole and 1,500 rows between."""
    L, hidden, n = 501, 256, 33_000
    lay, P, blob, pb = _params(lb, L, hidden, 60)
    S = li.random_skew(4242, n, L, 0)
    X = lb.mlp_features(L, _dev_i32(li.pack(S)))
    z = lb.mlp_forward(lay, blob, pb, X).cpu().numpy()[:, :lay.d_out]
    rows = np.unique(np.concatenate([np.arange(128), np.arange(n - 232, n),
                                     li.rng(61).choice(n, 1500, replace=False)]))
    Sr = S[rows]
    zr, _ = omlp.forward(P, omlp.features(Sr, _c_even(orc, Sr)), exact=False)
    err = np.abs(z[rows] - zr) / np.maximum(np.abs(zr), 1.0)
    assert err.max() <= 1e-2, err.max()


@pytest.mark.parametrize("L,hidden,n", [(37, 64, 100), (101, 64, 257), (501, 256, 512), (501, 256, 4096)])
def test_gradients(lb, orc, L, hidden, n):
    """Every gradient element against the oracle's, with a tolerance of its own:
    1e-2 of the element plus 2^-7 of the 2-norm of the batch products it sums
    (one bf16 rounding step of each product, the scale at which a flipped
    rounding of an operand shows).  n = 4096 is the training batch: the weight
    gradients split K = 4096 over 11-16 slices."""
    import torch
    lay, P, blob, pb = _params(lb, L, hidden, 56)
    S = li.random_skew(13 * L, n, L, 0)
    X = lb.mlp_features(L, _dev_i32(li.pack(S)))
    adm, labels, words = _mask_labels(L, n, lay.d_out)
    G, loss = lb.mlp_grads(lay, blob, pb, X, _dev_i32(words),
                           torch.from_numpy(labels).cuda())
    Gd = lb.mlp_dict_from_blob(lay, G.cpu().numpy())
    ops = {}
    lr, Gr = omlp.loss_and_grads(P, omlp.features(S, _c_even(orc, S)), adm, labels, exact=False,
                                 operands=ops)
    norms = omlp.term_norms(ops)
    assert abs(float(loss.item()) - lr) <= 1e-3 * max(1.0, abs(lr))
    for key in omlp_keys():
        ref = Gr[key]
        tol = 1e-2 * np.abs(ref) + 2.0 ** -7 * norms[key] + 1e-9
        bad = np.abs(Gd[key] - ref) > tol
        assert not bad.any(), (key, int(bad.sum()), float((np.abs(Gd[key] - ref) / tol).max()))
    # pads of the gradient blob are zero
    full = G.cpu().numpy()
    W1 = full[lay.off_W1:lay.off_W1 + hidden * lay.ld_in].reshape(hidden, lay.ld_in)
    assert np.all(W1[:, lay.d_in:] == 0)


def omlp_keys():
    return ("W1", "b1", "W2", "b2", "W3", "b3")


def test_adam_bit_exact(lb):
    import torch
    lay = lb.mlp_layout(101, 64)
    g = li.rng(9)
    n = lay.n_params
    P0 = g.normal(size=n).astype(np.float32)
    G0 = (g.normal(size=n) * 1e-2).astype(np.float32)
    M0 = (g.normal(size=n) * 1e-3).astype(np.float32)
    V0 = np.abs(g.normal(size=n) * 1e-5).astype(np.float32)
    Pd, Gd, Md, Vd = (torch.from_numpy(a.copy()).cuda() for a in (P0, G0, M0, V0))
    pb = torch.empty(n, dtype=torch.bfloat16, device="cuda")
    Ph, Mh, Vh = {"w": P0.copy()}, {"w": M0.copy()}, {"w": V0.copy()}
    for t in (1, 2, 3):
        lb.mlp_adam(lay, Pd, pb, Gd, Md, Vd, t, lr=1e-3)
        omlp.adam(Ph, {"w": G0}, Mh, Vh, t, lr=1e-3)
        assert np.array_equal(Pd.cpu().numpy().view(np.uint32), Ph["w"].view(np.uint32))
        assert np.array_equal(Md.cpu().numpy().view(np.uint32), Mh["w"].view(np.uint32))
        assert np.array_equal(Vd.cpu().numpy().view(np.uint32), Vh["w"].view(np.uint32))
    want_b = omlp.bf16_round(Ph["w"])
    assert np.array_equal(pb.float().cpu().numpy().view(np.uint32), want_b.view(np.uint32))


def test_train_step_is_features_grads_adam(lb, orc):
    import torch
    L, hidden, n = 101, 64, 200
    lay, P, blob, pb = _params(lb, L, hidden, 57)
    S = li.random_skew(17, n, L, 0)
    seqs = _dev_i32(li.pack(S))
    adm, labels, words = _mask_labels(3, n, lay.d_out)
    mask_d, lab_d = _dev_i32(words), torch.from_numpy(labels).cuda()
    # composition
    b1, p1 = blob.clone(), pb.clone()
    m1, v1 = torch.zeros_like(blob), torch.zeros_like(blob)
    X = lb.mlp_features(L, seqs)
    G1, loss1 = lb.mlp_grads(lay, b1, p1, X, mask_d, lab_d)
    lb.mlp_adam(lay, b1, p1, G1, m1, v1, 1)
    # one call
    b2, p2 = blob.clone(), pb.clone()
    m2, v2 = torch.zeros_like(blob), torch.zeros_like(blob)
    G2 = torch.empty_like(blob)
    loss2, _ = lb.mlp_train_step(lay, b2, p2, G2, m2, v2, 1, seqs, mask_d, lab_d)
    torch.cuda.synchronize()
    assert torch.equal(b1, b2) and torch.equal(G1, G2) and torch.equal(loss1, loss2)
    assert torch.equal(p1.view(torch.int16), p2.view(torch.int16))


def test_training_lowers_loss(lb, orc):
    """A few hundred steps on a fixed batch drive the masked cross-entropy down."""
    import torch
    L, hidden, n = 37, 64, 256
    lay, P, blob, pb = _params(lb, L, hidden, 58)
    S = li.random_skew(19, n, L, 0)
    seqs = _dev_i32(li.pack(S))
    adm, labels, words = _mask_labels(4, n, lay.d_out)
    mask_d, lab_d = _dev_i32(words), torch.from_numpy(labels).cuda()
    m, v, G = torch.zeros_like(blob), torch.zeros_like(blob), torch.empty_like(blob)
    ws = None
    losses = []
    for t in range(1, 301):
        loss, ws = lb.mlp_train_step(lay, blob, pb, G, m, v, t, seqs, mask_d, lab_d, lr=3e-3,
                                     workspace=ws)
        if t in (1, 300):
            losses.append(float(loss.item()))
    assert losses[1] < 0.5 * losses[0], losses


def test_empty_batch(lb):
    import torch
    L = 101
    lay, P, blob, pb = _params(lb, L, 64, 59)
    X = lb.mlp_features(L, torch.zeros((0, 4), dtype=torch.int32, device="cuda"))
    assert tuple(X.shape) == (0, lay.ld_in)
    z = lb.mlp_forward(lay, blob, pb, X)
    assert tuple(z.shape) == (0, lay.ld_out)
    G, loss = lb.mlp_grads(lay, blob, pb, X, torch.zeros((0, lay.mask_words), dtype=torch.int32,
                                                         device="cuda"),
                           torch.zeros(0, dtype=torch.int32, device="cuda"))
    assert float(loss.item()) == 0.0 and not bool(G.any().item())
