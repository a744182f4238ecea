"""GPU parity of the end operators (remove or append an element at either end)
against the oracle, bit for bit, and the second step run from their outputs at
the even neighbouring lengths."""
import numpy as np
import pytest

import labs_inputs as li

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lb():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2409_07222_amd import labs
    labs.lib()
    return labs


def _dev(packed):
    import torch
    return torch.from_numpy(np.ascontiguousarray(packed).view(np.int32)).cuda()


@pytest.mark.parametrize("L", [1, 2, 3, 31, 32, 33, 63, 64, 65, 500, 501, 1021, 1022])
def test_operators_parity(lb, orc, L):
    S = li.random_pm1(700 + L, 6, L)
    minus, Em, plus, Ep = lb.length_operators(L, _dev(li.pack(S)))
    gp = li.unpack(plus.cpu().numpy().view(np.uint32), L + 1)
    gE = Ep.cpu().numpy()
    if L >= 2:
        gm = li.unpack(minus.cpu().numpy().view(np.uint32), L - 1)
        gEm = Em.cpu().numpy()
    for j, s in enumerate(S):
        m, p = orc.length_operators(s)
        assert np.array_equal(gp[4 * j:4 * j + 4], p)
        assert np.array_equal(gE[4 * j:4 * j + 4], orc.energy_batch(p))
        if L >= 2:
            assert np.array_equal(gm[2 * j:2 * j + 2], m)
            assert np.array_equal(gEm[2 * j:2 * j + 2], orc.energy_batch(m))


def test_operators_edges(lb):
    import torch
    z = torch.zeros((0, 16), dtype=torch.int32, device="cuda")
    minus, Em, plus, Ep = lb.length_operators(501, z)
    assert plus.shape[0] == 0 and minus.shape[0] == 0
    with pytest.raises(lb.LabsError):
        lb.length_operators(1023, _dev(li.pack(li.random_pm1(1, 2, 1023))))


@pytest.mark.parametrize("L", [21, 33])
def test_second_step_at_even_lengths(lb, orc, L):
    """Sequences of odd length L carried to L - 1 and L + 1 seed the second step
    there; best, statistics and Open equal the oracle's search."""
    S = li.random_pm1(31 + L, 3, L)
    minus, Em, plus, Ep = lb.length_operators(L, _dev(li.pack(S)))
    for Lq, seqs in ((L - 1, minus), (L + 1, plus)):
        cands = li.unpack(seqs.cpu().numpy().view(np.uint32), Lq)
        g = lb.refine_step2(Lq, seqs, 4, 300, 120, 1 << 40, open_capacity=300)
        o = orc.step2(Lq, list(cands), 4, 300, 120, 1 << 40)
        for f in ("expansions", "pushes", "dup_skips", "evictions", "rounds", "best_round"):
            assert g[f] == o[f], (Lq, f)
        assert g["best_E"] == o["best_E"]
        got = sorted((int(e), orc.seq_key(s)) for e, s in
                     zip(g["open_E"].cpu().numpy(),
                         li.unpack(g["open_seqs"].cpu().numpy().view(np.uint32), Lq)))
        assert got == o["open_keys"]
