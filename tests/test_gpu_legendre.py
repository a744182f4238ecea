"""GPU parity of the Legendre-construction seeds (Sec. 4.1) against the oracle:
the sweep's sequences and energies bit for bit, the table's construction column,
and the second step seeded with them."""
import os

import numpy as np
import pytest

import labs_inputs as li

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden", "legendre_construct.txt")


@pytest.fixture(scope="module")
def lb():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2409_07222_amd import labs
    labs.lib()
    return labs


def _rows():
    out = []
    for line in open(GOLD):
        line = line.split("#")[0].strip()
        if line:
            L, n, o, F = line.split()
            out.append((int(L), int(n), int(o), F))
    return out


def _check_pairs(lb, orc, L, n, o):
    seqs, E = lb.legendre_build(L, n, o)
    got = li.unpack(seqs.cpu().numpy().view(np.uint32), L)
    Eg = E.cpu().numpy()
    chis = {}
    for i, (nn, oo) in enumerate(zip(n.tolist(), o.tolist())):
        if nn not in chis:
            chis[nn] = orc.legendre_chi(nn)
        want = orc.legendre_sequence(nn, oo, L, chis[nn])
        assert np.array_equal(got[i], want), (nn, oo)
    assert np.array_equal(Eg, orc.energy_batch(got))
    return got, Eg


@pytest.mark.parametrize("row", range(4))
def test_sweep_reproduces_the_construction_column(lb, orc, row):
    L, n0, o0, F = _rows()[row]
    n, o = lb.legendre_pairs(L)
    assert list(zip(n.tolist(), o.tolist())) == orc.legendre_pairs(L)
    got, E = _check_pairs(lb, orc, L, n, o)
    b = int(np.argmin(E))
    assert "%.4f" % orc.merit_factor(L, int(E[b])) == F
    assert (int(n[b]), int(o[b])) == (n0, o0)


def test_edge_pairs(lb, orc):
    # smallest primes, full rotation range, lengths shorter and longer than n
    for L, pairs in ((5, [(3, 0), (3, 2), (5, 0), (5, 4)]), (2, [(3, 1), (7, 6)]),
                     (64, [(1019, 0), (1019, 1018), (61, 13)]),
                     (1023, [(1021, 0), (1021, 230), (3, 1), (1019, 500)])):
        n = np.array([p[0] for p in pairs], np.int32)
        o = np.array([p[1] for p in pairs], np.int32)
        _check_pairs(lb, orc, L, n, o)
    s, E = lb.legendre_build(101, np.zeros(0, np.int32), np.zeros(0, np.int32))
    assert s.shape[0] == 0 and E.shape[0] == 0


def test_invalid_pairs(lb):
    for L, n, o in ((101, 9, 0), (101, 97, 97), (101, 97, -1), (1024, 97, 0), (101, 2, 0), (101, 1031, 0)):
        with pytest.raises(lb.LabsError):
            lb.legendre_build(L, np.array([n], np.int32), np.array([o], np.int32))


def test_seeded_second_step_parity(lb, orc):
    """The second step from the sweep's seeds at L = 61 equals the oracle's
    search: best, statistics and the final Open set."""
    L = 61
    n, o = lb.legendre_pairs(L)
    seqs, E = lb.legendre_build(L, n, o)
    cands = li.unpack(seqs.cpu().numpy().view(np.uint32), L)
    assert len(cands) >= 8
    g = lb.refine_step2(L, seqs, 8, 400, 160, 1 << 40, open_capacity=400)
    r = orc.step2(L, list(cands), 8, 400, 160, 1 << 40)
    for f in ("expansions", "pushes", "dup_skips", "evictions", "rounds", "best_round"):
        assert g[f] == r[f], f
    assert g["best_E"] == r["best_E"] <= int(E.min().item())
    gs = li.unpack(g["best_seq"].cpu().numpy().view(np.uint32), L)
    assert orc.seq_key(gs) == r["best_key"]


def test_seeded_second_step_L450(lb, orc):
    L = 450
    n, o = lb.legendre_pairs(L)
    seqs, E = lb.legendre_build(L, n, o)
    g = lb.refine_step2(L, seqs, 256, 1 << 16, 20000, 1 << 40)
    assert g["expansions"] == 20000
    assert g["best_E"] <= int(E.min().item())
    best = li.unpack(g["best_seq"].cpu().numpy().view(np.uint32)[None, :], L)[0]
    assert orc.energy(best) == g["best_E"]
