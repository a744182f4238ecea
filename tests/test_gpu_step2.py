"""GPU parity of the second step (batch-synchronous best-first search)
against the oracle: best, statistics and the final Open set, exactly."""
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


def _run_both(lb, orc, L, cands, B, Q, X, T_u, T_r=0):
    g = lb.refine_step2(L, _dev(li.pack(cands)), B, Q, X, T_u, open_capacity=Q, T_r=T_r)
    o = orc.step2(L, list(cands), B, Q, X, T_u, T_r=T_r)
    for f in ("expansions", "pushes", "dup_skips", "evictions", "rounds", "best_round"):
        assert g[f] == o[f], (f, g[f], o[f])
    assert g["best_E"] == o["best_E"]
    gs = li.unpack(g["best_seq"].cpu().numpy().view(np.uint32), L)
    assert orc.seq_key(gs) == o["best_key"]
    assert g["open_count"] == len(o["open_keys"])
    got = sorted((int(e), orc.seq_key(s)) for e, s in
                 zip(g["open_E"].cpu().numpy(),
                     li.unpack(g["open_seqs"].cpu().numpy().view(np.uint32), L)))
    assert got == o["open_keys"]
    return g, o


@pytest.mark.parametrize("L,n,B,Q,X,T_u", [
    (11, 3, 1, 1 << 20, 100, 1 << 40),     # Algorithm 2 exactly (batch 1)
    (13, 4, 4, 30, 200, 1 << 40),          # capacity cut and re-pushes
    (16, 2, 7, 1 << 20, 300, 1 << 40),     # even length, ragged batch
    (33, 5, 3, 64, 150, 12),               # dynamic depth stop
    (101, 6, 64, 3000, 1500, 300),         # second configuration's length
    (200, 2, 32, 500, 400, 1 << 40),
    (701, 2, 4, 200, 16, 1 << 40),         # direct expansion (lags beyond the bit-sliced kernels)
    (1023, 2, 2, 100, 8, 1 << 40),         # longest accepted length
    (17, 4, 8, 2, 60, 1 << 40),            # queue smaller than the batch: every survivor is popped
    (19, 6, 16, 5, 100, 1 << 40),
    (2, 3, 2, 8, 10, 1 << 40),             # the shortest lengths: every energy ties, the
    (3, 4, 2, 3, 12, 1 << 40),             # space is exhausted and Open ends empty
])
def test_step2_parity(lb, orc, L, n, B, Q, X, T_u):
    cands = li.random_pm1(L * 7 + n, n, L)
    _run_both(lb, orc, L, cands, B, Q, X, T_u)


@pytest.mark.parametrize("L", [257, 385, 386, 512, 513, 545, 546, 641])
def test_step2_expansion_shapes(lb, orc, L):
    """Each bit-sliced expansion kernel at the ends of its length range: 257 (two
    lane groups of 256 positions, the first full), 385 / 386 (12 / 16 lag words),
    512 / 513 (two / three groups), 545 / 546 (17 / 20 words) and 641 (the
    longest before the direct expansion).  A group's window words past the lags its
    positions reach are skipped, so these lengths put the last reachable word at
    every boundary the skip depends on."""
    cands = li.random_pm1(L * 7 + 2, 2, L)
    _run_both(lb, orc, L, cands, 4, 200, 16 if L > 400 else 24, 1 << 40)


def test_step2_table_rebuild(lb, orc):
    """More distinct sequences pass through Open than half of the hash set holds
    (9,699 in this run against 8,192 of the 16,384 slots sized for L = 33, batch 1,
    queue 1,600, 1,900 pops): the set is rebuilt without its evicted tombstones,
    and no result changes."""
    L, n, B, Q, X = 33, 3, 1, 1600, 1900
    cands = li.random_pm1(L * 7 + n, n, L)
    g, _ = _run_both(lb, orc, L, cands, B, Q, X, 1 << 40)
    assert g["rebuilds"] >= 1, g["rebuilds"]


def test_step2_L501(lb, orc):
    L = 501
    cands = li.random_skew(5, 3, L, 16)
    _run_both(lb, orc, L, cands, 16, 1000, 48, 1 << 40)


def test_step2_full_space(lb, orc):
    """Room for all 2^10 sequences: the search ends at the published optimum."""
    L = 10
    cands = li.random_pm1(3, 2, L)
    g, o = _run_both(lb, orc, L, cands, 5, 1 << 20, 1 << 20, 1 << 40)
    assert g["best_E"] == 13 and g["expansions"] == 1 << L


@pytest.mark.parametrize("T_r", [0, 3])
def test_step2_large_tie_sets(lb, orc, T_r):
    """Every sequence of length 18 as a seed: at this length many sequences share
    each energy, so both of each cut's thresholds (the queue's 30,000th entry and
    the 4,096th, the next round's pivots) fall inside tie sets of thousands of
    entries, beyond what the tie select holds on chip; most neighbours re-push
    evicted sequences (tombstones) or are duplicates."""
    L = 18
    cands = li.all_pm1_shuffled(3, L)
    g, o = _run_both(lb, orc, L, cands, 4096, 30000, 2 * 4096, 1 << 40, T_r=T_r)
    assert g["evictions"] > 50000 and g["pushes"] > 50000 and g["dup_skips"] > 50000


def test_step2_wide_range_large_bin(lb, orc):
    """40,000 random seeds of length 301 and the all-ones sequence: the energy range
    spans 2^22 values of (E - emin)/4, so the seeding cut's radix level leaves a bin
    of 256 such values holding about 2,700 entries, which the tie select resolves
    from device memory before the key bytes."""
    L = 301
    c = li.random_pm1(41, 40000, L)
    cands = np.concatenate([c, np.ones((1, L), np.int8)])
    _run_both(lb, orc, L, cands, 8, 10000, 32, 1 << 40)


@pytest.mark.parametrize("T_r", [0, 2])
def test_step2_unbounded_queue(lb, orc, T_r):
    """A queue no cut reaches (Alg. 2's, without capacity): nothing is evicted and
    Open and Closed hold exactly the distinct seeds and the pushes."""
    L, B, X = 23, 8, 200
    cands = li.random_pm1(12, 5, L)
    g, o = _run_both(lb, orc, L, cands, B, 5 + X * (L + 2 * T_r), X, 1 << 40, T_r=T_r)
    assert g["evictions"] == 0 and g["expansions"] == X
    assert g["open_count"] + g["expansions"] == 5 + g["pushes"]


def test_step2_duplicate_candidates(lb, orc):
    L = 21
    c = li.random_pm1(9, 4, L)
    cands = np.concatenate([c, c[:2], c[:1]])
    _run_both(lb, orc, L, cands, 2, 100, 40, 1 << 40)


def test_step2_zero_budget(lb, orc):
    L = 15
    cands = li.random_pm1(2, 3, L)
    g, o = _run_both(lb, orc, L, cands, 4, 100, 0, 1 << 40)
    assert g["expansions"] == 0 and g["rounds"] == 0


# ------------------------------------------------------------------ rotations
@pytest.mark.parametrize("L,n,B,Q,X,T_u,T_r", [
    (11, 3, 1, 1 << 20, 60, 1 << 40, 2),       # Algorithm 2 with rotations, batch 1
    (13, 4, 4, 30, 200, 1 << 40, 3),           # capacity cut and re-pushes
    (16, 2, 7, 1 << 20, 300, 1 << 40, 7),      # even length, 2 T_r = L - 2
    (33, 5, 3, 64, 150, 12, 1),                # dynamic depth stop
    (101, 6, 64, 3000, 1500, 300, 8),
    (200, 2, 32, 500, 400, 1 << 40, 32),       # the largest T_r
    (527, 2, 4, 200, 16, 1 << 40, 4),          # three lane groups of the bit-sliced expansion
    (701, 2, 4, 200, 16, 1 << 40, 4),          # direct expansion
    (1023, 2, 2, 100, 8, 1 << 40, 32),
    (5, 5, 3, 6, 40, 1 << 40, 1),              # exhausted space with rotations
    (6, 4, 2, 5, 30, 1 << 40, 2),              # even length, 2 T_r = L - 2
])
def test_step2_rotations_parity(lb, orc, L, n, B, Q, X, T_u, T_r):
    cands = li.random_pm1(L * 11 + n, n, L)
    g, o = _run_both(lb, orc, L, cands, B, Q, X, T_u, T_r)
    assert g["pushes"] + g["dup_skips"] == g["expansions"] * (L + 2 * T_r)


def test_step2_rotations_periodic_pivot(lb, orc):
    """A pivot of period 3 meets itself at shift 3 and repeats its own rotations."""
    L = 9
    c = np.array([[1, 1, -1] * 3], np.int8)
    _run_both(lb, orc, L, c, 1, 1 << 20, 1, 1 << 40, 4)
    _run_both(lb, orc, L, c, 2, 1 << 20, 40, 1 << 40, 4)


def test_step2_rotations_full_space(lb, orc):
    """Room for all 2^10 sequences: with rotations the search still ends at the
    published optimum after popping every sequence once."""
    L = 10
    cands = li.random_pm1(4, 2, L)
    g, o = _run_both(lb, orc, L, cands, 5, 1 << 20, 1 << 20, 1 << 40, 2)
    assert g["best_E"] == 13 and g["expansions"] == 1 << L


def test_step2_rotations_L501(lb, orc):
    L = 501
    cands = li.random_skew(6, 3, L, 16)
    _run_both(lb, orc, L, cands, 16, 1000, 48, 1 << 40, 4)


@pytest.mark.parametrize("L,B,Q,X", [(301, 4, 50, 40), (501, 3, 20, 12), (64, 2, 30, 30)])
def test_step2_wide_energy_range(lb, orc, L, B, Q, X):
    """Candidates whose energies span millions (the all +1 and alternating
    sequences beside random ones): one 14-bit radix level cannot resolve the
    selection, so the tie select resolves the threshold bin's energies first."""
    allp = np.ones(L, np.int8)
    alt = np.array([1 if i % 2 == 0 else -1 for i in range(L)], np.int8)
    rnd = li.random_pm1(L + 3, 5, L)
    cands = np.concatenate([allp[None], alt[None], rnd])
    E = [orc.energy(x) for x in cands]
    if L > 100:
        assert (max(E) - min(E)) // 4 >= 1 << 14
    _run_both(lb, orc, L, cands, B, Q, X, 1 << 40)
    _run_both(lb, orc, L, cands, B, Q, X, 1 << 40, T_r=2)
