"""Parity at the benchmark's full sizes (L = 501, p = 16, 16,384 walkers x 50,000
steps, F >= 8 sieve into a 2^20 pool, top-1024, second step with batch 1024,
queue 2^20 and 10^7 expansions), in the launch configuration bench.py times.
The oracle cannot replay these runs whole, so the checks are on sampled outputs
it computes one by one (energies of final, best, pool and Open sequences; the
first steps of sampled walkers) and on properties that hold at any size."""
import numpy as np
import pytest

import labs_inputs as li

pytestmark = pytest.mark.gpu

L, P, LO, HI, N, STEPS = 501, 16, 50, 100, 16384, 50000
E_MAX = (L * L) // 16          # tau = 8
CAP, TOPK = 1 << 20, 1024


@pytest.fixture(scope="module")
def lb():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2409_07222_amd import labs
    labs.lib()
    return labs


@pytest.fixture(scope="module")
def step1(lb):
    pool = lb.PoolBuffers.empty(L, CAP)
    r = lb.walk_step1(L, P, STEPS, LO, HI, 4, N, e_max=E_MAX, pool=pool, pool_walker_best=True,
                      want_traj=True)
    s, E = lb.pool_topk(pool, TOPK)
    return r, pool, s, E


def _seqs(t):
    return li.unpack(t.cpu().numpy().view(np.uint32), L)


def test_step1_full_size_sampled(lb, orc, step1):
    r, pool, s, E = step1
    assert int(r.flip_evals.item()) == N * STEPS * ((L - 1) // 2 + 1 - P)
    g = li.rng(11)
    sample = np.sort(g.choice(N, 64, replace=False))
    fin = _seqs(r.final_seqs[sample])
    best = _seqs(r.best_seqs[sample])
    fE = r.final_E.cpu().numpy()[sample]
    bE = r.best_E.cpu().numpy()[sample]
    assert np.array_equal(orc.energy_batch(fin), fE)
    assert np.array_equal(orc.energy_batch(best), bE)
    traj = r.traj_E[sample].cpu().numpy()
    bstep = r.best_step.cpu().numpy()[sample]
    for j in range(len(sample)):
        assert traj[j, -1] == fE[j]
        assert bE[j] <= traj[j].min()
        if bstep[j] > 0:   # the first step reaching the walk's lowest energy
            assert traj[j, bstep[j] - 1] == bE[j] and np.all(traj[j, :bstep[j] - 1] > bE[j])
    # the first steps of two walkers, replayed by the oracle
    o = orc.walk(L, P, 40, LO, HI, 4, [int(sample[0]), int(sample[-1])])
    assert np.array_equal(traj[[0, -1], :40], o["traj"])
    # three walkers replayed whole (50,000 steps: every pool segment and launch
    # boundary of the run) by the oracle's linear-time walker, which the CPU suite
    # pins step for step to the definitional one
    for w in (int(sample[0]), int(sample[len(sample) // 2]), int(sample[-1])):
        b = orc.baseline_walk(L, P, STEPS, LO, HI, 4, w, 1, threads=1, want_traj=True)
        j = int(np.flatnonzero(sample == w)[0])
        assert np.array_equal(traj[j], b["traj"][0]), w
        assert int(b["final_E"][0]) == fE[j] and int(b["best_E"][0]) == bE[j]


def test_pool_and_topk_full_size(lb, orc, step1):
    r, pool, s, E = step1
    c = int(pool.count.item())
    assert 0 < c <= CAP
    pe = pool.E[:c].cpu().numpy()
    assert pe.max() <= max(E_MAX, int(r.best_E.max().item()))
    seqs = pool.seqs[:c].cpu().numpy().view(np.uint32)
    assert len({row.tobytes() for row in seqs}) == c          # distinct sequences
    g = li.rng(12)
    idx = g.choice(c, min(c, 256), replace=False)
    assert np.array_equal(orc.energy_batch(li.unpack(seqs[idx], L)), pe[idx])
    # top-k: the k smallest (E, key) of the pool in key order (words compared as
    # unsigned integers, word 0 first)
    tE, tS = E.cpu().numpy(), s.cpu().numpy().view(np.uint32)
    keys = sorted(zip(pe.tolist(), [row.tobytes() for row in seqs.byteswap()]))[:len(tE)]
    assert tE.tolist() == [k[0] for k in keys]
    assert [row.tobytes() for row in tS.byteswap()] == [k[1] for k in keys]


def test_step2_full_size_properties(lb, orc, step1):
    r, pool, s, E = step1
    X = 10_000_000
    res = lb.refine_step2(L, s.contiguous(), 1024, 1 << 20, X, 1 << 62, open_capacity=1 << 20)
    assert res["expansions"] == X
    assert res["pushes"] + res["dup_skips"] == X * L
    assert res["open_count"] <= 1 << 20
    best = li.unpack(res["best_seq"].cpu().numpy().view(np.uint32)[None, :], L)[0]
    assert orc.energy(best) == res["best_E"]
    assert res["best_E"] <= int(E.min().item())
    oE = res["open_E"].cpu().numpy()
    oS = res["open_seqs"].cpu().numpy().view(np.uint32)
    assert len(oE) == res["open_count"]
    g = li.rng(13)
    idx = g.choice(len(oE), 256, replace=False)
    assert np.array_equal(orc.energy_batch(li.unpack(oS[idx], L)), oE[idx])
    assert oE.min() >= res["best_E"]
