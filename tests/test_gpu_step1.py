"""GPU parity: energies, flip deltas, the first-step walker and the pool,
through the C ABI, against the CPU oracle, bit for bit."""
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


def _host_seqs(t, L):
    return li.unpack(t.cpu().numpy().view(np.uint32), L)


# ------------------------------------------------------------------ energies
@pytest.mark.parametrize("L", [1, 2, 3, 5, 31, 32, 33, 37, 64, 101, 255, 501, 527, 1023])
def test_energy_parity(lb, orc, L):
    S = li.random_pm1(100 + L, 40, L)
    edge = np.stack([np.ones(L, np.int8), np.array([(-1) ** i for i in range(L)], np.int8),
                     -np.ones(L, np.int8)])
    S = np.concatenate([S, edge])
    E, C = lb.energy(L, _dev(li.pack(S)), want_c=True)
    Eo, Co = orc.energy_batch(S, with_c=True)
    assert np.array_equal(E.cpu().numpy(), Eo)
    assert np.array_equal(C.cpu().numpy(), Co)


def test_energy_empty(lb):
    import torch
    E = lb.energy(37, torch.zeros((0, 2), dtype=torch.int32, device="cuda"))
    assert E.numel() == 0


@pytest.mark.parametrize("L", [2, 3, 7, 37, 64, 101, 501])
def test_flip_deltas_single(lb, orc, L):
    S = li.random_pm1(7 * L, 12, L)
    dE = lb.flip_deltas(L, _dev(li.pack(S))).cpu().numpy()
    for j in range(len(S)):
        assert np.array_equal(dE[j], orc.deltas_single(S[j]))


@pytest.mark.parametrize("L,p", [(3, 0), (5, 1), (37, 0), (101, 8), (501, 16), (527, 16)])
def test_flip_deltas_skew(lb, orc, L, p):
    S = np.concatenate([li.random_skew(L, 6, L, p), li.random_pm1(L + 1, 2, L)])
    dE = lb.flip_deltas(L, _dev(li.pack(S)), skew=True, p=p).cpu().numpy()
    for j in range(len(S)):
        assert np.array_equal(dE[j], orc.deltas_skew(S[j], p))


def test_cfg1_exhaustive(lb, orc):
    """All 2^19 skew-symmetric sequences at L = 37: min E and its argmin set."""
    L = 37
    S = li.skew_all(L)
    E = lb.energy(L, _dev(li.pack(S))).cpu().numpy()
    m, allE = orc.skew_exhaustive(L, want_all=True)
    assert E.min() == m
    assert np.array_equal(np.nonzero(E == E.min())[0], np.nonzero(allE == m)[0])
    assert np.array_equal(E, allE)


# ------------------------------------------------------------------ walker
def _compare_walk(lb, orc, L, p, steps, lo, hi, seed, n, begin=0):
    r = lb.walk_step1(L, p, steps, lo, hi, seed, n, walker_begin=begin, want_traj=True)
    o = orc.walk(L, p, steps, lo, hi, seed, range(begin, begin + n))
    traj = r.traj_E.cpu().numpy()
    for j in range(n):
        assert np.array_equal(traj[j], o["traj"][j]), "walker %d" % (begin + j)
    assert np.array_equal(_host_seqs(r.final_seqs, L), o["final"])
    assert np.array_equal(r.final_E.cpu().numpy(), o["final_E"])
    assert np.array_equal(r.best_E.cpu().numpy(), o["best_E"])
    assert np.array_equal(r.best_step.cpu().numpy(), o["best_step"])
    assert np.array_equal(_host_seqs(r.best_seqs, L), o["best"])
    k = (L - 1) // 2
    halted = (o["traj"] < 0).sum(axis=1)
    assert int(r.flip_evals.item()) == int(((steps - halted) * (k + 1 - p)).sum())
    return r


def test_walk_cfg1_trajectories(lb, orc):
    """The first configuration: L = 37, p = 0, tenure 8, 256 walkers x 4096 steps."""
    _compare_walk(lb, orc, 37, 0, 4096, 8, 8, 1, 256)


@pytest.mark.parametrize("L,p,steps,lo,hi,n", [
    (5, 0, 40, 0, 2, 8),          # smallest length, zero tenure allowed
    (7, 2, 30, 0, 1, 4),
    (13, 0, 200, 2, 2, 16),
    (63, 3, 300, 4, 9, 8),        # k = 31: one full even-lag word
    (65, 0, 300, 5, 11, 8),       # k = 32: free count 33, second slot partly used
    (101, 8, 600, 10, 20, 12),    # the second configuration's shape
    (131, 1, 400, 13, 26, 4),     # k = 65: two chunks of 64 lags, 65 free positions
    (301, 12, 60, 30, 60, 2),     # third configuration's range
    (301, 120, 40, 3, 6, 2),      # long prefix: 31 free positions in the smallest slot group
    (385, 12, 30, 38, 77, 2),     # k = 192: six even-lag words, three slot groups
    (387, 12, 30, 38, 77, 2),     # k = 193: one lag into a seventh word, still three groups
    (389, 12, 30, 38, 77, 2),     # k = 194: two lags in the seventh word, backward word in use
    (133, 4, 200, 13, 26, 4),     # k = 66: three words, two lags in the last, backward word in use
    (141, 2, 200, 14, 28, 4),     # k = 70: six lags in the last word
    (143, 2, 200, 14, 28, 4),     # k = 71: seven lags in the last word
    (259, 8, 100, 25, 50, 2),     # k = 129: five words, one lag in the last
    (527, 16, 20, 52, 105, 2),    # k = 263: nine words, four slot groups
    (409, 12, 30, 40, 81, 2),     # k = 204: seven words, four slot groups (the half tile, held to four waves)
    (449, 12, 30, 44, 89, 2),     # k = 224: seven full words, four slot groups
])
def test_walk_shapes(lb, orc, L, p, steps, lo, hi, n):
    _compare_walk(lb, orc, L, p, steps, lo, hi, 7 + L, n)


def test_walk_L501_cfg4_shape(lb, orc):
    _compare_walk(lb, orc, 501, 16, 40, 50, 100, 4, 3)


def test_walk_long_no_pool(lb, orc):
    """9,000 steps without a pool run as three launches of up to 4,096 steps; the
    whole trajectories, final and best sequences equal the oracle's."""
    L, p, steps, n = 37, 0, 9000, 12
    r = lb.walk_step1(L, p, steps, 8, 8, 21, n, want_traj=True)
    o = orc.walk(L, p, steps, 8, 8, 21, range(n))
    assert np.array_equal(r.traj_E.cpu().numpy(), o["traj"])
    assert np.array_equal(_host_seqs(r.final_seqs, L), o["final"])
    assert np.array_equal(_host_seqs(r.best_seqs, L), o["best"])
    assert np.array_equal(r.best_step.cpu().numpy(), o["best_step"])


def test_walk_L501_across_pool_segments(lb, orc):
    """L = 501 with the pool on: the walk runs in segments of 256, 512, ... steps
    with a compaction between them.  Two walkers' 1,200-step trajectories equal the
    oracle's linear-time walker (pinned to the definitional one in the CPU suite),
    and the pool holds exactly the distinct sequences the walkers reached at
    E <= e_max, each at an energy their trajectories show."""
    L, p, steps, n = 501, 16, 1200, 2
    em = orc.e_max_for_tau(L, 4, 1)
    pool = lb.PoolBuffers.empty(L, 1 << 16)
    r = lb.walk_step1(L, p, steps, 50, 100, 4, n, e_max=em, pool=pool, want_traj=True)
    b = orc.baseline_walk(L, p, steps, 50, 100, 4, 0, n, threads=2, want_traj=True)
    traj = r.traj_E.cpu().numpy()
    assert np.array_equal(traj, b["traj"])
    assert np.array_equal(r.final_E.cpu().numpy(), b["final_E"])
    assert np.array_equal(r.best_E.cpu().numpy(), b["best_E"])
    cnt = int(pool.count.item())
    assert cnt > 0 and int(pool.dropped.item()) == 0
    pw, ps, pe = (pool.walker[:cnt].cpu().numpy(), pool.step[:cnt].cpu().numpy(),
                  pool.E[:cnt].cpu().numpy())
    assert np.array_equal(traj[pw, ps - 1], pe)
    assert np.array_equal(orc.energy_batch(_host_seqs(pool.seqs[:cnt], L)), pe)
    # every step at or below e_max was offered; distinct sequences, so at most that many
    assert cnt <= int((traj <= em).sum()) and pe.max() <= em


def test_walk_halts(lb, orc):
    """Tenure = free count - 1 with p = k-1 leaves 2 free positions: the walker
    alternates; tenure equal to the free count is rejected, so check the edge
    where every move becomes tabu is unreachable and the trajectory has no -1."""
    _compare_walk(lb, orc, 9, 3, 20, 1, 1, 5, 3)


def test_walk_sharding_invariance(lb, orc):
    """Any split of the walker range gives the same per-walker results."""
    L, p, steps = 101, 8, 300
    a = lb.walk_step1(L, p, steps, 10, 20, 99, 64, want_traj=True)
    b1 = lb.walk_step1(L, p, steps, 10, 20, 99, 21, walker_begin=0, want_traj=True)
    b2 = lb.walk_step1(L, p, steps, 10, 20, 99, 43, walker_begin=21, want_traj=True)
    import torch
    assert torch.equal(a.traj_E, torch.cat([b1.traj_E, b2.traj_E]))
    assert torch.equal(a.final_seqs, torch.cat([b1.final_seqs, b2.final_seqs]))


def test_walk_default_steps(lb):
    r = lb.walk_step1(37, 0, 0, 8, 8, 1, 2, want_traj=True)
    assert r.traj_E.shape[1] == 4 * 38


def test_walk_invalid_args(lb):
    with pytest.raises(lb.LabsError):
        lb.walk_step1(36, 0, 10, 1, 1, 1, 4)          # even L
    with pytest.raises(lb.LabsError):
        lb.walk_step1(37, 0, 10, 19, 19, 1, 4)        # tenure >= free count
    with pytest.raises(lb.LabsError):
        lb.walk_step1(37, 18, 10, 0, 0, 1, 4)         # p > k-1


# ------------------------------------------------------------------ pool
def test_pool_sieve_cfg2_shape(lb, orc):
    """Second configuration's shape (L = 101, p = 8) at reduced size; the
    threshold is lowered to F >= 4.4 so that 500 steps produce offers."""
    L, p, steps, n = 101, 8, 500, 24
    em = orc.e_max_for_tau(L, 22, 5)
    for cap in (1 << 20, 50):
        pool = lb.PoolBuffers.empty(L, cap)
        r = lb.walk_step1(L, p, steps, 10, 20, 2, n, e_max=em, pool=pool, want_traj=True)
        o = orc.walk(L, p, steps, 10, 20, 2, range(n), e_max=em)
        assert np.array_equal(r.traj_E.cpu().numpy(), o["traj"])
        ref, dropped = orc.pool(o["emits"], cap)
        cnt = int(pool.count.item())
        assert len(ref) >= 20
        assert cnt == len(ref)
        assert int(pool.dropped.item()) == dropped
        got_E = pool.E[:cnt].cpu().numpy()
        got_S = _host_seqs(pool.seqs[:cnt], L)
        assert [int(e) for e in got_E] == [e for e, _ in ref]
        assert [orc.seq_key(s) for s in got_S] == [k for _, k in ref]
        # walker/step of the earliest offer of each sequence
        first = {}
        for E, s, w, t in o["emits"]:
            key = orc.seq_key(s)
            if key not in first or (w, t) < first[key]:
                first[key] = (w, t)
        gw = pool.walker[:cnt].cpu().numpy()
        gt = pool.step[:cnt].cpu().numpy()
        for i, (_, key) in enumerate(ref):
            assert (int(gw[i]), int(gt[i])) == first[key]


def test_pool_dropped_repeats_across_segments(lb, orc):
    """At L = 21 the walkers revisit sequences often, so the same sequence is
    offered in several compaction segments (the pool path starts with 256-step
    segments) and is cut each time the capacity is reached: `dropped` counts it
    once.  A second call on the same pool counts the distinct sequences of (its
    previous contents) U (the new offers) beyond the capacity."""
    L, p, steps, n, cap = 21, 0, 3000, 48, 30
    em = orc.e_max_for_tau(L, 3, 1)
    pool = lb.PoolBuffers.empty(L, cap)
    lb.walk_step1(L, p, steps, 1, 3, 7, n, e_max=em, pool=pool)
    o = orc.walk(L, p, steps, 1, 3, 7, range(n), e_max=em, want_traj=False)
    ref, dropped = orc.pool(o["emits"], cap)
    assert len(o["emits"]) > 2 * (len(ref) + dropped)      # the case has many repeats
    assert dropped > 0
    cnt = int(pool.count.item())
    assert cnt == cap
    assert int(pool.dropped.item()) == dropped
    assert [orc.seq_key(s) for s in _host_seqs(pool.seqs[:cnt], L)] == [k for _, k in ref]
    # a second call adds to the same pool
    lb.walk_step1(L, p, 700, 1, 3, 8, n, e_max=em, pool=pool)
    o2 = orc.walk(L, p, 700, 1, 3, 8, range(n), e_max=em, want_traj=False)
    prev = [(E, orc.key_seq(k, L)) for E, k in ref]
    ref2, dropped2 = orc.pool(prev + o2["emits"], cap)
    assert int(pool.dropped.item()) == dropped + dropped2
    assert [orc.seq_key(s) for s in _host_seqs(pool.seqs[:cap], L)] == [k for _, k in ref2]


def test_pool_topk_edges(lb, orc):
    """k beyond the pool's distinct sequences returns all of them, in order; an
    empty pool returns none."""
    L, p, steps, n = 63, 4, 200, 40
    pool = lb.PoolBuffers.empty(L, 1000)
    lb.walk_step1(L, p, steps, 4, 9, 11, n, e_max=-1, pool=pool, pool_walker_best=True)
    o = orc.walk(L, p, steps, 4, 9, 11, range(n))
    ref, _ = orc.pool([(int(o["best_E"][j]), o["best"][j]) for j in range(n)], 1000)
    s, E = lb.pool_topk(pool, len(ref) + 25)
    assert [int(e) for e in E.cpu().numpy()] == [e for e, _ in ref]
    assert [orc.seq_key(x) for x in _host_seqs(s, L)] == [k for _, k in ref]
    s, E = lb.pool_topk(lb.PoolBuffers.empty(L, 16), 4)
    assert len(E) == 0 and len(s) == 0


def test_pool_topk_and_walker_best(lb, orc):
    L, p, steps, n = 63, 4, 200, 40
    pool = lb.PoolBuffers.empty(L, 1000)
    lb.walk_step1(L, p, steps, 4, 9, 11, n, e_max=-1, pool=pool, pool_walker_best=True)
    o = orc.walk(L, p, steps, 4, 9, 11, range(n))
    entries = [(int(o["best_E"][j]), o["best"][j]) for j in range(n)]
    ref, _ = orc.pool(entries, 1000)
    assert int(pool.count.item()) == len(ref)
    s, E = lb.pool_topk(pool, 10)
    assert [int(e) for e in E.cpu().numpy()] == [e for e, _ in ref[:10]]
    assert [orc.seq_key(x) for x in _host_seqs(s, L)] == [k for _, k in ref[:10]]
