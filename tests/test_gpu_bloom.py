"""GPU parity of the first step with the Bloom filter of Algorithm 1
(labs_walk_step1_bloom) against the oracle's Bloom walker, bit for bit:
trajectories, final and best sequences, flip-evaluation counts, sieve pools,
filters small enough to give false positives and to saturate (the walk stops),
segment boundaries, walker-range splits and the largest length."""
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


def _host_seqs(t, L):
    return li.unpack(t.cpu().numpy().view(np.uint32), L)


def _compare(lb, orc, L, p, steps, log2_bits, n_hash, seed, n, begin=0):
    r = lb.walk_step1(L, p, steps, 0, 0, seed, n, walker_begin=begin, want_traj=True,
                      bloom=(log2_bits, n_hash))
    steps_eff = steps if steps else 4 * (L + 1)
    o = orc.walk_bloom(L, p, steps_eff, log2_bits, n_hash, seed, range(begin, begin + n))
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
    assert int(r.flip_evals.item()) == int(((steps_eff - halted) * (k + 1 - p)).sum())
    return r, o


@pytest.mark.parametrize("L,p,steps,log2_bits,n_hash,n", [
    (5, 0, 40, 6, 1, 8),          # smallest length: the restricted space traps every walker
    (9, 2, 0, 10, 2, 6),          # default T_i = 4(L+1)
    (37, 0, 152, 15, 6, 16),
    (37, 0, 152, 6, 1, 8),        # 64-bit filter: saturates, every walker stops early
    (63, 3, 300, 8, 3, 8),        # small filter: false positives change the path
    (101, 8, 0, 12, 4, 12),       # the second configuration's shape, T_i steps
    (131, 1, 400, 16, 8, 4),      # two chunks of 64 lags
    (301, 12, 120, 18, 16, 2),    # the largest filter and probe count
])
def test_bloom_walk_shapes(lb, orc, L, p, steps, log2_bits, n_hash, n):
    r, o = _compare(lb, orc, L, p, steps, log2_bits, n_hash, 5 + L, n)
    if log2_bits == 6 and L == 37:
        assert (o["traj"][:, -1] == -1).all()


def test_bloom_walk_L501_shape(lb, orc):
    _compare(lb, orc, 501, 16, 40, 15, 8, 4, 3)


def test_bloom_walk_largest_length(lb, orc):
    _compare(lb, orc, 639, 0, 24, 12, 5, 6, 2)


def test_bloom_walk_across_segments(lb, orc):
    """More steps than one launch segment: the filter and key persist in the
    workspace between launches."""
    _compare(lb, orc, 37, 1, 4500, 18, 8, 21, 3)


def test_bloom_walk_sharding_invariance(lb):
    import torch
    L, p, steps = 101, 8, 300
    a = lb.walk_step1(L, p, steps, 0, 0, 99, 40, want_traj=True, bloom=(10, 3))
    b1 = lb.walk_step1(L, p, steps, 0, 0, 99, 13, walker_begin=0, want_traj=True, bloom=(10, 3))
    b2 = lb.walk_step1(L, p, steps, 0, 0, 99, 27, walker_begin=13, want_traj=True, bloom=(10, 3))
    assert torch.equal(a.traj_E, torch.cat([b1.traj_E, b2.traj_E]))
    assert torch.equal(a.final_seqs, torch.cat([b1.final_seqs, b2.final_seqs]))


def test_bloom_pool_sieve(lb, orc):
    """Sieve into the pool over several segments (the pool path starts with short
    segments), including a capacity cut, against the oracle's emissions."""
    L, p, steps, n = 101, 8, 600, 16
    em = orc.e_max_for_tau(L, 22, 5)
    o = orc.walk_bloom(L, p, steps, 11, 4, 3, range(n), e_max=em)
    for cap in (1 << 20, 40):
        pool = lb.PoolBuffers.empty(L, cap)
        r = lb.walk_step1(L, p, steps, 0, 0, 3, n, e_max=em, pool=pool, want_traj=True,
                          bloom=(11, 4))
        assert np.array_equal(r.traj_E.cpu().numpy(), o["traj"])
        ref, dropped = orc.pool(o["emits"], cap)
        cnt = int(pool.count.item())
        assert len(ref) >= 20 and cnt == len(ref)
        assert int(pool.dropped.item()) == dropped
        assert [int(e) for e in pool.E[:cnt].cpu().numpy()] == [e for e, _ in ref]
        assert [orc.seq_key(s) for s in _host_seqs(pool.seqs[:cnt], L)] == [k for _, k in ref]


def test_bloom_pool_walker_best(lb, orc):
    L, p, steps, n = 63, 4, 200, 24
    pool = lb.PoolBuffers.empty(L, 1000)
    lb.walk_step1(L, p, steps, 0, 0, 11, n, e_max=-1, pool=pool, pool_walker_best=True,
                  bloom=(9, 3))
    o = orc.walk_bloom(L, p, steps, 9, 3, 11, range(n))
    ref, _ = orc.pool([(int(o["best_E"][j]), o["best"][j]) for j in range(n)], 1000)
    cnt = int(pool.count.item())
    assert cnt == len(ref)
    assert [orc.seq_key(s) for s in _host_seqs(pool.seqs[:cnt], L)] == [k for _, k in ref]


def test_bloom_invalid_args(lb):
    with pytest.raises(lb.LabsError):
        lb.walk_step1(37, 0, 10, 1, 1, 1, 4, bloom=(12, 4))     # a tenure with the filter
    with pytest.raises(lb.LabsError):
        lb.walk_step1(37, 0, 10, 0, 0, 1, 4, bloom=(5, 4))      # filter below 2^6 bits
    with pytest.raises(lb.LabsError):
        lb.walk_step1(37, 0, 10, 0, 0, 1, 4, bloom=(19, 4))     # above 2^18 bits
    with pytest.raises(lb.LabsError):
        lb.walk_step1(37, 0, 10, 0, 0, 1, 4, bloom=(12, 0))     # no probe
    with pytest.raises(lb.LabsError):
        lb.walk_step1(37, 0, 10, 0, 0, 1, 4, bloom=(12, 17))
