"""Pins of the oracle's Bloom-filter walker (Algorithm 1 with its Bloom filter).

The key is pinned through the SplitMix64 reference vector and linearity, the
filter through the false-positive law of a Bloom filter and the absence of
false negatives, and the walk through a brute-force self-avoiding walk (a
Python set of visited sequences, energies from numpy's correlate) that it must
equal whenever the filter is large enough to make no false positive.  No GPU.
"""
import numpy as np
import pytest

import labs_inputs as li


def np_energy(s):
    s = np.asarray(s, dtype=np.int64)
    c = np.correlate(s, s, mode="full")[len(s):]
    return int(np.dot(c, c))


def _flip(s, a):
    L = len(s)
    u = s.copy()
    u[a - 1] *= -1
    if a != L + 1 - a:
        u[L - a] *= -1
    return u


# ------------------------------------------------------------------ key
def test_walk_key_is_the_zobrist_table_over_the_free_half(orc):
    """h(all -1) = 0 and a skew flip at a changes h by Z_a, Z_a being output a-1 of
    the SplitMix64 stream of the second step's table (pinned by its reference
    vector): together these fix h on every sequence."""
    for L in (5, 37, 101, 501):
        k = (L - 1) // 2
        z = orc.splitmix64_stream(orc.ZOBRIST_STATE, k + 1)
        assert [orc.walk_zobrist(i) for i in range(1, k + 2)] == z
        assert orc.walk_hash(L, -np.ones(L, np.int8)) == 0
        for s in li.random_skew(L, 3, L, 0):
            h = orc.walk_hash(L, s)
            for a in (1, 2, k, k + 1):
                assert orc.walk_hash(L, _flip(s, a)) == h ^ z[a - 1]


def test_walk_key_has_no_collisions_on_small_lengths(orc):
    L = 21
    k = (L - 1) // 2
    seen = set()
    for x in range(1 << (k + 1)):
        s = orc.skew_complete(np.array([1 if (x >> j) & 1 else -1 for j in range(k + 1)], np.int8))
        seen.add(orc.walk_hash(L, s))
    assert len(seen) == 1 << (k + 1)


# ------------------------------------------------------------------ filter
@pytest.mark.parametrize("log2_bits,n_hash,n_ins", [(10, 3, 200), (12, 5, 500), (8, 1, 100)])
def test_bloom_filter_law(orc, log2_bits, n_hash, n_ins):
    """No false negatives; each key sets n_hash distinct bits (odd stride modulo a
    power of two); the set fraction follows 1 - (1 - 1/m)^(n_hash n) and the
    false-positive rate of fresh keys follows (set fraction)^n_hash."""
    g = li.rng(100 + log2_bits)
    m = 1 << log2_bits
    keys = [int(x) for x in g.integers(0, 1 << 63, size=n_ins, dtype=np.int64) * 2 + 1]
    one = orc.Bloom(log2_bits, n_hash)
    one.insert(keys[0])
    assert int(np.unpackbits(one.bits).sum()) == n_hash
    assert len({one.index(keys[0], j) for j in range(n_hash)}) == n_hash
    b = orc.Bloom(log2_bits, n_hash)
    for h in keys:
        b.insert(h)
    assert all(h in b for h in keys)
    frac = np.unpackbits(b.bits).sum() / m
    want = 1 - (1 - 1 / m) ** (n_hash * n_ins)
    assert abs(frac - want) < 5 * np.sqrt(want * (1 - want) / m) + 2 / m
    q = 40000
    fresh = [int(x) for x in g.integers(0, 1 << 63, size=q, dtype=np.int64)]
    fp = sum(h in b for h in fresh) / q
    rate = frac ** n_hash
    assert abs(fp - rate) < 5 * np.sqrt(rate * (1 - rate) / q) + 1e-3, (fp, rate)


# ------------------------------------------------------------------ walk
def _exact_saw(orc, L, p, steps, seed, walker):
    """Algorithm 1 with an exact visited set in place of the filter."""
    s, _ = orc.walker_init(seed, L, p, walker, 0, 0)
    k = (L - 1) // 2
    seen = {s[:k + 1].tobytes()}
    e = np_energy(s)
    traj, moves = [], []
    for t in range(1, steps + 1):
        cands = []
        for a in range(p + 1, k + 2):
            u = _flip(s, a)
            if u[:k + 1].tobytes() not in seen:
                cands.append((np_energy(u) - e, a))
        if not cands:
            break
        d, a = min(cands)
        s = _flip(s, a)
        seen.add(s[:k + 1].tobytes())
        e += d
        traj.append(e)
        moves.append(a)
    pad = steps - len(traj)
    return np.array(traj + [-1] * pad), np.array(moves + [-1] * pad), s, e


@pytest.mark.parametrize("L,p,seed,walkers", [(9, 2, 1, range(4)), (11, 0, 2, range(4)),
                                              (15, 1, 3, range(3)), (21, 2, 4, range(2)),
                                              (27, 0, 5, [7])])
def test_bloom_walk_equals_exact_self_avoiding_walk(orc, L, p, seed, walkers):
    """With 2^24 bits and 8 probes no false positive occurs over <= 4(L+1) keys,
    so the walk is the exact self-avoiding walk; small restricted spaces trap it
    before the step limit, which checks the stop of Algorithm 1."""
    steps = 4 * (L + 1)
    r = orc.walk_bloom(L, p, steps, 24, 8, seed, walkers)
    stopped = 0
    for j, w in enumerate(walkers):
        traj, moves, s, e = _exact_saw(orc, L, p, steps, seed, w)
        assert np.array_equal(r["traj"][j], traj)
        assert np.array_equal(r["moves"][j], moves)
        assert np.array_equal(r["final"][j], s) and r["final_E"][j] == e
        stopped += int(traj[-1] == -1)
    if L <= 11:
        assert stopped > 0


@pytest.mark.parametrize("log2_bits,n_hash", [(6, 1), (7, 2), (9, 3)])
def test_small_filters_never_revisit_and_stop_when_saturated(orc, log2_bits, n_hash):
    """Whatever the filter's size the walk never returns to a sequence (a filter
    has no false negatives); when it stops, every neighbour of the last sequence
    tests as a member of the filter rebuilt from the path."""
    L, p, steps = 37, 0, 4 * 38
    k = (L - 1) // 2
    r = orc.walk_bloom(L, p, steps, log2_bits, n_hash, 11, range(3))
    for j in range(3):
        s, _ = orc.walker_init(11, L, p, j, 0, 0)
        path = [s]
        for a in r["moves"][j]:
            if a < 0:
                break
            path.append(_flip(path[-1], int(a)))
        keys = {x[:k + 1].tobytes() for x in path}
        assert len(keys) == len(path)
        for x, E in zip(path[1:], r["traj"][j]):
            assert np_energy(x) == E
        if r["traj"][j, -1] == -1:
            b = orc.Bloom(log2_bits, n_hash)
            for x in path:
                b.insert(orc.walk_hash(L, x))
            assert all(orc.walk_hash(L, _flip(path[-1], a)) in b for a in range(p + 1, k + 2))
    # a 64-bit filter probed once saturates well before 4(L+1) steps
    if log2_bits == 6:
        assert (r["traj"][:, -1] == -1).all()


def test_bloom_walk_first_move_and_sieve(orc):
    """Before any revisit is possible the walk takes the tabu walker's first move
    (lowest (dE, a) over the whole neighbourhood); sieve emissions are the steps
    at or below e_max."""
    L, p, steps = 37, 2, 120
    em = orc.e_max_for_tau(L, 4)
    rb = orc.walk_bloom(L, p, steps, 15, 6, 9, range(4), e_max=em)
    rt = orc.walk(L, p, 1, 0, 0, 9, range(4))
    assert np.array_equal(rb["moves"][:, 0], rt["moves"][:, 0])
    assert rb["emits"]
    for j in range(4):
        hits = [t + 1 for t in range(steps) if 0 <= rb["traj"][j, t] <= em]
        assert [t for (E, s, w, t) in rb["emits"] if w == j] == hits
    for E, s, w, t in rb["emits"]:
        assert np_energy(s) == E <= em
