"""Pins of the proposer walk reference: with every step a full scan, or with
subsets covering every admissible position, it is the plain first-step walker
(the oracle's C implementation); the random proposer's counter-form draws equal
the sequential SplitMix64 stream."""
import numpy as np

from oracle import learned as ol


def test_full_scan_every_step_is_the_plain_walker(orc):
    L, p, steps, lo, hi, seed = 37, 3, 120, 3, 6, 11
    for w in (0, 5):
        ref = orc.walk(L, p, steps, lo, hi, seed, [w])
        got = ol.proposal_walk(L, p, steps, lo, hi, seed, w, 1, propose=None)
        assert np.array_equal(np.array(got["traj"]), ref["traj"][0])
        assert np.array_equal(np.array(got["moves"]), ref["moves"][0])


def test_covering_subsets_are_the_plain_walker(orc):
    L, p, steps, lo, hi, seed = 45, 4, 90, 2, 5, 3
    k = (L - 1) // 2
    ref = orc.walk(L, p, steps, lo, hi, seed, [2])
    got = ol.proposal_walk(L, p, steps, lo, hi, seed, 2, 7,
                           ol.random_proposer(9, L, 2, k + 1 - p))
    assert np.array_equal(np.array(got["traj"]), ref["traj"][0])


def test_narrow_subsets_follow_their_candidates(orc):
    L, p, steps, lo, hi, seed = 37, 0, 60, 3, 6, 4
    got = ol.proposal_walk(L, p, steps, lo, hi, seed, 1, 5, ol.random_proposer(7, L, 1, 3))
    for t, (c, s, a, e) in enumerate(zip(got["cands"], got["states"], got["moves"], got["traj"]), 1):
        if c is None:
            assert (t - 1) % 5 == 0
            continue
        assert len(c) == min(3, len(got["admissible"][t - 1]))
        dE = [orc.energy(orc.flip_skew(s, x)) - orc.energy(s) for x in c]
        best = min(zip(dE, c))
        assert a == best[1] and e == orc.energy(s) + best[0]


def test_counter_form_matches_the_stream(orc):
    key = orc.walker_key(5, 37, 3)
    stream = orc.splitmix64_stream(key, 40)
    assert [ol.sm64_at(key, i) for i in range(40)] == stream
