"""The CPU baseline walker (oracle/labs_baseline.c: linear-time neighbour
evaluation of Sec. 3, OpenMP over walkers) against the definitional walker of
the oracle (every energy change recomputed from the definition of E): whole
trajectories, final and best energies, equal step by step."""
import numpy as np
import pytest


@pytest.mark.parametrize("L,p,steps,lo,hi,n", [
    (5, 0, 40, 0, 1, 6),          # smallest odd length with a free pair, tenure 0
    (37, 0, 600, 8, 8, 8),        # the exhaustive configuration's walker (tenure 8)
    (63, 4, 300, 4, 9, 6),
    (101, 8, 400, 10, 20, 6),     # L = 101 with p = 8, tenure [L/10, L/5]
    (501, 16, 12, 50, 100, 2),    # the benchmark's length, a few steps
])
def test_baseline_equals_definitional_walker(orc, L, p, steps, lo, hi, n):
    b = orc.baseline_walk(L, p, steps, lo, hi, 7, 3, n, threads=4, want_traj=True)
    o = orc.walk(L, p, steps, lo, hi, 7, range(3, 3 + n))
    assert np.array_equal(b["traj"], o["traj"])
    assert np.array_equal(b["final_E"], o["final_E"])
    assert np.array_equal(b["best_E"], o["best_E"])
    taken = (o["traj"] >= 0).sum()
    assert b["flip_evals"] == taken * ((L - 1) // 2 + 1 - p)


def test_baseline_thread_count_invariance(orc):
    a = orc.baseline_walk(101, 8, 200, 10, 20, 3, 0, 16, threads=1, want_traj=True)
    b = orc.baseline_walk(101, 8, 200, 10, 20, 3, 0, 16, threads=8, want_traj=True)
    assert a["threads"] == 1 and b["threads"] >= 1
    assert np.array_equal(a["traj"], b["traj"])
    # a split of the walker range gives the same walkers
    c = orc.baseline_walk(101, 8, 200, 10, 20, 3, 5, 11, threads=3, want_traj=True)
    assert np.array_equal(a["traj"][5:], c["traj"])
