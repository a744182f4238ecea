"""CPU reference of the first-step walk with a proposer (test infrastructure
only; see the package header for who may import it).

The walk is the plain first step (skew flips of the free positions p+1..k+1,
Eq. (2)/(3); best admissible neighbour with a tabu tenure, Alg. 1 as read for
the plain walker) except that at steps t with (t-1) mod fallback_every != 0 only
a proposed subset of the admissible positions is evaluated.  Every evaluated
energy is recomputed from the definition (oracle C library); the move is the
evaluated position of least dE, ties to the lower position.  The network that
proposes subsets in the GPU library is not part of the paper; this module
only fixes what a step does with a given subset, and the random proposer used
as an ablation.
"""
from __future__ import annotations

import numpy as np

from . import energy, flip_skew, lib, walker_init, walker_key

GAMMA = 0x9E3779B97F4A7C15
M64 = (1 << 64) - 1


def sm64_at(key: int, i: int) -> int:
    """Output i (from 0) of the SplitMix64 stream whose state starts at key."""
    return int(lib().or_mix64((key + (i + 1) * GAMMA) & M64))


def random_scores(prop_seed: int, L: int, walker: int, t: int, positions) -> list:
    """The random proposer's score of each position at step t: the high 32 bits of
    draw (t-1)(k+1) + (a-1) of the stream keyed like a walker with prop_seed."""
    k = (L - 1) // 2
    key = walker_key(prop_seed, L, walker)
    return [sm64_at(key, (t - 1) * (k + 1) + (a - 1)) >> 32 for a in positions]


def top_by_score(positions, scores, m: int) -> list:
    """The m positions of largest score (ties: lower position), best first."""
    order = sorted(zip(positions, scores), key=lambda x: (-x[1], x[0]))
    return [a for a, _ in order[:m]]


def proposal_walk(L: int, p: int, steps: int, tenure_lo: int, tenure_hi: int, seed: int,
                  walker: int, fallback_every: int, propose, e_max: int = -1):
    """Run one walker.  propose(t, s, admissible) returns the positions to
    evaluate at a non-full step.  Returns traj/moves (-1 after a halt), the
    candidate lists (None on full steps), the states before each move, the
    admissible sets, the final state, best E/step and the first step with
    E <= e_max (-1 if none)."""
    k = (L - 1) // 2
    s, tenure = walker_init(seed, L, p, walker, tenure_lo, tenure_hi)
    E = energy(s)
    tabu = {a: 0 for a in range(p + 1, k + 2)}
    out = dict(traj=[], moves=[], cands=[], states=[], admissible=[], best_E=E, best_step=0,
               hit_step=-1, tenure=tenure)
    halted = False
    for t in range(1, steps + 1):
        if halted:
            out["traj"].append(-1)
            out["moves"].append(-1)
            out["cands"].append(None)
            continue
        adm = [a for a in range(p + 1, k + 2) if tabu[a] < t]
        full = (t - 1) % fallback_every == 0
        cands = list(adm) if full else list(propose(t, s, adm))
        assert set(cands) <= set(adm) and len(set(cands)) == len(cands)
        out["states"].append(s.copy())
        out["admissible"].append(adm)
        out["cands"].append(None if full else cands)
        if not cands:
            halted = True
            out["traj"].append(-1)
            out["moves"].append(-1)
            continue
        dE = {a: energy(flip_skew(s, a)) - E for a in cands}
        a = min(cands, key=lambda x: (dE[x], x))
        s = flip_skew(s, a)
        E += dE[a]
        tabu[a] = t + tenure
        out["traj"].append(E)
        out["moves"].append(a)
        if E < out["best_E"]:
            out["best_E"], out["best_step"] = E, t
        if e_max >= 0 and E <= e_max and out["hit_step"] < 0:
            out["hit_step"] = t
    out["final"] = s
    out["final_E"] = E
    return out


def random_proposer(prop_seed: int, L: int, walker: int, m: int):
    def propose(t, s, adm):
        return top_by_score(adm, random_scores(prop_seed, L, walker, t, adm), m)
    return propose
