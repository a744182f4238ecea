"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself: values the
paper prints (tests/golden), textbook sequences and optima from the literature,
numpy's correlate (a library autocorrelation), closed identities and
invariants, and brute force on tiny inputs.  No GPU is involved.
"""
import os

import numpy as np
import pytest

import labs_inputs as li

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _rows(name):
    out = []
    for line in open(os.path.join(GOLD, name)):
        line = line.split("#")[0].strip()
        if line:
            out.append(line.split())
    return out


def np_autocorr(s):
    """C_1..C_{L-1} from numpy's correlate (library routine)."""
    s = np.asarray(s, dtype=np.int64)
    full = np.correlate(s, s, mode="full")
    return full[len(s):]


def np_energy(s):
    c = np_autocorr(s)
    return int(np.dot(c, c))


# ------------------------------------------------------------------ energy
def test_energy_matches_library_correlate(orc):
    for L in (1, 2, 3, 7, 37, 101, 256, 501):
        S = li.random_pm1(10 + L, 6, L)
        E, C = orc.energy_batch(S, with_c=True)
        for j in range(len(S)):
            assert np.array_equal(C[j], np_autocorr(S[j]))
            assert E[j] == np_energy(S[j])


def test_energy_closed_identities(orc):
    for L in (5, 20, 101, 333):
        for s in li.random_pm1(L, 5, L):
            E, C = orc.energy(s, with_c=True)
            ks = np.arange(1, L)
            # C_k has the parity of L - k (it sums L - k terms of +-1)
            assert np.all((C - (L - ks)) % 2 == 0)
            # sum_k C_k = ((sum s)^2 - L) / 2
            assert C.sum() == (int(s.sum()) ** 2 - L) // 2
            # C_k + C_{L-k} == L (mod 4)
            for k in range(1, L):
                assert (C[k - 1] + C[L - k - 1] - L) % 4 == 0
            assert E == int((C * C).sum())


def test_energy_invariants(orc):
    for L in (9, 37, 101):
        for s in li.random_pm1(3 * L, 4, L):
            e = orc.energy(s)
            alt = s * np.array([(-1) ** i for i in range(L)], dtype=np.int8)
            assert orc.energy(-s) == e
            assert orc.energy(s[::-1].copy()) == e
            assert orc.energy(alt) == e


def test_barker_sequences(orc):
    for L, txt in _rows("barker.txt"):
        L = int(L)
        s = np.array([1 if c == "+" else -1 for c in txt], dtype=np.int8)
        assert len(s) == L
        C = orc.energy(s, with_c=True)[1]
        assert np.all(np.abs(C) <= 1)
        assert orc.energy(s) == (L - 1) // 2
        assert orc.is_skew(s)


def test_optimal_energies_exhaustive(orc):
    for L, e in _rows("labs_optimal_energies.txt"):
        L, e = int(L), int(e)
        if L > 16:
            continue
        m, cnt = orc.exhaustive_min(L)
        assert m == e, L
        # the optimum set is closed under negation, reversal and alternation
        assert cnt % 4 == 0


def test_legendre_construction_values(orc):
    """Sec. 4.1 table: the best Legendre construction's F at L = 450..526."""
    for L, n, o, F in _rows("legendre_construct.txt"):
        L, n, o = int(L), int(n), int(o)
        s = li.legendre_rotated(n, o, L)
        E = orc.energy(s)
        assert E == np_energy(s)
        assert "%.4f" % orc.merit_factor(L, E) == F


def test_legendre_sweep_best_is_the_printed_construction(orc):
    """Sec. 4.1 table: over the sweep (primes with appended fraction <= 0.09,
    rotations 0.18..0.26 of n) the best construction's F is the printed one at all
    four lengths, and it is the tabulated (n, o) pair; Euler's criterion agrees
    with the squaring table of the input generator."""
    for L, n, o, F in _rows("legendre_construct.txt"):
        L, n, o = int(L), int(n), int(o)
        sw = orc.legendre_sweep(L)
        assert len(sw) > 40
        bn, bo, bE = min(sw, key=lambda x: (x[2], x[0], x[1]))
        assert "%.4f" % orc.merit_factor(L, bE) == F
        assert (bn, bo) == (n, o)
        assert np.array_equal(orc.legendre_chi(n), li.legendre_symbol_table(n))
        assert np.array_equal(orc.legendre_sequence(n, o, L), li.legendre_rotated(n, o, L))
    # the pair enumeration's boundaries are inclusive and exact
    prs = orc.legendre_pairs(53, t_lo=0, t_hi=10000, r_lo=0, r_hi=10000)
    assert (53, 0) in prs and (53, 52) in prs and (29, 28) in prs and (23, 0) not in prs
    assert all(orc._is_prime(n) for n, _ in prs)


def test_length_operators(orc):
    """The end operators: removing after appending gives the sequence back; the
    first-element operators are the last-element ones under reversal (which keeps
    E); a removal changes C_k by exactly the dropped products (numpy correlate)."""
    for L in (2, 3, 8, 37, 500, 501):
        for s in li.random_pm1(40 + L, 3, L):
            minus, plus = orc.length_operators(s)
            assert minus.shape == (2, L - 1) and plus.shape == (4, L + 1)
            for q in range(4):
                m2, _ = orc.length_operators(plus[q])
                assert np.array_equal(m2[0 if q < 2 else 1], s)
                assert plus[q][0 if q < 2 else L] == (1 if q % 2 == 0 else -1)
            rm, rp = orc.length_operators(s[::-1])
            assert np.array_equal(minus[0], rm[1][::-1]) and np.array_equal(plus[0], rp[2][::-1])
            assert orc.energy(minus[0]) == orc.energy(rm[1])
            c_full = np_autocorr(s)
            c_last = np_autocorr(minus[1])
            for k in range(1, L - 1):
                assert c_last[k - 1] == c_full[k - 1] - int(s[L - 1 - k]) * int(s[L - 1])


def test_merit_factor_printed_values(orc):
    """Eq. (1) with the F values printed in Sec. 4: exactly one integer energy
    rounds to each printed F."""
    for L, F in _rows("paper_merit_factors.txt"):
        L = int(L)
        hits = [E for E in range(1, L * L) if "%.4f" % orc.merit_factor(L, E) == F]
        assert len(hits) == 1
        assert hits[0] == round(L * L / (2 * float(F)))


def test_e_max_threshold(orc):
    for L in (37, 101, 451, 475, 501, 527):
        for num, den in ((6, 1), (8, 1), (13, 2), (15, 2)):
            em = orc.e_max_for_tau(L, num, den)
            assert L * L * den >= 2 * num * em          # F(em) >= tau
            assert L * L * den < 2 * num * (em + 1)     # F(em + 1) < tau


# ------------------------------------------------------------------ skew symmetry
def test_skew_complete_eq2(orc):
    for L in (3, 5, 37, 101, 501):
        k = (L - 1) // 2
        h = li.random_pm1(L, 1, k + 1)[0]
        s = orc.skew_complete(h)
        for i in range(1, k + 1):
            assert s[k + i] == (-1) ** i * s[k - i]
        assert orc.is_skew(s)
        assert np.array_equal(s, li.skew_from_half(h))


def test_skew_odd_lags_vanish(orc):
    """Sec. 1: skew-symmetry makes every odd-lag C_k zero."""
    for L in (5, 37, 101, 301, 501):
        for s in li.random_skew(L, 4, L):
            C = orc.energy(s, with_c=True)[1]
            assert np.all(C[0::2] == 0)      # k = 1, 3, 5, ...


def test_skew_flip_stays_skew(orc):
    L = 37
    k = 18
    s = li.random_skew(5, 1, L)[0]
    for a in range(1, k + 2):
        t = orc.flip_skew(s, a)
        assert orc.is_skew(t)
        diff = set(np.nonzero(t != s)[0] + 1)
        assert diff == ({a, L + 1 - a} if a <= k else {a})


def test_deltas_match_library_energy(orc):
    for L, p in ((13, 0), (37, 0), (101, 8)):
        k = (L - 1) // 2
        s = li.random_skew(L + p, 1, L, p)[0]
        e0 = np_energy(s)
        ds = orc.deltas_skew(s, p)
        for a in range(p + 1, k + 2):
            t = s.copy()
            t[a - 1] *= -1
            if a != L + 1 - a:
                t[L - a] *= -1
            assert ds[a - p - 1] == np_energy(t) - e0
        d1 = orc.deltas_single(s)
        for i in range(1, L + 1):
            t = s.copy()
            t[i - 1] *= -1
            assert d1[i - 1] == np_energy(t) - e0


def test_skew_minimum_bound_and_barker_lengths(orc):
    """For odd L every even-lag C_k is odd, so E >= k = (L-1)/2 with equality
    exactly at the Barker lengths; brute force over the skew space."""
    for L in (3, 5, 7, 9, 11, 13, 15, 17):
        m = orc.skew_exhaustive(L)
        assert m >= (L - 1) // 2
        assert (m == (L - 1) // 2) == (L in (3, 5, 7, 11, 13))


def test_skew_exhaustive_agrees_with_global_where_skew_is_optimal(orc):
    """At L = 11 and 13 the optimum (a Barker sequence) is skew-symmetric, so the
    skew enumeration reaches the global optimum of the literature table."""
    table = {int(a): int(b) for a, b in _rows("labs_optimal_energies.txt")}
    for L in (11, 13):
        assert orc.skew_exhaustive(L) == table[L]


def test_skew_exhaustive_L37_orbit(orc):
    """The first configuration's exhaustive skew search (L = 37, 2^19 patterns):
    the argmin set is closed under negation and alternation."""
    L = 37
    m, allE = orc.skew_exhaustive(L, want_all=True)
    assert m == allE.min()
    arg = np.nonzero(allE == m)[0]
    S = li.skew_all(L)[arg]
    keys = {tuple(x) for x in S}
    alt = np.array([(-1) ** i for i in range(L)], dtype=np.int8)
    for s in S:
        assert tuple(-s) in keys
        assert tuple(s * alt) in keys
        assert np_energy(s) == m
    assert len(arg) % 2 == 0


# ------------------------------------------------------------------ generator
def test_splitmix64_reference_vector(orc):
    vals = [int(r[0]) for r in _rows("splitmix64.txt")]
    assert orc.splitmix64_stream(vals[0], 5) == vals[1:]


def test_walker_init_layout(orc):
    for L, p, lo, hi in ((37, 0, 8, 8), (101, 8, 10, 20), (501, 16, 50, 100)):
        tens = []
        ones = 0
        for w in range(64):
            s, ten = orc.walker_init(7, L, p, w, lo, hi)
            assert orc.is_skew(s)
            if p >= 1:
                assert s[0] == 1
            assert lo <= ten <= hi
            tens.append(ten)
            ones += int((s[: (L + 1) // 2] > 0).sum())
        # draws are roughly balanced
        assert 0.35 < ones / (64 * (L + 1) / 2) < 0.65
        if hi > lo:
            assert len(set(tens)) > 1


# ------------------------------------------------------------------ walker
def _check_walk_moves(orc, L, p, steps, lo, hi, seed, walker):
    r = orc.walk(L, p, steps, lo, hi, seed, [walker])
    s, ten = orc.walker_init(seed, L, p, walker, lo, hi)
    k = (L - 1) // 2
    e = np_energy(s)
    last = {}
    for t in range(1, steps + 1):
        a = int(r["moves"][0, t - 1])
        cands = []
        for x in range(p + 1, k + 2):
            u = s.copy()
            u[x - 1] *= -1
            if x != L + 1 - x:
                u[L - x] *= -1
            d = np_energy(u) - e
            admissible = (x not in last) or (t > last[x] + ten)
            if admissible:
                cands.append((d, x))
        assert cands, "this configuration never runs out of admissible moves"
        dmin, xmin = min(cands)
        assert a == xmin
        s[a - 1] *= -1
        if a != L + 1 - a:
            s[L - a] *= -1
        e += dmin
        last[a] = t
        assert r["traj"][0, t - 1] == e
        assert np_energy(s) == e
    assert np.array_equal(r["final"][0], s)
    assert r["final_E"][0] == e
    tr = np.concatenate([[np_energy(orc.walker_init(seed, L, p, walker, lo, hi)[0])],
                         r["traj"][0]])
    assert r["best_E"][0] == tr.min()
    assert r["best_step"][0] == int(np.argmin(tr))


def test_walker_moves_are_best_admissible(orc):
    """Each oracle move is the admissible skew flip of least energy change
    (lowest index on ties) under the tabu tenure, energies by numpy."""
    _check_walk_moves(orc, 13, 0, 60, 2, 2, 1, 0)
    _check_walk_moves(orc, 37, 0, 40, 8, 8, 1, 3)
    _check_walk_moves(orc, 41, 4, 40, 4, 8, 9, 5)


def test_walker_halts_without_admissible_moves(orc):
    """Tenure equal to the free count leaves no admissible move after every
    free position has been flipped once: the walk stops and pads with -1."""
    L, p = 9, 0
    nfree = 5
    r = orc.walk(L, p, 12, nfree, nfree, 3, [0])
    assert list(r["traj"][0, nfree:]) == [-1] * (12 - nfree)
    assert sorted(r["moves"][0, :nfree]) == list(range(1, nfree + 1))


def test_walker_sieve(orc):
    L, p, steps = 37, 0, 200
    em = orc.e_max_for_tau(L, 4)
    r = orc.walk(L, p, steps, 8, 8, 1, range(4), e_max=em)
    n = 0
    for j in range(4):
        hits = [t + 1 for t in range(steps) if 0 <= r["traj"][j, t] <= em]
        got = [t for (E, s, w, t) in r["emits"] if w == j]
        assert got == hits
        n += len(hits)
    assert len(r["emits"]) == n
    for E, s, w, t in r["emits"]:
        assert np_energy(s) == E <= em


# ------------------------------------------------------------------ pool
def test_pool_set_semantics(orc):
    L = 21
    S = li.random_pm1(4, 200, L)
    S = np.concatenate([S, S[:50]])            # duplicates
    E = np.array([np_energy(s) for s in S])
    entries = [(int(E[i]), S[i]) for i in range(len(S))]
    full, dropped = orc.pool(entries, 10 ** 9)
    assert dropped == 0
    uniq = np.unique(S, axis=0)
    assert len(full) == len(uniq)
    # (E, key) order with numpy's lexsort over (E, s_1, ..., s_L)
    Eu = np.array([np_energy(s) for s in uniq])
    order = np.lexsort(tuple(uniq[:, i] for i in range(L - 1, -1, -1)) + (Eu,))
    assert [e for e, _ in full] == list(Eu[order])
    assert [orc.key_seq(k, L).tolist() for _, k in full] == uniq[order].tolist()
    part, dropped = orc.pool(entries, 17)
    assert part == full[:17] and dropped == len(full) - 17


def test_key_and_hex_codec(orc):
    for L in (1, 5, 8, 37, 101):
        for s in li.random_pm1(L, 4, L):
            k = orc.seq_key(s)
            assert np.array_equal(orc.key_seq(k, L), s)
            h = li.hex_encode(s)
            assert int(h, 16) == k
            assert np.array_equal(li.hex_decode(h, L), s)
            assert np.array_equal(li.unpack(li.pack(s), L), s)
    # a sequence starting with -1 keeps its length through the codec
    s = np.array([-1, -1, 1, -1, 1], dtype=np.int8)
    assert np.array_equal(li.hex_decode(li.hex_encode(s), 5), s)


# ------------------------------------------------------------------ second step
def test_step2_reaches_exhaustive_optimum(orc):
    """With room for the whole space the best-first search visits every
    sequence once, so it ends at the exhaustive optimum (literature table)."""
    table = {int(a): int(b) for a, b in _rows("labs_optimal_energies.txt")}
    for L in (7, 9, 10):
        c = li.random_pm1(L, 2, L)
        for B in (1, 5):
            r = orc.step2(L, list(c), B, 1 << 20, 1 << 20, 1 << 40)
            assert r["best_E"] == table[L]
            assert r["expansions"] == 2 ** L
            assert r["pushes"] == 2 ** L - len({tuple(x) for x in c})
            assert r["pushes"] + r["dup_skips"] == r["expansions"] * L
            assert r["evictions"] == 0


def test_step2_pop_order_single(orc):
    """B = 1: the expansion budget pops exactly the sequences a best-first
    search reaches, and the result improves monotonically with the budget."""
    L = 11
    c = li.random_pm1(11, 1, L)
    prev = None
    for X in (1, 2, 5, 20, 100):
        r = orc.step2(L, list(c), 1, 1 << 20, X, 1 << 40)
        assert r["expansions"] == X
        if prev is not None:
            assert r["best_E"] <= prev
        prev = r["best_E"]
    r1 = orc.step2(L, list(c), 1, 1 << 20, 1, 1 << 40)
    e0 = np_energy(c[0])
    nb = []
    for i in range(L):
        t = c[0].copy()
        t[i] *= -1
        nb.append(np_energy(t))
    assert r1["best_E"] == min(e0, min(nb))
    assert r1["pushes"] == L


def _moved(s, r):
    """The text's rotation: r times, move the first element to the end (r > 0),
    or the last element to the start (r < 0)."""
    t = list(s)
    for _ in range(abs(r)):
        t = t[1:] + t[:1] if r > 0 else t[-1:] + t[:-1]
    return np.array(t, dtype=np.int8)


def test_step2_rotations_first_round(orc):
    """B = 1, one pop: Open is the pivot's single flips and its rotations left and
    right by 1..T_r, each once, with energies from numpy; a pivot of period 3
    meets itself at shift 3, which is skipped."""
    for L, T_r, c in ((11, 2, li.random_pm1(4, 1, 11)[0]),
                      (9, 4, np.array([1, 1, -1] * 3, np.int8))):
        r = orc.step2(L, [c], 1, 1 << 20, 1, 1 << 40, T_r=T_r)
        want = {}
        for i in range(L):
            t = c.copy()
            t[i] *= -1
            want[orc.seq_key(t)] = np_energy(t)
        for q in list(range(1, T_r + 1)) + [-q for q in range(1, T_r + 1)]:
            t = _moved(c, q)
            if orc.seq_key(t) != orc.seq_key(c):
                want.setdefault(orc.seq_key(t), np_energy(t))
        assert r["open_keys"] == sorted((E, k) for k, E in want.items())
        assert r["pushes"] == len(want)
        assert r["pushes"] + r["dup_skips"] == L + 2 * T_r


def test_step2_rotations_full_space(orc):
    """With rotations the search still visits every sequence once and ends at the
    exhaustive optimum; the accounting counts L + 2 T_r products per pop."""
    table = {int(a): int(b) for a, b in _rows("labs_optimal_energies.txt")}
    for L, T_r in ((7, 1), (9, 3), (10, 2)):
        c = li.random_pm1(L + 50, 2, L)
        for B in (1, 4):
            r = orc.step2(L, list(c), B, 1 << 20, 1 << 20, 1 << 40, T_r=T_r)
            assert r["best_E"] == table[L]
            assert r["expansions"] == 2 ** L
            assert r["pushes"] == 2 ** L - len({tuple(x) for x in c})
            assert r["pushes"] + r["dup_skips"] == r["expansions"] * (L + 2 * T_r)
    with pytest.raises(ValueError):
        orc.step2(9, list(li.random_pm1(1, 1, 9)), 1, 10, 10, 10, T_r=5)


def test_step2_dynamic_depth(orc):
    """T_u bounds the pops since the last strict improvement."""
    L = 13
    c = li.random_pm1(5, 1, L)
    r = orc.step2(L, list(c), 1, 1 << 20, 10 ** 6, 3)
    assert r["expansions"] <= (r["best_round"] + 1) + 3


def test_step2_capacity_eviction(orc):
    L = 15
    c = li.random_pm1(6, 3, L)
    r = orc.step2(L, list(c), 4, 50, 200, 1 << 40)
    assert r["evictions"] > 0
    assert len(r["open_keys"]) <= 50


@pytest.mark.parametrize("T_r", [0, 2])
def test_step2_unbounded_queue(orc, T_r):
    """Alg. 2's queue has no capacity: with Q >= seeds + X (L + 2 T_r) no cut ever
    evicts, every pushed sequence is new to Open and Closed, and the two sets hold
    exactly the distinct seeds and the pushes (Closed = the expansions)."""
    L, B, X = 23, 8, 200
    c = li.random_pm1(12, 5, L)
    seeds = len({orc.seq_key(s) for s in c})
    r = orc.step2(L, list(c), B, seeds + X * (L + 2 * T_r), X, 1 << 40, T_r=T_r)
    assert r["evictions"] == 0 and r["expansions"] == X
    assert len(r["open_keys"]) + r["expansions"] == seeds + r["pushes"]
    assert len({k for _, k in r["open_keys"]}) == len(r["open_keys"])


def test_zobrist_keys(orc):
    """Zobrist keys: XOR of SplitMix64 outputs over the +1 positions (low bit
    forced to 1), so one flip changes the key by exactly that position's output
    (Alg. 2's HASH_FLIP)."""
    L = 37
    z = orc.zobrist_table(L)
    assert z == orc.splitmix64_stream(orc.ZOBRIST_STATE, L)
    s = li.random_pm1(3, 1, L)[0]
    k = orc.seq_key(s)
    h = orc.zobrist(k, L)
    assert h & 1
    for i in range(L):
        assert orc.zobrist(k ^ (1 << (L - 1 - i)), L) == (h ^ z[i]) | 1
    assert orc.zobrist(0, L) == 1
