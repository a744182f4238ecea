"""Plain, slow CPU oracle for the LABS dual-step hot path (arXiv 2409.07222).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The product
library (``paper_2409_07222_amd``) never imports it, and it never imports the
product library: the two share no code.

Layers:
  * ``labs_oracle.c`` (built to ``liblabs_oracle.so`` with gcc): definitional
    energy, skew completion, skew flips, the first-step walker (Algorithm 1 with
    a tabu tenure, and with its Bloom filter), exhaustive enumeration,
    SplitMix64.  Every energy change is
    recomputed from the definition of E; no incremental formula is used.
  * ``labs_baseline.c`` (built to ``liblabs_baseline.so`` with gcc -O3 and
    OpenMP): the CPU baseline of the first step, the tabu walker with the
    linear-time neighbour evaluation of Sec. 3, one walker per thread.  The
    benchmark times it; a test pins its trajectories to the definitional walker.
  * this module: ctypes bindings, the candidate pool (set semantics, kept in
    (E, key) order), and the second step (Algorithm 2) as a batch-synchronous
    best-first search over Python sets and dicts.

Ordering key (a reading; the paper is silent on ties): sequences compare by
(E, key) where key is the sequence read as a binary number with s_1 the most
significant bit and +1 -> 1, -1 -> 0, the same digit order as the hexadecimal
coding used for the record table in Sec. 4.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "labs_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liblabs_oracle.so")
_lock = threading.Lock()
_lib = None

_i8p = ctypes.POINTER(ctypes.c_int8)
_i32p = ctypes.POINTER(ctypes.c_int32)
_i64p = ctypes.POINTER(ctypes.c_int64)
_u64p = ctypes.POINTER(ctypes.c_uint64)


def build(force: bool = True) -> str:
    """Compile labs_oracle.c into liblabs_oracle.so with gcc (plain -O2)."""
    if not force and os.path.exists(_LIB_PATH) and \
            os.path.getmtime(_LIB_PATH) >= os.path.getmtime(_SRC):
        return _LIB_PATH
    tmp = _LIB_PATH + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-shared", "-fPIC", "-Wall",
                           "-o", tmp, _SRC])
    os.replace(tmp, _LIB_PATH)
    build_baseline(native=False)
    return _LIB_PATH


_BL_SRC = os.path.join(_HERE, "labs_baseline.c")
_BL_PATH = os.path.join(_HERE, "liblabs_baseline.so")
_bl_libs = {}


def build_baseline(native: bool = False) -> str:
    """Compile labs_baseline.c with gcc -O3 -fopenmp.  native=False: a portable
    x86-64-v2 build in-tree (what the tests load); native=True: -march=native
    for the host that runs it, into a temporary directory (the benchmark's CPU
    baseline is timed with this one)."""
    import tempfile
    if native:
        path = os.path.join(tempfile.mkdtemp(prefix="labs_baseline_"), "liblabs_baseline_native.so")
        arch = "-march=native"
    else:
        path = _BL_PATH
        arch = "-march=x86-64-v2"
    tmp = path + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O3", arch, "-fopenmp", "-std=c99", "-shared", "-fPIC", "-Wall",
                           "-o", tmp, _BL_SRC])
    os.replace(tmp, path)
    return path


def baseline_lib(native: bool = False):
    with _lock:
        if native not in _bl_libs:
            if native:
                path = build_baseline(native=True)
            else:
                path = _BL_PATH
                if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_BL_SRC):
                    build_baseline(native=False)
            L = ctypes.CDLL(path)
            L.bl_walk.restype = ctypes.c_int32
            L.bl_walk.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                  ctypes.c_int32, ctypes.c_uint64, ctypes.c_int64, ctypes.c_int64,
                                  ctypes.c_int32, _i32p, _i32p, _i32p, _i64p]
            _bl_libs[native] = L
        return _bl_libs[native]


def baseline_walk(L: int, p: int, steps: int, tenure_lo: int, tenure_hi: int, seed: int,
                  walker_begin: int, n: int, threads: int = 0, want_traj: bool = False,
                  native: bool = False) -> dict:
    """The CPU baseline walker (labs_baseline.c) over walkers walker_begin..+n-1 on
    `threads` OpenMP threads (0: the runtime default).  Returns final and best
    energies, the trajectories when asked, flip-evals and the threads used."""
    lb = baseline_lib(native)
    traj = np.zeros((n, steps), dtype=np.int32) if want_traj else None
    fin = np.zeros(n, dtype=np.int32)
    best = np.zeros(n, dtype=np.int32)
    fe = ctypes.c_int64(0)
    used = lb.bl_walk(L, p, steps, tenure_lo, tenure_hi, seed, walker_begin, n, threads,
                      _p(traj, _i32p) if want_traj else None, _p(fin, _i32p), _p(best, _i32p),
                      ctypes.byref(fe))
    return {"traj": traj, "final_E": fin, "best_E": best, "flip_evals": int(fe.value),
            "threads": int(used)}


def lib():
    global _lib
    with _lock:
        if _lib is None:
            build(force=False)
            L = ctypes.CDLL(_LIB_PATH)
            L.or_autocorr.restype = ctypes.c_int64
            L.or_autocorr.argtypes = [ctypes.c_int32, _i8p, ctypes.c_int32]
            L.or_energy.restype = ctypes.c_int64
            L.or_energy.argtypes = [ctypes.c_int32, _i8p, _i64p]
            L.or_energy_batch.restype = None
            L.or_energy_batch.argtypes = [ctypes.c_int32, ctypes.c_int64, _i8p, _i64p, _i64p]
            L.or_skew_complete.restype = None
            L.or_skew_complete.argtypes = [ctypes.c_int32, _i8p]
            L.or_is_skew.restype = ctypes.c_int32
            L.or_is_skew.argtypes = [ctypes.c_int32, _i8p]
            L.or_flip_skew.restype = None
            L.or_flip_skew.argtypes = [ctypes.c_int32, _i8p, ctypes.c_int32]
            L.or_delta_single.restype = ctypes.c_int64
            L.or_delta_single.argtypes = [ctypes.c_int32, _i8p, ctypes.c_int32]
            L.or_delta_skew.restype = ctypes.c_int64
            L.or_delta_skew.argtypes = [ctypes.c_int32, _i8p, ctypes.c_int32]
            L.or_deltas_single.restype = None
            L.or_deltas_single.argtypes = [ctypes.c_int32, _i8p, _i64p]
            L.or_deltas_skew.restype = None
            L.or_deltas_skew.argtypes = [ctypes.c_int32, ctypes.c_int32, _i8p, _i64p]
            L.or_mix64.restype = ctypes.c_uint64
            L.or_mix64.argtypes = [ctypes.c_uint64]
            L.or_splitmix64_next.restype = ctypes.c_uint64
            L.or_splitmix64_next.argtypes = [_u64p]
            L.or_walker_key.restype = ctypes.c_uint64
            L.or_walker_key.argtypes = [ctypes.c_uint64, ctypes.c_int32, ctypes.c_int64]
            L.or_walker_init.restype = None
            L.or_walker_init.argtypes = [ctypes.c_uint64, ctypes.c_int32, ctypes.c_int32,
                                         ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                         _i8p, _i32p]
            L.or_walk_one.restype = ctypes.c_int64
            L.or_walk_one.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                      ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64,
                                      ctypes.c_int64, ctypes.c_int32,
                                      _i32p, _i32p, _i8p, _i64p, _i8p, _i64p, _i32p,
                                      ctypes.c_int64, _i64p, _i8p, _i32p]
            _u8p = ctypes.POINTER(ctypes.c_uint8)
            L.or_zobrist_key.restype = ctypes.c_uint64
            L.or_zobrist_key.argtypes = [ctypes.c_int32]
            L.or_seq_hash.restype = ctypes.c_uint64
            L.or_seq_hash.argtypes = [ctypes.c_int32, _i8p]
            L.or_bloom_index.restype = ctypes.c_uint32
            L.or_bloom_index.argtypes = [ctypes.c_uint64, ctypes.c_int32, ctypes.c_int32]
            L.or_bloom_insert.restype = None
            L.or_bloom_insert.argtypes = [_u8p, ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64]
            L.or_bloom_member.restype = ctypes.c_int32
            L.or_bloom_member.argtypes = [_u8p, ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64]
            L.or_walk_bloom_one.restype = ctypes.c_int64
            L.or_walk_bloom_one.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                            ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64,
                                            ctypes.c_int64, ctypes.c_int32,
                                            _i32p, _i32p, _i8p, _i64p, _i8p, _i64p, _i32p,
                                            ctypes.c_int64, _i64p, _i8p, _i32p]
            L.or_skew_exhaustive.restype = ctypes.c_int64
            L.or_skew_exhaustive.argtypes = [ctypes.c_int32, ctypes.c_int32, _i8p, _i64p]
            L.or_exhaustive_min.restype = ctypes.c_int64
            L.or_exhaustive_min.argtypes = [ctypes.c_int32, _i64p]
            _lib = L
    return _lib


def _p(a, t):
    return a.ctypes.data_as(t)


def _seq(s) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(s, dtype=np.int8))
    if a.ndim != 1 or not np.all(np.abs(a) == 1):
        raise ValueError("a sequence is a 1-D array of +1/-1")
    return a


# ---------------------------------------------------------------- definitions
def autocorr(s, k: int) -> int:
    """C_k(S) (Sec. 1)."""
    a = _seq(s)
    return int(lib().or_autocorr(len(a), _p(a, _i8p), k))


def energy(s, with_c: bool = False):
    """E(S) = sum_k C_k^2 (Sec. 1); optionally also C_1..C_{L-1}."""
    a = _seq(s)
    L = len(a)
    c = np.zeros(max(L - 1, 0), dtype=np.int64)
    e = int(lib().or_energy(L, _p(a, _i8p), _p(c, _i64p)))
    return (e, c) if with_c else e


def energy_batch(seqs: np.ndarray, with_c: bool = False):
    s = np.ascontiguousarray(seqs, dtype=np.int8)
    n, L = s.shape
    E = np.zeros(n, dtype=np.int64)
    C = np.zeros((n, max(L - 1, 0)), dtype=np.int64) if with_c else None
    lib().or_energy_batch(L, n, _p(s, _i8p), _p(E, _i64p),
                          _p(C, _i64p) if with_c else None)
    return (E, C) if with_c else E


def merit_factor(L: int, E: int) -> float:
    """Eq. (1): F = L^2 / (2E)."""
    return (L * L) / (2.0 * E)


def e_max_for_tau(L: int, num: int, den: int = 1) -> int:
    """Largest integer E with F = L^2/(2E) >= num/den, i.e. floor(L^2 den / (2 num))."""
    return (L * L * den) // (2 * num)


def skew_complete(first_half) -> np.ndarray:
    """Eq. (2): extend s_1..s_{k+1} to the skew-symmetric sequence of length 2k+1."""
    h = _seq(first_half)
    L = 2 * len(h) - 1
    s = np.zeros(L, dtype=np.int8)
    s[:len(h)] = h
    lib().or_skew_complete(L, _p(s, _i8p))
    return s


def is_skew(s) -> bool:
    a = _seq(s)
    return bool(lib().or_is_skew(len(a), _p(a, _i8p)))


def flip_skew(s, a: int) -> np.ndarray:
    t = _seq(s).copy()
    lib().or_flip_skew(len(t), _p(t, _i8p), a)
    return t


def delta_single(s, i: int) -> int:
    a = _seq(s)
    return int(lib().or_delta_single(len(a), _p(a, _i8p), i))


def delta_skew(s, a: int) -> int:
    x = _seq(s)
    return int(lib().or_delta_skew(len(x), _p(x, _i8p), a))


def deltas_single(s) -> np.ndarray:
    a = _seq(s)
    out = np.zeros(len(a), dtype=np.int64)
    lib().or_deltas_single(len(a), _p(a, _i8p), _p(out, _i64p))
    return out


def deltas_skew(s, p: int) -> np.ndarray:
    a = _seq(s)
    L = len(a)
    k = (L - 1) // 2
    out = np.zeros(k + 1 - p, dtype=np.int64)
    lib().or_deltas_skew(L, p, _p(a, _i8p), _p(out, _i64p))
    return out


# ---------------------------------------------------------------- generator
def splitmix64_stream(state: int, n: int) -> list:
    st = ctypes.c_uint64(state)
    return [int(lib().or_splitmix64_next(ctypes.byref(st))) for _ in range(n)]


def walker_key(seed: int, L: int, walker: int) -> int:
    return int(lib().or_walker_key(seed, L, walker))


def walker_init(seed: int, L: int, p: int, walker: int, tenure_lo: int, tenure_hi: int):
    s = np.zeros(L, dtype=np.int8)
    ten = ctypes.c_int32(0)
    lib().or_walker_init(seed, L, p, walker, tenure_lo, tenure_hi, _p(s, _i8p),
                         ctypes.byref(ten))
    return s, int(ten.value)


# ---------------------------------------------------------------- first step
def walk(L: int, p: int, steps: int, tenure_lo: int, tenure_hi: int, seed: int,
         walkers, e_max: int = -1, want_traj: bool = True, emit_cap: int = 1 << 16):
    """Run the first-step walker for each id in ``walkers`` (Algorithm 1 with a
    tabu tenure; see or_walk_one).  Returns a dict of numpy arrays plus the list
    of sieve emissions (E, seq, walker, t)."""
    lb = lib()

    def one(w, *rest):
        return lb.or_walk_one(L, p, steps, tenure_lo, tenure_hi, seed, w, e_max, *rest)
    return _walks(L, steps, walkers, e_max, want_traj, emit_cap, one)


def walk_bloom(L: int, p: int, steps: int, log2_bits: int, n_hash: int, seed: int, walkers,
               e_max: int = -1, want_traj: bool = True, emit_cap: int = 1 << 16):
    """Run the first-step walker with the Bloom filter of Algorithm 1 for each id
    in ``walkers`` (see or_walk_bloom_one): same outputs as :func:`walk`."""
    lb = lib()

    def one(w, *rest):
        return lb.or_walk_bloom_one(L, p, steps, log2_bits, n_hash, seed, w, e_max, *rest)
    return _walks(L, steps, walkers, e_max, want_traj, emit_cap, one)


def walk_hash(L: int, s) -> int:
    """Key of a skew sequence in the first step's Bloom filter: the Zobrist hash
    of its first k+1 elements (or_seq_hash)."""
    a = np.ascontiguousarray(np.asarray(s, dtype=np.int8))
    return int(lib().or_seq_hash(L, _p(a, _i8p)))


def walk_zobrist(i: int) -> int:
    """Z_i of the first step's key (1-based position), or_zobrist_key."""
    return int(lib().or_zobrist_key(i))


class Bloom:
    """The oracle's Bloom filter of 2^log2_bits bits probed n_hash times."""

    def __init__(self, log2_bits: int, n_hash: int):
        self.log2_bits, self.n_hash = log2_bits, n_hash
        self.bits = np.zeros(max(1, (1 << log2_bits) // 8), dtype=np.uint8)
        self._p = self.bits.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))

    def index(self, h: int, j: int) -> int:
        return int(lib().or_bloom_index(h, self.log2_bits, j))

    def insert(self, h: int) -> None:
        lib().or_bloom_insert(self._p, self.log2_bits, self.n_hash, h)

    def __contains__(self, h: int) -> bool:
        return bool(lib().or_bloom_member(self._p, self.log2_bits, self.n_hash, h))


def _walks(L, steps, walkers, e_max, want_traj, emit_cap, one):
    ids = list(walkers)
    n = len(ids)
    traj = np.zeros((n, steps), dtype=np.int32)
    moves = np.zeros((n, steps), dtype=np.int32)
    fin = np.zeros((n, L), dtype=np.int8)
    finE = np.zeros(n, dtype=np.int64)
    best = np.zeros((n, L), dtype=np.int8)
    bestE = np.zeros(n, dtype=np.int64)
    bestT = np.zeros(n, dtype=np.int32)
    emits = []
    for j, w in enumerate(ids):
        cap = emit_cap if e_max >= 0 else 0
        while True:
            eE = np.zeros(max(cap, 1), dtype=np.int64)
            eS = np.zeros((max(cap, 1), L), dtype=np.int8)
            eT = np.zeros(max(cap, 1), dtype=np.int32)
            tr = traj[j]
            b_t = ctypes.c_int32(0)
            f_e = np.zeros(1, dtype=np.int64)
            b_e = np.zeros(1, dtype=np.int64)
            cnt = one(w, _p(tr, _i32p) if want_traj else None,
                      _p(moves[j], _i32p) if want_traj else None,
                      _p(fin[j], _i8p), _p(f_e, _i64p),
                      _p(best[j], _i8p), _p(b_e, _i64p), ctypes.byref(b_t),
                      cap, _p(eE, _i64p), _p(eS, _i8p), _p(eT, _i32p))
            if cnt <= cap:
                break
            cap = int(cnt)
        finE[j] = f_e[0]
        bestE[j] = b_e[0]
        bestT[j] = b_t.value
        for q in range(int(cnt)):
            emits.append((int(eE[q]), eS[q].copy(), int(w), int(eT[q])))
    return dict(traj=traj if want_traj else None, moves=moves if want_traj else None, final=fin, final_E=finE,
                best=best, best_E=bestE, best_step=bestT, emits=emits)


def skew_exhaustive(L: int, p: int = 0, prefix=None, want_all: bool = False):
    """All skew-symmetric sequences with the given prefix: min E (and every E)."""
    k = (L - 1) // 2
    nfree = k + 1 - p
    pre = np.ascontiguousarray(np.asarray(prefix if prefix is not None else [], dtype=np.int8))
    if len(pre) != p:
        raise ValueError("prefix length must be p")
    allE = np.zeros(1 << nfree, dtype=np.int64) if want_all else None
    m = int(lib().or_skew_exhaustive(L, p, _p(pre, _i8p) if p else None,
                                     _p(allE, _i64p) if want_all else None))
    return (m, allE) if want_all else m


def exhaustive_min(L: int):
    cnt = ctypes.c_int64(0)
    m = int(lib().or_exhaustive_min(L, ctypes.byref(cnt)))
    return m, int(cnt.value)


# ---------------------------------------------------------------- ordering
def seq_key(s) -> int:
    """Sequence as a binary number, s_1 most significant, +1 -> 1."""
    a = _seq(s)
    v = 0
    for x in a:
        v = (v << 1) | (1 if x > 0 else 0)
    return v


def key_seq(key: int, L: int) -> np.ndarray:
    return np.array([1 if (key >> (L - 1 - i)) & 1 else -1 for i in range(L)], dtype=np.int8)


# ---------------------------------------------------------------- pool
def pool(entries, capacity: int):
    """The candidate pool: the distinct emitted sequences, in (E, key) order,
    truncated to the ``capacity`` smallest.  ``entries`` is an iterable of
    (E, seq) or (E, seq, ...).  Returns (list of (E, key), dropped) where
    dropped counts the distinct sequences cut by the capacity."""
    seen = {}
    for ent in entries:
        E, s = int(ent[0]), ent[1]
        key = seq_key(s)
        if key in seen:
            if seen[key] != E:
                raise AssertionError("one sequence with two energies")
            continue
        seen[key] = E
    order = sorted((E, key) for key, E in seen.items())
    return order[:capacity], max(0, len(order) - capacity)


def topk(entries, k: int):
    return pool(entries, k)[0]


# ---------------------------------------------------------------- Legendre seeds
def legendre_chi(n: int) -> np.ndarray:
    """chi(a), a = 0..n-1, for an odd prime n by Euler's criterion: a^((n-1)/2) mod n
    is 1 for quadratic residues; chi(0) = -1 (the construction's reading)."""
    chi = np.array([1 if pow(a, (n - 1) // 2, n) == 1 else -1 for a in range(n)], dtype=np.int8)
    chi[0] = -1
    return chi


def _is_prime(n: int) -> bool:
    if n < 2:
        return False
    d = 2
    while d * d <= n:
        if n % d == 0:
            return False
        d += 1
    return True


def legendre_pairs(L: int, t_lo: int = 0, t_hi: int = 900, r_lo: int = 1800, r_hi: int = 2600):
    """Sec. 4.1 sweep (a reading): every odd prime n <= L whose appended fraction
    (L - n)/n lies in [t_lo, t_hi] / 10^4 and every rotation o with o/n in
    [r_lo, r_hi] / 10^4, in (n, o) order.  The paper's narrower ranges
    (0.055..0.063, 0.20..0.24) hold no prime at most lengths; this sweep's best
    reproduces its construction column."""
    out = []
    for n in range(3, L + 1):
        if not _is_prime(n):
            continue
        if not (t_lo * n <= (L - n) * 10000 <= t_hi * n):
            continue
        for o in range(n):
            if r_lo * n <= o * 10000 <= r_hi * n:
                out.append((n, o))
    return out


def legendre_sequence(n: int, o: int, L: int, chi=None) -> np.ndarray:
    """The rotated Legendre sequence extended periodically: s_j = chi((j + o) mod n), j = 0..L-1."""
    c = legendre_chi(n) if chi is None else chi
    return c[(np.arange(L) + o) % n].astype(np.int8)


def legendre_sweep(L: int, **kw):
    """[(n, o, E)] over the sweep's pairs, each energy from the definition."""
    out = []
    chis = {}
    for n, o in legendre_pairs(L, **kw):
        if n not in chis:
            chis[n] = legendre_chi(n)
        out.append((n, o, energy(legendre_sequence(n, o, L, chis[n]))))
    return out


# ---------------------------------------------------------------- length operators
def length_operators(s):
    """Sec. 3 (the sequence operators that extend the search to even lengths):
    from a sequence of length L, the two sequences of length L-1 that remove its
    first or its last element, and the four of length L+1 that put +1 or -1
    before its first or after its last element.  Returns (minus, plus) as int8
    arrays [2, L-1] (remove first, remove last) and [4, L+1] (+1 first, -1 first,
    +1 last, -1 last)."""
    a = _seq(s)
    minus = np.stack([a[1:], a[:-1]])
    one = np.ones(1, np.int8)
    plus = np.stack([np.concatenate([one, a]), np.concatenate([-one, a]),
                     np.concatenate([a, one]), np.concatenate([a, -one])])
    return minus, plus


# ---------------------------------------------------------------- second step
# Second-step tie order (a reading; the paper is silent on ties): (E, z, key)
# where z is the sequence's Zobrist key -- the XOR, over the positions i with
# s_i = +1, of output i-1 of the SplitMix64 stream started at ZOBRIST_STATE, with
# its lowest bit set -- and key the sequence as above.
ZOBRIST_STATE = 0x6A09E667F3BCC909


def zobrist_table(L: int) -> list:
    return splitmix64_stream(ZOBRIST_STATE, L)


def zobrist(key: int, L: int, table=None) -> int:
    z = table if table is not None else zobrist_table(L)
    h = 0
    for i in range(L):
        if (key >> (L - 1 - i)) & 1:
            h ^= z[i]
    return h | 1


def step2(L: int, candidates, batch: int, pq_capacity: int, max_expansions: int,
          T_u: int, T_r: int = 0):
    """Second step (Algorithm 2) as a batch-synchronous best-first search.

    Open (the priority queue) and Closed (popped sequences) are exact sets of
    sequences.  Each round pops the min(batch, remaining) smallest Open entries in
    (E, Zobrist key, key) order, moves them to Closed, and expands every single flip of every
    pivot; a neighbour already in Closed, Open or this round's batch is skipped
    (the PQ.contains test).  Energies are recomputed from the definition.  The
    best sequence improves only on a strictly lower energy; u counts pops since
    the last improvement (reset to 0 by an improving round, else += pops), which
    for batch = 1 is exactly the dynamic-depth counter of Algorithm 2.  Open is
    then cut to the pq_capacity smallest.

    MAKE_ROTATIONS (T_r > 0; Sec. 3, rotations of the pivot): after the single
    flips of every pivot of the round, each pivot in pop order also produces its
    cyclic rotations left by 1..T_r (the first element moved to the end, repeatedly)
    and then right by 1..T_r, each skipped or pushed like a neighbour.
    """
    if T_r < 0 or (T_r and 2 * T_r >= L):
        raise ValueError("T_r must satisfy 0 <= 2 T_r < L")
    lb = lib()
    zt = zobrist_table(L)

    def order(key, E):
        return (E, zobrist(key, L, zt), key)

    open_ = {}
    for c in candidates:
        s = _seq(c)
        if len(s) != L:
            raise ValueError("candidate length")
        open_[seq_key(s)] = energy(s)
    if len(open_) > pq_capacity:
        keep = sorted(order(k, E) for k, E in open_.items())[:pq_capacity]
        open_ = {k: E for E, _, k in keep}
    closed = set()
    if not open_:
        return dict(best_E=None, best_key=None, expansions=0, pushes=0, dup_skips=0,
                    evictions=0, best_round=-1, rounds=0, open_keys=[])
    bE, _, bK = min(order(k, E) for k, E in open_.items())
    u = 0
    done = 0
    pushes = dups = evictions = 0
    best_round = -1
    rnd = 0
    while open_ and done < max_expansions and u < T_u:
        ordered = sorted(order(k, E) for k, E in open_.items())
        P = ordered[:min(batch, max_expansions - done)]
        for E, _, k in P:
            del open_[k]
            closed.add(k)
        done += len(P)
        new = {}
        for E, _, k in P:
            s = key_seq(k, L)
            for i in range(L):
                nk = k ^ (1 << (L - 1 - i))
                if nk in closed or nk in open_ or nk in new:
                    dups += 1
                    continue
                t = s.copy()
                t[i] = -t[i]
                new[nk] = int(lb.or_energy(L, _p(t, _i8p), None))
        for E, _, k in P if T_r else ():
            s = key_seq(k, L)
            for shift in list(range(1, T_r + 1)) + [-r for r in range(1, T_r + 1)]:
                t = np.ascontiguousarray(np.roll(s, -shift))   # left by shift (right if negative)
                nk = seq_key(t)
                if nk in closed or nk in open_ or nk in new:
                    dups += 1
                    continue
                new[nk] = int(lb.or_energy(L, _p(t, _i8p), None))
        pushes += len(new)
        if new:
            mE, _, mK = min(order(k, E) for k, E in new.items())
            if mE < bE:
                bE, bK = mE, mK
                u = 0
                best_round = rnd
            else:
                u += len(P)
        else:
            u += len(P)
        open_.update(new)
        if len(open_) > pq_capacity:
            keep = sorted(order(k, E) for k, E in open_.items())
            evictions += len(keep) - pq_capacity
            open_ = {k: E for E, _, k in keep[:pq_capacity]}
        rnd += 1
    return dict(best_E=bE, best_key=bK, expansions=done, pushes=pushes, dup_skips=dups,
                evictions=evictions, best_round=best_round, rounds=rnd,
                open_keys=sorted((E, k) for k, E in open_.items()))
