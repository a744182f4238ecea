"""Seeded synthetic inputs and the sequence wire format.

Shared by the tests, the oracle checks and the benchmark.  This module holds no
energy, flip, search or ordering arithmetic: only random-number generation,
the structure of the paper's workloads (skew-symmetric sequences, Eq. (2);
restriction-class prefixes, Eq. (3); Legendre-symbol constructions, Sec. 4.1)
and the packing of +1/-1 sequences into 32-bit words.

Packed format (the library's wire format): sequence s_1..s_L occupies
W = ceil(L/32) uint32 words; s_i is bit 31 - ((i-1) mod 32) of word (i-1)//32,
set for +1 and clear for -1; unused low bits of the last word are zero.  Read
word by word, most significant bit first, the words spell the sequence in
order, which is also the digit order of the hexadecimal coding of Sec. 4.
"""
from __future__ import annotations

import numpy as np


def words(L: int) -> int:
    return (L + 31) // 32


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def random_pm1(seed: int, n: int, L: int) -> np.ndarray:
    """n uniform +1/-1 sequences of length L, int8 [n, L]."""
    g = rng(seed)
    return (g.integers(0, 2, size=(n, L), dtype=np.int8) * 2 - 1).astype(np.int8)


def all_pm1_shuffled(seed: int, L: int) -> np.ndarray:
    """Every +1/-1 sequence of length L (2^L of them), int8 [2^L, L], in a seeded
    random order."""
    idx = np.arange(1 << L, dtype=np.int64)
    s = (1 - 2 * ((idx[:, None] >> np.arange(L)) & 1)).astype(np.int8)
    return s[rng(seed).permutation(1 << L)]


def skew_from_half(half: np.ndarray) -> np.ndarray:
    """Extend rows s_1..s_{k+1} to skew-symmetric rows of length 2k+1 (Eq. (2))."""
    h = np.asarray(half, dtype=np.int8)
    if h.ndim == 1:
        return skew_from_half(h[None, :])[0]
    n, kp1 = h.shape
    k = kp1 - 1
    L = 2 * k + 1
    out = np.zeros((n, L), dtype=np.int8)
    out[:, :kp1] = h
    for i in range(1, k + 1):
        sign = 1 if i % 2 == 0 else -1
        out[:, k + i] = sign * h[:, k - i]
    return out


def random_skew(seed: int, n: int, L: int, p: int = 0) -> np.ndarray:
    """n random skew-symmetric sequences of odd length L; with p >= 1 the first
    element is +1 (restriction-class prefixes start with +1)."""
    if L % 2 != 1:
        raise ValueError("skew-symmetric sequences have odd length")
    k = (L - 1) // 2
    h = random_pm1(seed, n, k + 1)
    if p >= 1:
        h[:, 0] = 1
    return skew_from_half(h)


def skew_all(L: int, p: int = 0, prefix=None) -> np.ndarray:
    """Every skew-symmetric sequence with the given prefix, free pattern x in
    LSB-first order over s_{p+1}..s_{k+1} (bit j set -> s_{p+1+j} = +1)."""
    k = (L - 1) // 2
    nfree = k + 1 - p
    x = np.arange(1 << nfree, dtype=np.int64)
    h = np.zeros((1 << nfree, k + 1), dtype=np.int8)
    if p:
        h[:, :p] = np.asarray(prefix, dtype=np.int8)[None, :]
    for j in range(nfree):
        h[:, p + j] = (((x >> j) & 1) * 2 - 1).astype(np.int8)
    return skew_from_half(h)


def legendre_symbol_table(n: int) -> np.ndarray:
    """chi(j) for j = 0..n-1, prime n: +1 for non-zero quadratic residues,
    -1 for non-residues, and -1 at j = 0 (a reading; see the Legendre pins)."""
    res = np.zeros(n, dtype=bool)
    for j in range(1, n):
        res[(j * j) % n] = True
    chi = np.where(res, 1, -1).astype(np.int8)
    chi[0] = -1
    return chi


def legendre_rotated(n: int, o: int, L: int) -> np.ndarray:
    """Legendre sequence of prime length n rotated by o and extended periodically
    to length L: s_j = chi((j + o) mod n), j = 0..L-1 (Sec. 4.1 construction)."""
    chi = legendre_symbol_table(n)
    return chi[(np.arange(L) + o) % n].astype(np.int8)


def pack(seqs: np.ndarray) -> np.ndarray:
    """int8 +1/-1 [n, L] (or [L]) -> uint32 [n, W] (or [W]) in the wire format."""
    s = np.asarray(seqs)
    one = s.ndim == 1
    if one:
        s = s[None, :]
    n, L = s.shape
    W = words(L)
    bits = np.zeros((n, W * 32), dtype=np.uint32)
    bits[:, :L] = (s > 0).astype(np.uint32)
    bits = bits.reshape(n, W, 32)
    shifts = (31 - np.arange(32, dtype=np.uint32))[None, None, :]
    out = np.bitwise_or.reduce(bits << shifts, axis=2).astype(np.uint32)
    return out[0] if one else out


def unpack(packed: np.ndarray, L: int) -> np.ndarray:
    """uint32 [n, W] (or [W]) -> int8 +1/-1 [n, L] (or [L])."""
    w = np.asarray(packed, dtype=np.uint32)
    one = w.ndim == 1
    if one:
        w = w[None, :]
    shifts = (31 - np.arange(32, dtype=np.uint32))[None, None, :]
    bits = ((w[:, :, None] >> shifts) & 1).reshape(w.shape[0], w.shape[1] * 32)[:, :L]
    out = (bits.astype(np.int8) * 2 - 1).astype(np.int8)
    return out[0] if one else out


def hex_encode(s: np.ndarray) -> str:
    """Hexadecimal coding of Sec. 4: +1 -> 1, -1 -> 0, left-padded with zero bits
    to a multiple of 4, upper-case digits."""
    a = np.asarray(s)
    L = len(a)
    pad = (-L) % 4
    bits = "0" * pad + "".join("1" if x > 0 else "0" for x in a)
    return "".join("%X" % int(bits[i:i + 4], 2) for i in range(0, len(bits), 4))


def hex_decode(h: str, L: int) -> np.ndarray:
    """Inverse of hex_encode: drop exactly 4*len(h) - L leading pad bits (so a
    sequence that starts with -1 decodes correctly), 0 -> -1."""
    bits = "".join(format(int(c, 16), "04b") for c in h.strip())
    pad = len(bits) - L
    if pad < 0 or pad > 3 or "1" in bits[:pad]:
        raise ValueError("hex string does not hold a sequence of length %d" % L)
    return np.array([1 if b == "1" else -1 for b in bits[pad:]], dtype=np.int8)


def mlp_init(seed: int, d_in: int, d_h: int, d_out: int) -> dict:
    """Initial MLP weights: U(-1/sqrt(fan_in), 1/sqrt(fan_in)) per layer from a
    seeded PCG64 stream, zero biases (float32).  W1 [d_h, d_in], W2 [d_h, d_h],
    W3 [d_out, d_h]."""
    g = rng(seed)

    def u(rows, cols):
        b = 1.0 / np.sqrt(cols)
        return g.uniform(-b, b, size=(rows, cols)).astype(np.float32)

    return {"W1": u(d_h, d_in), "b1": np.zeros(d_h, np.float32),
            "W2": u(d_h, d_h), "b2": np.zeros(d_h, np.float32),
            "W3": u(d_out, d_h), "b3": np.zeros(d_out, np.float32)}
