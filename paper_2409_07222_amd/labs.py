"""Thin ctypes binding of liblabs.so (include/labs.h).

Argument marshalling only: every computation runs in the library's HIP
kernels.  Tensors are torch tensors on a ROCm device; the binding passes their
data pointers and the current HIP stream.  If the library has not been built,
or no GPU is present, calls raise -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
import threading
from dataclasses import dataclass

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblabs.so")

LABS_OK = 0
LABS_POOL_WALKER_BEST = 1

_lock = threading.Lock()
_lib = None


class LabsError(RuntimeError):
    pass


class BloomCfg(ctypes.Structure):
    _fields_ = [("log2_bits", ctypes.c_int32), ("n_hash", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 2)]


class LegendreSweep(ctypes.Structure):
    _fields_ = [("t_lo", ctypes.c_int32), ("t_hi", ctypes.c_int32),
                ("r_lo", ctypes.c_int32), ("r_hi", ctypes.c_int32)]


class Step1Cfg(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int32), ("p", ctypes.c_int32), ("steps", ctypes.c_int32),
                ("tenure_lo", ctypes.c_int32), ("tenure_hi", ctypes.c_int32),
                ("e_max", ctypes.c_int32), ("walker_begin", ctypes.c_int64),
                ("n_walkers", ctypes.c_int64), ("seed", ctypes.c_uint64),
                ("flags", ctypes.c_uint32), ("reserved", ctypes.c_int32)]


class Pool(ctypes.Structure):
    _fields_ = [("seqs", ctypes.c_void_p), ("E", ctypes.c_void_p), ("walker", ctypes.c_void_p),
                ("step", ctypes.c_void_p), ("capacity", ctypes.c_int64),
                ("count", ctypes.c_void_p), ("dropped", ctypes.c_void_p)]


MAX_LEVELS = 16
_STAMP_FIELDS = [("n_levels", ctypes.c_int32), ("level_E", ctypes.c_int32 * MAX_LEVELS),
                 ("first_hit_ticks", ctypes.c_void_p), ("start_ticks", ctypes.c_void_p)]


class Step1Out(ctypes.Structure):
    _fields_ = [("final_seqs", ctypes.c_void_p), ("final_E", ctypes.c_void_p),
                ("best_seqs", ctypes.c_void_p), ("best_E", ctypes.c_void_p),
                ("best_step", ctypes.c_void_p), ("traj_E", ctypes.c_void_p),
                ("flip_evals", ctypes.c_void_p)] + _STAMP_FIELDS


class Step2Cfg(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int32), ("batch", ctypes.c_int32), ("T_r", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("pq_capacity", ctypes.c_int64),
                ("max_expansions", ctypes.c_int64), ("T_u", ctypes.c_int64)]


class Step2Stats(ctypes.Structure):
    _fields_ = [("expansions", ctypes.c_int64), ("pushes", ctypes.c_int64),
                ("dup_skips", ctypes.c_int64), ("evictions", ctypes.c_int64),
                ("rounds", ctypes.c_int64), ("open_count", ctypes.c_int64),
                ("best_E", ctypes.c_int32), ("best_round", ctypes.c_int32),
                ("rebuilds", ctypes.c_int64)]


class Step2Out(ctypes.Structure):
    _fields_ = [("best_seq", ctypes.c_void_p), ("best_E", ctypes.c_void_p),
                ("stats", ctypes.c_void_p), ("open_seqs", ctypes.c_void_p),
                ("open_E", ctypes.c_void_p), ("open_capacity", ctypes.c_int64)]


class MlpLayout(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int32), ("k", ctypes.c_int32), ("d_in", ctypes.c_int32),
                ("d_out", ctypes.c_int32), ("hidden", ctypes.c_int32), ("ld_in", ctypes.c_int32),
                ("ld_out", ctypes.c_int32), ("mask_words", ctypes.c_int32),
                ("off_W1", ctypes.c_int64), ("off_b1", ctypes.c_int64), ("off_W2", ctypes.c_int64),
                ("off_b2", ctypes.c_int64), ("off_W3", ctypes.c_int64), ("off_b3", ctypes.c_int64),
                ("n_params", ctypes.c_int64)]


class Proposer(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("top_m", ctypes.c_int32),
                ("fallback_every", ctypes.c_int32), ("hidden", ctypes.c_int32),
                ("params", ctypes.c_void_p), ("params_bf16", ctypes.c_void_p),
                ("seed", ctypes.c_uint64), ("log_every", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class LearnedOut(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in (
        "final_seqs", "final_E", "best_seqs", "best_E", "best_step", "hit_step", "traj_E", "moves",
        "cands", "log_seqs", "log_mask", "log_label", "flip_evals")] + _STAMP_FIELDS


class Stamps:
    """First-hit stamps of the device real-time counter: pass one object to
    several calls to accumulate over them.  ticks[l] is the counter's value when
    a walker first reached E <= level_E[l] (2^64 - 1: never), start the earliest
    walker-init start; seconds() converts to seconds since start."""

    def __init__(self, level_E, device="cuda"):
        torch = _torch()
        if not 1 <= len(level_E) <= MAX_LEVELS:
            raise LabsError("1..%d levels" % MAX_LEVELS)
        self.level_E = [int(e) for e in level_E]
        self.ticks = torch.full((len(level_E),), -1, dtype=torch.int64, device=device)
        self.start = torch.full((1,), -1, dtype=torch.int64, device=device)

    def fill(self, out):
        out.n_levels = len(self.level_E)
        for i, e in enumerate(self.level_E):
            out.level_E[i] = e
        out.first_hit_ticks = self.ticks.data_ptr()
        out.start_ticks = self.start.data_ptr()

    def seconds(self):
        """Per level, seconds from the earliest start to the first hit (None: no hit)."""
        hz = realtime_hz()
        t = [x & 0xFFFFFFFFFFFFFFFF for x in self.ticks.cpu().tolist()]
        s0 = self.start.cpu().tolist()[0] & 0xFFFFFFFFFFFFFFFF
        return [None if x == 0xFFFFFFFFFFFFFFFF else (x - s0) / hz for x in t]


def realtime_hz() -> int:
    """labs_realtime_hz: ticks per second of the stamps' counter on the current device."""
    v = ctypes.c_int64(0)
    _check(lib().labs_realtime_hz(ctypes.byref(v)))
    return int(v.value)


PROPOSE_MLP = 0
PROPOSE_RANDOM = 1


def lib():
    """Load liblabs.so (never builds it)."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise LabsError("liblabs.so is not built; run __graft_entry__.build()")
            L = ctypes.CDLL(LIB_PATH)
            vp, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
            L.labs_abi_version.restype = i32
            L.labs_status_str.restype = ctypes.c_char_p
            L.labs_status_str.argtypes = [i32]
            L.labs_last_error.restype = ctypes.c_char_p
            L.labs_words.restype = i32
            L.labs_words.argtypes = [i32]
            L.labs_realtime_hz.restype = i32
            L.labs_realtime_hz.argtypes = [ctypes.POINTER(i64)]
            L.labs_energy.restype = i32
            L.labs_energy.argtypes = [i32, i64, vp, vp, vp, vp]
            L.labs_flip_deltas.restype = i32
            L.labs_flip_deltas.argtypes = [i32, i32, i32, i64, vp, vp, vp]
            L.labs_walk_step1_workspace.restype = i32
            L.labs_walk_step1_workspace.argtypes = [ctypes.POINTER(Step1Cfg), i32, i64,
                                                    ctypes.POINTER(sz)]
            L.labs_walk_step1.restype = i32
            L.labs_walk_step1.argtypes = [ctypes.POINTER(Step1Cfg), i32, vp, ctypes.POINTER(Pool),
                                          ctypes.POINTER(Step1Out), vp, sz, vp]
            L.labs_walk_step1_bloom_workspace.restype = i32
            L.labs_walk_step1_bloom_workspace.argtypes = [ctypes.POINTER(Step1Cfg), ctypes.POINTER(BloomCfg),
                                                          i64, ctypes.POINTER(sz)]
            L.labs_walk_step1_bloom.restype = i32
            L.labs_walk_step1_bloom.argtypes = [ctypes.POINTER(Step1Cfg), ctypes.POINTER(BloomCfg),
                                                ctypes.POINTER(Pool), ctypes.POINTER(Step1Out), vp, sz, vp]
            L.labs_legendre_pairs.restype = i32
            L.labs_legendre_pairs.argtypes = [i32, ctypes.POINTER(LegendreSweep), ctypes.POINTER(i32),
                                              ctypes.POINTER(i32), i64, ctypes.POINTER(i64)]
            L.labs_legendre_build_workspace.restype = i32
            L.labs_legendre_build_workspace.argtypes = [i64, ctypes.POINTER(sz)]
            L.labs_legendre_build.restype = i32
            L.labs_legendre_build.argtypes = [i32, i64, ctypes.POINTER(i32), ctypes.POINTER(i32), vp, vp,
                                              vp, sz, vp]
            L.labs_length_operators.restype = i32
            L.labs_length_operators.argtypes = [i32, i64, vp, vp, vp, vp, vp, vp]
            L.labs_pool_topk_workspace.restype = i32
            L.labs_pool_topk_workspace.argtypes = [i64, i32, ctypes.POINTER(sz)]
            L.labs_pool_topk.restype = i32
            L.labs_pool_topk.argtypes = [ctypes.POINTER(Pool), i32, i32, vp, vp, vp, vp, sz, vp]
            L.labs_pool_topk_noalloc.restype = i32
            L.labs_pool_topk_noalloc.argtypes = [ctypes.POINTER(Pool), i32, i32, vp, vp, vp, vp]
            L.labs_refine_step2_workspace.restype = i32
            L.labs_refine_step2_workspace.argtypes = [ctypes.POINTER(Step2Cfg), i64,
                                                      ctypes.POINTER(sz)]
            L.labs_refine_step2.restype = i32
            L.labs_refine_step2.argtypes = [ctypes.POINTER(Step2Cfg), i64, vp,
                                            ctypes.POINTER(Step2Out), vp, sz, vp]
            L.labs_autotune_step1.restype = i32
            L.labs_autotune_step1.argtypes = [ctypes.POINTER(i32), i32, i32, i32, i32, vp]
            L.labs_autotune_save.restype = i32
            L.labs_autotune_save.argtypes = [ctypes.c_char_p]
            L.labs_autotune_load.restype = i32
            L.labs_autotune_load.argtypes = [ctypes.c_char_p]
            L.labs_autotune_get.restype = i32
            L.labs_autotune_get.argtypes = [i32, i32, ctypes.POINTER(i32), ctypes.POINTER(i32)]
            L.labs_timing_enable.restype = i32
            L.labs_timing_enable.argtypes = [i32]
            L.labs_timing_reset.restype = i32
            L.labs_timing_read.restype = i32
            L.labs_timing_read.argtypes = [ctypes.c_char_p, ctypes.POINTER(ctypes.c_double),
                                           ctypes.POINTER(i64)]
            LP = ctypes.POINTER(MlpLayout)
            dbl = ctypes.c_double
            L.labs_mlp_layout_of.restype = i32
            L.labs_mlp_layout_of.argtypes = [i32, i32, LP]
            L.labs_mlp_features.restype = i32
            L.labs_mlp_features.argtypes = [i32, i64, vp, vp, vp]
            for name in ("labs_mlp_forward_workspace", "labs_mlp_grads_workspace",
                         "labs_mlp_train_workspace"):
                getattr(L, name).restype = i32
                getattr(L, name).argtypes = [LP, i64, ctypes.POINTER(sz)]
            L.labs_mlp_forward.restype = i32
            L.labs_mlp_forward.argtypes = [LP, vp, vp, i64, vp, vp, vp, sz, vp]
            L.labs_mlp_grads.restype = i32
            L.labs_mlp_grads.argtypes = [LP, vp, vp, i64, vp, vp, vp, vp, vp, vp, sz, vp]
            L.labs_mlp_adam.restype = i32
            L.labs_mlp_adam.argtypes = [LP, vp, vp, vp, vp, vp, i32, dbl, dbl, dbl, dbl, vp]
            L.labs_mlp_cast.restype = i32
            L.labs_mlp_cast.argtypes = [LP, vp, vp, vp]
            L.labs_mlp_train_step.restype = i32
            L.labs_mlp_train_step.argtypes = [LP, vp, vp, vp, vp, vp, i32, dbl, dbl, dbl, dbl, i64,
                                              vp, vp, vp, vp, vp, sz, vp]
            L.labs_learned_walk_workspace.restype = i32
            L.labs_learned_walk_workspace.argtypes = [ctypes.POINTER(Step1Cfg),
                                                      ctypes.POINTER(Proposer), ctypes.POINTER(sz)]
            L.labs_learned_walk.restype = i32
            L.labs_learned_walk.argtypes = [ctypes.POINTER(Step1Cfg), ctypes.POINTER(Proposer),
                                            ctypes.POINTER(LearnedOut), vp, sz, vp]
            _lib = L
    return _lib


def _check(status: int) -> None:
    if status != LABS_OK:
        L = lib()
        raise LabsError("%s: %s" % (L.labs_status_str(status).decode(),
                                    L.labs_last_error().decode()))


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise LabsError("no ROCm GPU is visible; the library has no CPU path")
    return torch


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _stream(device):
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _dev(t, dtype, name):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise LabsError("%s must be a device tensor" % name)
    if t.dtype != dtype or not t.is_contiguous():
        raise LabsError("%s must be a contiguous %s tensor" % (name, dtype))
    return t


def words(L: int) -> int:
    return int(lib().labs_words(L))


def abi_version() -> int:
    return int(lib().labs_abi_version())


# ---------------------------------------------------------------- timing
def timing_enable(on: bool = True) -> None:
    _check(lib().labs_timing_enable(1 if on else 0))


def timing_reset() -> None:
    _check(lib().labs_timing_reset())


def timing_read(kernel: str):
    """(total milliseconds, launches) accumulated for a timed kernel."""
    ms = ctypes.c_double(0)
    n = ctypes.c_int64(0)
    _check(lib().labs_timing_read(kernel.encode(), ctypes.byref(ms), ctypes.byref(n)))
    return float(ms.value), int(n.value)


# ---------------------------------------------------------------- energies
def energy(L: int, seqs, want_c: bool = False):
    """labs_energy over packed sequences seqs (uint32 [n, W] stored as int32)."""
    torch = _torch()
    s = _dev(seqs, torch.int32, "seqs")
    n = s.shape[0] if s.numel() else 0
    E = torch.empty(n, dtype=torch.int32, device=s.device)
    C = torch.empty((n, max(L - 1, 0)), dtype=torch.int32, device=s.device) if want_c else None
    _check(lib().labs_energy(L, n, _ptr(s), _ptr(E), _ptr(C), _stream(s.device)))
    return (E, C) if want_c else E


def flip_deltas(L: int, seqs, skew: bool = False, p: int = 0):
    torch = _torch()
    s = _dev(seqs, torch.int32, "seqs")
    n = s.shape[0] if s.numel() else 0
    width = L if not skew else (L - 1) // 2 + 1 - p
    dE = torch.empty((n, width), dtype=torch.int32, device=s.device)
    _check(lib().labs_flip_deltas(L, p, 1 if skew else 0, n, _ptr(s), _ptr(dE), _stream(s.device)))
    return dE


# ---------------------------------------------------------------- pool
@dataclass
class PoolBuffers:
    L: int
    capacity: int
    seqs: object
    E: object
    walker: object
    step: object
    count: object
    dropped: object

    @staticmethod
    def empty(L: int, capacity: int, device="cuda"):
        torch = _torch()
        W = words(L)
        return PoolBuffers(L, capacity,
                           torch.zeros((capacity, W), dtype=torch.int32, device=device),
                           torch.zeros(capacity, dtype=torch.int32, device=device),
                           torch.zeros(capacity, dtype=torch.int64, device=device),
                           torch.zeros(capacity, dtype=torch.int32, device=device),
                           torch.zeros(1, dtype=torch.int64, device=device),
                           torch.zeros(1, dtype=torch.int64, device=device))

    def struct(self) -> Pool:
        return Pool(self.seqs.data_ptr(), self.E.data_ptr(), self.walker.data_ptr(),
                    self.step.data_ptr(), self.capacity, self.count.data_ptr(),
                    self.dropped.data_ptr())


def pool_topk(pool: PoolBuffers, k: int):
    torch = _torch()
    sz = ctypes.c_size_t(0)
    _check(lib().labs_pool_topk_workspace(pool.capacity, pool.L, ctypes.byref(sz)))
    dev = pool.seqs.device
    ws = torch.empty(max(int(sz.value), 1), dtype=torch.uint8, device=dev)
    W = words(pool.L)
    out_s = torch.zeros((k, W), dtype=torch.int32, device=dev)
    out_E = torch.zeros(k, dtype=torch.int32, device=dev)
    out_n = torch.zeros(1, dtype=torch.int64, device=dev)
    ps = pool.struct()
    _check(lib().labs_pool_topk(ctypes.byref(ps), pool.L, k, _ptr(out_s), _ptr(out_E), _ptr(out_n),
                                _ptr(ws), ws.numel(), _stream(dev)))
    n = int(out_n.item())
    return out_s[:n], out_E[:n]


def pool_topk_noalloc(pool: PoolBuffers, k: int):
    """labs_pool_topk_noalloc: as pool_topk, with the library's fixed scratch
    array in place of a workspace (only the outputs are allocated here)."""
    torch = _torch()
    dev = pool.seqs.device
    W = words(pool.L)
    out_s = torch.zeros((k, W), dtype=torch.int32, device=dev)
    out_E = torch.zeros(k, dtype=torch.int32, device=dev)
    out_n = torch.zeros(1, dtype=torch.int64, device=dev)
    ps = pool.struct()
    _check(lib().labs_pool_topk_noalloc(ctypes.byref(ps), pool.L, k, _ptr(out_s), _ptr(out_E), _ptr(out_n),
                                        _stream(dev)))
    n = int(out_n.item())
    return out_s[:n], out_E[:n]


# ---------------------------------------------------------------- first step
@dataclass
class Step1Result:
    final_seqs: object
    final_E: object
    best_seqs: object
    best_E: object
    best_step: object
    traj_E: object
    flip_evals: object


def walk_step1(L: int, p: int, steps: int, tenure_lo: int, tenure_hi: int, seed: int,
               n_walkers: int, walker_begin: int = 0, e_max: int = -1,
               pool: PoolBuffers | None = None, want_traj: bool = False,
               pool_walker_best: bool = False, device="cuda", workspace=None,
               bloom: tuple | None = None, stamps: Stamps | None = None) -> Step1Result:
    """labs_walk_step1 for one configuration; with bloom = (log2_bits, n_hash),
    labs_walk_step1_bloom (tenure_lo = tenure_hi = 0).  `stamps` (a Stamps)
    receives the first-hit stamps of its levels."""
    torch = _torch()
    cfg = Step1Cfg(L, p, steps, tenure_lo, tenure_hi, e_max, walker_begin, n_walkers, seed,
                   LABS_POOL_WALKER_BEST if pool_walker_best else 0, 0)
    bc = BloomCfg(bloom[0], bloom[1]) if bloom is not None else None
    W = words(L)
    steps_eff = steps if steps else 4 * (L + 1)
    cap = pool.capacity if pool is not None else 0
    sz = ctypes.c_size_t(0)
    if bc is not None:
        _check(lib().labs_walk_step1_bloom_workspace(ctypes.byref(cfg), ctypes.byref(bc), cap,
                                                     ctypes.byref(sz)))
    else:
        _check(lib().labs_walk_step1_workspace(ctypes.byref(cfg), 1, cap, ctypes.byref(sz)))
    if workspace is None or workspace.numel() < sz.value:
        workspace = torch.empty(int(sz.value), dtype=torch.uint8, device=device)
    r = Step1Result(
        final_seqs=torch.empty((n_walkers, W), dtype=torch.int32, device=device),
        final_E=torch.empty(n_walkers, dtype=torch.int32, device=device),
        best_seqs=torch.empty((n_walkers, W), dtype=torch.int32, device=device),
        best_E=torch.empty(n_walkers, dtype=torch.int32, device=device),
        best_step=torch.empty(n_walkers, dtype=torch.int32, device=device),
        traj_E=(torch.empty((n_walkers, steps_eff), dtype=torch.int32, device=device)
                if want_traj else None),
        flip_evals=torch.zeros(1, dtype=torch.int64, device=device))
    out = Step1Out(r.final_seqs.data_ptr(), r.final_E.data_ptr(), r.best_seqs.data_ptr(),
                   r.best_E.data_ptr(), r.best_step.data_ptr(),
                   r.traj_E.data_ptr() if want_traj else None, r.flip_evals.data_ptr())
    if stamps is not None:
        stamps.fill(out)
    ps = pool.struct() if pool is not None else None
    if bc is not None:
        _check(lib().labs_walk_step1_bloom(ctypes.byref(cfg), ctypes.byref(bc),
                                           ctypes.byref(ps) if ps is not None else None,
                                           ctypes.byref(out), _ptr(workspace), workspace.numel(),
                                           _stream(torch.device(device))))
    else:
        _check(lib().labs_walk_step1(ctypes.byref(cfg), 1, None,
                                     ctypes.byref(ps) if ps is not None else None,
                                     ctypes.byref(out), _ptr(workspace), workspace.numel(),
                                     _stream(torch.device(device))))
    return r


# ---------------------------------------------------------------- Legendre seeds
def legendre_pairs(L: int, t_lo: int = 0, t_hi: int = 900, r_lo: int = 1800, r_hi: int = 2600):
    """labs_legendre_pairs: the sweep's (n, o) pairs as two int32 numpy arrays."""
    import numpy as np
    sw = LegendreSweep(t_lo, t_hi, r_lo, r_hi)
    cnt = ctypes.c_int64(0)
    _check(lib().labs_legendre_pairs(L, ctypes.byref(sw), None, None, 0, ctypes.byref(cnt)))
    n = np.zeros(max(cnt.value, 1), dtype=np.int32)
    o = np.zeros(max(cnt.value, 1), dtype=np.int32)
    i32p = ctypes.POINTER(ctypes.c_int32)
    _check(lib().labs_legendre_pairs(L, ctypes.byref(sw), n.ctypes.data_as(i32p), o.ctypes.data_as(i32p),
                                     cnt.value, ctypes.byref(cnt)))
    return n[:cnt.value], o[:cnt.value]


def legendre_build(L: int, n, o, device="cuda"):
    """labs_legendre_build: packed sequences (int32 [m, W]) and energies of the pairs."""
    import numpy as np
    torch = _torch()
    n = np.ascontiguousarray(n, dtype=np.int32)
    o = np.ascontiguousarray(o, dtype=np.int32)
    m = len(n)
    sz = ctypes.c_size_t(0)
    _check(lib().labs_legendre_build_workspace(m, ctypes.byref(sz)))
    ws = torch.empty(max(int(sz.value), 1), dtype=torch.uint8, device=device)
    seqs = torch.empty((m, words(L)), dtype=torch.int32, device=device)
    E = torch.empty(m, dtype=torch.int32, device=device)
    i32p = ctypes.POINTER(ctypes.c_int32)
    _check(lib().labs_legendre_build(L, m, n.ctypes.data_as(i32p), o.ctypes.data_as(i32p), _ptr(seqs),
                                     _ptr(E), _ptr(ws), ws.numel(), _stream(torch.device(device))))
    return seqs, E


# ---------------------------------------------------------------- end operators
def length_operators(L: int, seqs):
    """labs_length_operators: (minus [2n, W(L-1)], E_minus [2n], plus [4n, W(L+1)],
    E_plus [4n]) for packed sequences of length L (int32 [n, W] device tensor)."""
    torch = _torch()
    s = _dev(seqs, torch.int32, "seqs")
    n = s.shape[0]
    dev = s.device
    minus = torch.empty((2 * n, words(max(L - 1, 1))), dtype=torch.int32, device=dev)
    Em = torch.empty(2 * n, dtype=torch.int32, device=dev)
    plus = torch.empty((4 * n, words(L + 1)), dtype=torch.int32, device=dev)
    Ep = torch.empty(4 * n, dtype=torch.int32, device=dev)
    _check(lib().labs_length_operators(L, n, _ptr(s), _ptr(minus) if L >= 2 else None,
                                       _ptr(Em) if L >= 2 else None, _ptr(plus), _ptr(Ep), _stream(dev)))
    return minus, Em, plus, Ep


# ---------------------------------------------------------------- second step
def refine_step2(L: int, cands, batch: int, pq_capacity: int, max_expansions: int, T_u: int,
                 open_capacity: int = 0, workspace=None, T_r: int = 0):
    """labs_refine_step2 over packed candidates (int32 [n, W] device tensor).
    Returns a dict with best_seq, best_E, the stats and (optionally) Open."""
    torch = _torch()
    c = _dev(cands, torch.int32, "cands")
    n = c.shape[0]
    dev = c.device
    cfg = Step2Cfg(L, batch, T_r, 0, pq_capacity, max_expansions, T_u)
    sz = ctypes.c_size_t(0)
    _check(lib().labs_refine_step2_workspace(ctypes.byref(cfg), n, ctypes.byref(sz)))
    if workspace is None or workspace.numel() < sz.value:
        workspace = torch.empty(int(sz.value), dtype=torch.uint8, device=dev)
    W = words(L)
    best_seq = torch.zeros(W, dtype=torch.int32, device=dev)
    best_E = torch.zeros(1, dtype=torch.int32, device=dev)
    stats = torch.zeros(ctypes.sizeof(Step2Stats), dtype=torch.uint8, device=dev)
    oc = int(open_capacity)
    open_seqs = torch.zeros((max(oc, 1), W), dtype=torch.int32, device=dev)
    open_E = torch.zeros(max(oc, 1), dtype=torch.int32, device=dev)
    out = Step2Out(best_seq.data_ptr(), best_E.data_ptr(), stats.data_ptr(),
                   open_seqs.data_ptr() if oc else None, open_E.data_ptr() if oc else None, oc)
    _check(lib().labs_refine_step2(ctypes.byref(cfg), n, _ptr(c), ctypes.byref(out), _ptr(workspace),
                                   workspace.numel(), _stream(dev)))
    st = Step2Stats.from_buffer_copy(bytes(stats.cpu().numpy().tobytes()))
    res = {f: getattr(st, f) for f, _ in Step2Stats._fields_}
    res["best_seq"] = best_seq
    res["best_E_dev"] = best_E
    if oc:
        m = min(res["open_count"], oc)
        res["open_seqs"] = open_seqs[:m]
        res["open_E"] = open_E[:m]
    return res


# ---------------------------------------------------------------- batched first step
def walk_step1_batch(cfgs, want_traj: bool = False, device="cuda", workspace=None, results=None):
    """One batched launch over several configurations (dicts with L, p, steps,
    tenure_lo, tenure_hi, seed, n_walkers and optionally walker_begin).
    Returns (results, workspace); the launch is asynchronous.  Passing back the
    same results and workspace replays the captured graph."""
    torch = _torch()
    n = len(cfgs)
    arr = (Step1Cfg * n)()
    for i, c in enumerate(cfgs):
        arr[i] = Step1Cfg(c["L"], c["p"], c["steps"], c["tenure_lo"], c["tenure_hi"], -1,
                          c.get("walker_begin", 0), c["n_walkers"], c["seed"], 0, 0)
    sz = ctypes.c_size_t(0)
    _check(lib().labs_walk_step1_workspace(arr, n, 0, ctypes.byref(sz)))
    if workspace is None or workspace.numel() < sz.value:
        workspace = torch.empty(int(sz.value), dtype=torch.uint8, device=device)
    outs = (Step1Out * n)()
    res = []
    for i, c in enumerate(cfgs):
        if results is not None:
            r = results[i]
            r.flip_evals.zero_()
            outs[i] = Step1Out(r.final_seqs.data_ptr(), r.final_E.data_ptr(), r.best_seqs.data_ptr(),
                               r.best_E.data_ptr(), r.best_step.data_ptr(),
                               r.traj_E.data_ptr() if r.traj_E is not None else None,
                               r.flip_evals.data_ptr())
            res.append(r)
            continue
        L, nw = c["L"], c["n_walkers"]
        W = words(L)
        steps_eff = c["steps"] if c["steps"] else 4 * (L + 1)
        r = Step1Result(
            final_seqs=torch.empty((nw, W), dtype=torch.int32, device=device),
            final_E=torch.empty(nw, dtype=torch.int32, device=device),
            best_seqs=torch.empty((nw, W), dtype=torch.int32, device=device),
            best_E=torch.empty(nw, dtype=torch.int32, device=device),
            best_step=torch.empty(nw, dtype=torch.int32, device=device),
            traj_E=(torch.empty((nw, steps_eff), dtype=torch.int32, device=device)
                    if want_traj else None),
            flip_evals=torch.zeros(1, dtype=torch.int64, device=device))
        outs[i] = Step1Out(r.final_seqs.data_ptr(), r.final_E.data_ptr(), r.best_seqs.data_ptr(),
                           r.best_E.data_ptr(), r.best_step.data_ptr(),
                           r.traj_E.data_ptr() if want_traj else None, r.flip_evals.data_ptr())
        res.append(r)
    _check(lib().labs_walk_step1(arr, n, None, None, outs, _ptr(workspace), workspace.numel(),
                                 _stream(torch.device(device))))
    return res, workspace


def autotune_step1(Ls, p: int, walkers: int, steps: int, device="cuda") -> None:
    torch = _torch()
    arr = (ctypes.c_int32 * len(Ls))(*Ls)
    _check(lib().labs_autotune_step1(arr, len(Ls), p, walkers, steps,
                                     _stream(torch.device(device))))


def autotune_save(path: str) -> None:
    _check(lib().labs_autotune_save(path.encode()))


def autotune_load(path: str) -> None:
    _check(lib().labs_autotune_load(path.encode()))


def autotune_get(L: int, p: int):
    rb = ctypes.c_int32(0)
    wv = ctypes.c_int32(0)
    _check(lib().labs_autotune_get(L, p, ctypes.byref(rb), ctypes.byref(wv)))
    return int(rb.value), int(wv.value)


# ---------------------------------------------------------------- learned proposal network
MLP_KEYS = ("W1", "b1", "W2", "b2", "W3", "b3")


def mlp_layout(L: int, hidden: int = 256) -> MlpLayout:
    lay = MlpLayout()
    _check(lib().labs_mlp_layout_of(L, hidden, ctypes.byref(lay)))
    return lay


def _mlp_slices(lay: MlpLayout):
    h = lay.hidden
    return {"W1": (lay.off_W1, (h, lay.ld_in), (h, lay.d_in)),
            "b1": (lay.off_b1, (h,), (h,)),
            "W2": (lay.off_W2, (h, h), (h, h)),
            "b2": (lay.off_b2, (h,), (h,)),
            "W3": (lay.off_W3, (lay.ld_out, h), (lay.d_out, h)),
            "b3": (lay.off_b3, (lay.ld_out,), (lay.d_out,))}


def mlp_blob_from_dict(lay: MlpLayout, P: dict):
    """Host-side placement of {W1 [h,d_in], b1, W2 [h,h], b2, W3 [d_out,h], b3} into the
    FP32 parameter blob (numpy), pads zero."""
    import numpy as np
    blob = np.zeros(lay.n_params, np.float32)
    for key, (off, full, used) in _mlp_slices(lay).items():
        size = int(np.prod(full))
        view = blob[off:off + size].reshape(full)
        view[tuple(slice(0, u) for u in used)] = np.asarray(P[key], np.float32)
    return blob


def mlp_dict_from_blob(lay: MlpLayout, blob):
    """Inverse of mlp_blob_from_dict (numpy in, numpy out)."""
    import numpy as np
    blob = np.asarray(blob)
    out = {}
    for key, (off, full, used) in _mlp_slices(lay).items():
        size = int(np.prod(full))
        out[key] = blob[off:off + size].reshape(full)[tuple(slice(0, u) for u in used)].copy()
    return out


def mlp_features(L: int, seqs):
    torch = _torch()
    s = _dev(seqs, torch.int32, "seqs")
    lay = mlp_layout(L, 64)
    n = s.numel() // words(L)
    X = torch.empty((n, lay.ld_in), dtype=torch.bfloat16, device=s.device)
    _check(lib().labs_mlp_features(L, n, _ptr(s), _ptr(X), _stream(s.device)))
    return X


def _ws(name, lay, n, device, ws):
    torch = _torch()
    b = ctypes.c_size_t(0)
    _check(getattr(lib(), name)(ctypes.byref(lay), n, ctypes.byref(b)))
    if ws is None or ws.numel() < b.value:
        ws = torch.empty(max(1, b.value), dtype=torch.uint8, device=device)
    return ws


def mlp_forward(lay: MlpLayout, params, params_bf16, X, workspace=None):
    torch = _torch()
    n = X.shape[0]
    logits = torch.empty((n, lay.ld_out), dtype=torch.float32, device=X.device)
    ws = _ws("labs_mlp_forward_workspace", lay, n, X.device, workspace)
    _check(lib().labs_mlp_forward(ctypes.byref(lay), _ptr(params), _ptr(params_bf16), n, _ptr(X),
                                  _ptr(logits), _ptr(ws), ws.numel(), _stream(X.device)))
    return logits


def mlp_grads(lay: MlpLayout, params, params_bf16, X, mask, labels, workspace=None):
    torch = _torch()
    n = X.shape[0]
    grads = torch.empty(lay.n_params, dtype=torch.float32, device=X.device)
    loss = torch.empty(1, dtype=torch.float32, device=X.device)
    ws = _ws("labs_mlp_grads_workspace", lay, n, X.device, workspace)
    _check(lib().labs_mlp_grads(ctypes.byref(lay), _ptr(params), _ptr(params_bf16), n, _ptr(X),
                                _ptr(mask), _ptr(labels), _ptr(grads), _ptr(loss), _ptr(ws),
                                ws.numel(), _stream(X.device)))
    return grads, loss


def mlp_adam(lay: MlpLayout, params, params_bf16, grads, m, v, t: int, lr=1e-3, beta1=0.9,
             beta2=0.999, eps=1e-8):
    _check(lib().labs_mlp_adam(ctypes.byref(lay), _ptr(params), _ptr(params_bf16), _ptr(grads),
                               _ptr(m), _ptr(v), t, lr, beta1, beta2, eps, _stream(params.device)))


def mlp_cast(lay: MlpLayout, params, params_bf16):
    _check(lib().labs_mlp_cast(ctypes.byref(lay), _ptr(params), _ptr(params_bf16),
                               _stream(params.device)))


def mlp_train_step(lay: MlpLayout, params, params_bf16, grads, m, v, t: int, seqs, mask, labels,
                   lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, workspace=None, loss=None):
    torch = _torch()
    n = seqs.shape[0]
    if loss is None:
        loss = torch.empty(1, dtype=torch.float32, device=seqs.device)
    ws = _ws("labs_mlp_train_workspace", lay, n, seqs.device, workspace)
    _check(lib().labs_mlp_train_step(ctypes.byref(lay), _ptr(params), _ptr(params_bf16), _ptr(grads),
                                     _ptr(m), _ptr(v), t, lr, beta1, beta2, eps, n, _ptr(seqs),
                                     _ptr(mask), _ptr(labels), _ptr(loss), _ptr(ws), ws.numel(),
                                     _stream(seqs.device)))
    return loss, ws


# ---------------------------------------------------------------- walk with a proposer
def learned_walk(L: int, p: int, steps: int, tenure_lo: int, tenure_hi: int, seed: int,
                 n_walkers: int, mode: int = PROPOSE_MLP, top_m: int = 8, fallback_every: int = 64,
                 hidden: int = 256, params=None, params_bf16=None, prop_seed: int = 0,
                 log_every: int = 0, e_max: int = -1, walker_begin: int = 0, want_traj: bool = False,
                 want_cands: bool = False, device="cuda", workspace=None, stamps: Stamps | None = None):
    """labs_learned_walk; returns a dict of device tensors (and the workspace).
    `stamps` (a Stamps) receives the first-hit stamps of its levels."""
    torch = _torch()
    dev = torch.device(device)
    W = words(L)
    k = (L - 1) // 2
    steps = steps if steps else 4 * (L + 1)
    cfg = Step1Cfg(L, p, steps, tenure_lo, tenure_hi, e_max, walker_begin, n_walkers, seed, 0, 0)
    pr = Proposer(mode, top_m, fallback_every, hidden, _ptr(params).value, _ptr(params_bf16).value,
                  prop_seed, log_every, 0)
    b = ctypes.c_size_t(0)
    _check(lib().labs_learned_walk_workspace(ctypes.byref(cfg), ctypes.byref(pr), ctypes.byref(b)))
    if workspace is None or workspace.numel() < b.value:
        workspace = torch.empty(b.value, dtype=torch.uint8, device=dev)
    i32 = torch.int32
    r = {"final_seqs": torch.empty((n_walkers, W), dtype=i32, device=dev),
         "final_E": torch.empty(n_walkers, dtype=i32, device=dev),
         "best_seqs": torch.empty((n_walkers, W), dtype=i32, device=dev),
         "best_E": torch.empty(n_walkers, dtype=i32, device=dev),
         "best_step": torch.empty(n_walkers, dtype=i32, device=dev),
         "hit_step": torch.empty(n_walkers, dtype=i32, device=dev),
         "flip_evals": torch.zeros(1, dtype=torch.int64, device=dev)}
    if want_traj:
        r["traj_E"] = torch.empty((n_walkers, steps), dtype=i32, device=dev)
        r["moves"] = torch.empty((n_walkers, steps), dtype=i32, device=dev)
    if want_cands:
        r["cands"] = torch.empty((n_walkers, steps, top_m), dtype=torch.int16, device=dev)
    n_log = steps // log_every if log_every > 0 else 0
    if n_log:
        mw = (k + 1 + 31) // 32
        r["log_seqs"] = torch.empty((n_walkers * n_log, W), dtype=i32, device=dev)
        r["log_mask"] = torch.empty((n_walkers * n_log, mw), dtype=i32, device=dev)
        r["log_label"] = torch.empty(n_walkers * n_log, dtype=i32, device=dev)
    out = LearnedOut(*[_ptr(r.get(name)).value for name, _ in LearnedOut._fields_[:-len(_STAMP_FIELDS)]])
    if stamps is not None:
        stamps.fill(out)
    _check(lib().labs_learned_walk(ctypes.byref(cfg), ctypes.byref(pr), ctypes.byref(out),
                                   _ptr(workspace), workspace.numel(), _stream(dev)))
    r["workspace"] = workspace
    return r
