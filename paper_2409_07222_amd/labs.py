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


class Step1Out(ctypes.Structure):
    _fields_ = [("final_seqs", ctypes.c_void_p), ("final_E", ctypes.c_void_p),
                ("best_seqs", ctypes.c_void_p), ("best_E", ctypes.c_void_p),
                ("best_step", ctypes.c_void_p), ("traj_E", ctypes.c_void_p),
                ("flip_evals", ctypes.c_void_p)]


class Step2Cfg(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int32), ("batch", ctypes.c_int32), ("T_r", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("pq_capacity", ctypes.c_int64),
                ("max_expansions", ctypes.c_int64), ("T_u", ctypes.c_int64)]


class Step2Stats(ctypes.Structure):
    _fields_ = [("expansions", ctypes.c_int64), ("pushes", ctypes.c_int64),
                ("dup_skips", ctypes.c_int64), ("evictions", ctypes.c_int64),
                ("rounds", ctypes.c_int64), ("open_count", ctypes.c_int64),
                ("best_E", ctypes.c_int32), ("best_round", ctypes.c_int32)]


class Step2Out(ctypes.Structure):
    _fields_ = [("best_seq", ctypes.c_void_p), ("best_E", ctypes.c_void_p),
                ("stats", ctypes.c_void_p), ("open_seqs", ctypes.c_void_p),
                ("open_E", ctypes.c_void_p), ("open_capacity", ctypes.c_int64)]


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
            L.labs_pool_topk_workspace.restype = i32
            L.labs_pool_topk_workspace.argtypes = [i64, i32, ctypes.POINTER(sz)]
            L.labs_pool_topk.restype = i32
            L.labs_pool_topk.argtypes = [ctypes.POINTER(Pool), i32, i32, vp, vp, vp, vp, sz, vp]
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
               pool_walker_best: bool = False, device="cuda", workspace=None) -> Step1Result:
    torch = _torch()
    cfg = Step1Cfg(L, p, steps, tenure_lo, tenure_hi, e_max, walker_begin, n_walkers, seed,
                   LABS_POOL_WALKER_BEST if pool_walker_best else 0, 0)
    W = words(L)
    steps_eff = steps if steps else 4 * (L + 1)
    cap = pool.capacity if pool is not None else 0
    sz = ctypes.c_size_t(0)
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
    ps = pool.struct() if pool is not None else None
    _check(lib().labs_walk_step1(ctypes.byref(cfg), 1, None,
                                 ctypes.byref(ps) if ps is not None else None,
                                 ctypes.byref(out), _ptr(workspace), workspace.numel(),
                                 _stream(torch.device(device))))
    return r


# ---------------------------------------------------------------- second step
def refine_step2(L: int, cands, batch: int, pq_capacity: int, max_expansions: int, T_u: int,
                 open_capacity: int = 0, workspace=None):
    """labs_refine_step2 over packed candidates (int32 [n, W] device tensor).
    Returns a dict with best_seq, best_E, the stats and (optionally) Open."""
    torch = _torch()
    c = _dev(cands, torch.int32, "cands")
    n = c.shape[0]
    dev = c.device
    cfg = Step2Cfg(L, batch, 0, 0, pq_capacity, max_expansions, T_u)
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
