#!/usr/bin/env python3
"""Benchmark of the dual-step hot path at L = 501 on one MI355X.

One benchmark step = one pass of the implemented hot path over a fresh seeded
batch: walker init, the first-step walk of 16,384 skew-symmetric walkers
(p = 16, tabu tenure in [L/10, L/5]) for 50,000 steps each, the F >= 8 sieve
into a 2^20-entry pool (each walker's best offered too), the pool's top 1024,
and the second step from those 1024 candidates (batch-synchronous best-first,
2^20-entry queue, 10^7 expansions).  The headline value is flip-evaluations
per second over the whole step (first-step skew flips plus second-step single
flips).  A separate instrumented pass times the dominant kernels for the
roofline; the oracle timed on the host cores gives the CPU baseline.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

L = 501
P = 16
TAU_NUM, TAU_DEN = 8, 1
METRIC = "flip-evals/sec and time-to-F>=tau at L=501, learned vs plain walker"
# Nominal integer cost of one skew flip-evaluation: 4 ops per even lag, k lags.
W_OPS = 2 * (L - 1)
# Nominal cost of one single-flip evaluation in the second step: 4 ops per lag.
W2_OPS = 4 * (L - 1)
# gfx950 integer VALU peak: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz.
PEAK_INT_OPS = 256 * 4 * 16 * 2.4e9
# Bloom filter of the first step's own walk: 2^15 bits and 8 probes per walker
# (about 5e-4 false positives per test once T_i = 4(L+1) keys are in at L = 501).
BLOOM = (15, 8)


def log(msg: str) -> None:
    """Progress on stderr (the JSON line alone goes to stdout)."""
    print("[bench] " + msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--walkers", type=int, default=16384)
    ap.add_argument("--walk-steps", type=int, default=50000)
    ap.add_argument("--s2-expansions", type=int, default=10_000_000)
    ap.add_argument("--s2-batch", type=int, default=1024)
    ap.add_argument("--s2-capacity", type=int, default=1 << 20)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--cpu-threads", type=int, default=0,
                    help="host threads of the CPU baseline (0: OMP_NUM_THREADS, else every core "
                         "this process may use)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-roofline-pass", action="store_true")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the uneven-length batched launch measurement")
    ap.add_argument("--batched-steps", type=int, default=20000)
    ap.add_argument("--no-rotations", action="store_true",
                    help="skip the second step with rotations (T_r = 1, 4, 16)")
    ap.add_argument("--rot-expansions", type=int, default=2_000_000)
    ap.add_argument("--rot-values", default="0,1,4,16", help="comma-separated T_r values")
    ap.add_argument("--no-even", action="store_true",
                    help="skip carrying the result to L - 1 and L + 1 with the end operators")
    ap.add_argument("--even-expansions", type=int, default=2_000_000)
    ap.add_argument("--no-legendre", action="store_true",
                    help="skip the Legendre-seeded second step at L = 450, 471, 491, 526")
    ap.add_argument("--legendre-expansions", type=int, default=10_000_000)
    ap.add_argument("--no-bloom", action="store_true",
                    help="skip the Bloom-filter walk measurement")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the first-step rates of the L=101 and L=451/475/527 configurations")
    ap.add_argument("--ab-seeds", type=int, default=3,
                    help="comparison seeds 1001.. (median and IQR are reported for more than one)")
    ap.add_argument("--no-ab", action="store_true",
                    help="skip the learned-vs-plain comparison at equal wall budgets")
    ap.add_argument("--ab-budget", type=float, default=6.0, help="seconds of walking per arm")
    ap.add_argument("--ab-pairs", type=int, default=10_000_000, help="logged training pairs")
    ap.add_argument("--ab-log-steps", type=int, default=4880, help="plain-walker steps logged")
    ap.add_argument("--ab-epochs", type=float, default=1.0)
    ap.add_argument("--no-counters", action="store_true",
                    help="skip the rocprofv3 counter pass of the walk kernel (the hardware roofline "
                         "fraction and HBM traffic are then null)")
    ap.add_argument("--counter-probe", default="", choices=["", "walk", "step2"],
                    help=argparse.SUPPRESS)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB five times (the reference "
                         "kernel for scaling the FETCH_SIZE / WRITE_SIZE counters) and exit")
    return ap.parse_args()


def copy_calibration(mib: int):
    import torch
    n = mib << 20
    src = torch.ones(n, dtype=torch.uint8, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes": n, "launches": 5}), flush=True)


# ---------------------------------------------------------------- counter pass
# The walk kernel's hardware work per walker-step, measured by rocprofv3 on a
# probe launch of the benchmark's walk (L = 501, p = 16, the benchmark's walker
# count, PROBE_STEPS steps, one launch) that this script runs as a child process
# before it touches the GPU itself.
PROBE_STEPS = 1024
PROBE_S2_EXPANSIONS = 500_000
PROBE_SQ = ["SQ_WAVES", "SQ_INSTS_VALU", "SQ_INSTS_SALU", "SQ_INSTS_LDS", "SQ_INSTS_LDS_LOAD_BANDWIDTH",
            "SQ_INSTS_LDS_STORE_BANDWIDTH", "SQ_INSTS_LDS_ATOMIC_BANDWIDTH", "SQ_ACTIVE_INST_VALU"]
# copy-calibrated scale of the L2 counters (a plain device copy of known size
# reads FETCH_SIZE = half the bytes it reads and WRITE_SIZE = the bytes it writes;
# profiles/walk_L501_counters.txt)
FETCH_SCALE, WRITE_SCALE = 2.0, 1.0
# gfx950 LDS: 128 bytes per clock per CU
PEAK_LDS_BYTES = 256 * 128 * 2.4e9


def counter_probe(a):
    """The child's work under rocprofv3: one walk launch of the benchmark's shape."""
    import torch
    from paper_2409_07222_amd import labs
    labs.walk_step1(L, P, PROBE_STEPS, L // 10, L // 5, 4, a.walkers)
    torch.cuda.synchronize()
    print(json.dumps({"walker_steps": a.walkers * PROBE_STEPS}), flush=True)


def counter_probe_step2(a):
    """The second step of the benchmark's shape (batch, queue capacity, seeds: the
    top-1024 of a shorter pooled walk at L = 501) for PROBE_S2_EXPANSIONS pops,
    for rocprofv3 counter and trace runs of the second step's kernels alone."""
    import torch
    from paper_2409_07222_amd import labs
    pool = labs.PoolBuffers.empty(L, 1 << 20)
    labs.walk_step1(L, P, 6000, L // 10, L // 5, 4, a.walkers, e_max=(L * L) // 16,
                    pool=pool, pool_walker_best=True)
    s, _ = labs.pool_topk(pool, 1024)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g = labs.refine_step2(L, s.contiguous(), a.s2_batch, a.s2_capacity, PROBE_S2_EXPANSIONS, 1 << 62)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    print(json.dumps({"rounds": g["rounds"], "us_per_round": dt / g["rounds"] * 1e6,
                      "pushes": g["pushes"], "best_E": g["best_E"]}), flush=True)


def _rocprof_walk(counters, walkers):
    """Counter values (summed over the dispatches of the walk kernel) of one probe
    run, or an error string."""
    import csv
    import glob
    import shutil
    import subprocess
    import tempfile
    exe = shutil.which("rocprofv3")
    if not exe:
        return "rocprofv3 not found"
    out = tempfile.mkdtemp(prefix="labs_pmc_", dir="/tmp")
    cmd = [exe, "--pmc"] + counters + ["--output-format", "csv", "-d", out, "-o", "probe", "--",
                                       sys.executable, os.path.abspath(__file__), "--counter-probe", "walk",
                                       "--walkers", str(walkers)]
    try:
        r = subprocess.run(cmd, cwd="/tmp", env=dict(os.environ, TMPDIR="/tmp"), capture_output=True,
                           text=True, timeout=180)
    except subprocess.TimeoutExpired:
        return "rocprofv3 timed out"
    files = glob.glob(os.path.join(out, "**", "*counter_collection.csv"), recursive=True)
    if r.returncode != 0 and not files:
        return "rocprofv3 exited %d: %s" % (r.returncode, (r.stderr or "")[-300:])
    vals, disp = {}, set()
    for fn in files:
        with open(fn) as f:
            for row in csv.DictReader(f):
                if "k_walk<" not in row.get("Kernel_Name", ""):
                    continue
                disp.add(row.get("Dispatch_Id") or row.get("Correlation_Id"))
                vals[row["Counter_Name"]] = vals.get(row["Counter_Name"], 0.0) + float(row["Counter_Value"])
    shutil.rmtree(out, ignore_errors=True)
    if not vals:
        return "no walk-kernel counters in the profiler output"
    vals["dispatches"] = len(disp)
    return vals


def walk_counters(a):
    """Per walker-step VALU instructions, LDS bytes and HBM bytes of the walk
    kernel, from three probe runs (the SQ set, FETCH_SIZE, WRITE_SIZE: the L2
    counters each in a run of their own)."""
    ws = a.walkers * PROBE_STEPS
    sq = _rocprof_walk(PROBE_SQ, a.walkers)
    if isinstance(sq, str):
        return {"error": sq}
    res = {"probe": "L=%d p=%d, %d walkers x %d steps, one launch" % (L, P, a.walkers, PROBE_STEPS),
           "dispatches": sq["dispatches"], "counters": {k: v for k, v in sq.items() if k != "dispatches"},
           "valu_insts_per_walker_step": sq["SQ_INSTS_VALU"] / ws,
           "lds_bytes_per_walker_step": 64.0 * sum(sq.get(k, 0.0) for k in PROBE_SQ
                                                   if k.endswith("_BANDWIDTH")) / ws}
    fb = _rocprof_walk(["FETCH_SIZE"], a.walkers)
    wb = _rocprof_walk(["WRITE_SIZE"], a.walkers)
    if isinstance(fb, dict) and isinstance(wb, dict):
        res["hbm_bytes_per_launch"] = (FETCH_SCALE * fb["FETCH_SIZE"] + WRITE_SCALE * wb["WRITE_SIZE"]) * 1024.0
    else:
        res["hbm_error"] = fb if isinstance(fb, str) else wb
    return res


def host_threads():
    """Threads the CPU baseline runs on: the OpenMP thread count the host sets
    (OMP_NUM_THREADS, the CPU share of one GPU on a shared box), else every core
    this process may run on."""
    avail = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    env = os.environ.get("OMP_NUM_THREADS", "")
    return min(int(env), avail) if env.isdigit() and int(env) > 0 else avail


def cpu_baseline(budget_s: float, threads: int):
    """CPU baseline of the first step: the oracle's linear-time tabu walker
    (oracle/labs_baseline.c: Sec. 3's O(L) neighbour evaluation, one walker per
    OpenMP thread, gcc -O3 -march=native for this host) on a bounded sample of
    the benchmark's walk (L = 501, p = 16, tenure [50, 100], seed 4): 4 walkers per
    thread, steps sized to about `budget_s` seconds.  Beside it, the definitional
    oracle walker (O(L^2) per neighbour) on one core, for reference."""
    import oracle
    k = (L - 1) // 2
    nf = k + 1 - P
    lo, hi = L // 10, L // 5
    t0 = time.perf_counter()
    oracle.baseline_lib(native=True)
    t_build = time.perf_counter() - t0
    n = 4 * threads
    t0 = time.perf_counter()
    probe = oracle.baseline_walk(L, P, 64, lo, hi, 4, 0, n, threads=threads, native=True)
    per_step = (time.perf_counter() - t0) / 64
    steps = max(64, int(budget_s / max(per_step, 1e-9)))
    t0 = time.perf_counter()
    r = oracle.baseline_walk(L, P, steps, lo, hi, 4, 0, n, threads=threads, native=True)
    dt = time.perf_counter() - t0
    # the definitional walker, one core, a few steps
    t0 = time.perf_counter()
    oracle.walk(L, P, 8, lo, hi, 4, [0], want_traj=False)
    t_def = time.perf_counter() - t0
    import platform
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), "")
    except OSError:
        pass
    return {"value": r["flip_evals"] / dt, "unit": "flip-evals/s", "cores": r["threads"],
            "kind": "oracle",
            "method": "linear-time tabu walker (Sec. 3), plain C, gcc -O3 -march=native -fopenmp, "
                      "one walker per thread",
            "sample": "%d walkers (%d per thread) x %d steps of the L=501 p=16 first-step walk "
                      "(%d flip-evals in %.1f s)" % (n, n // max(1, r["threads"]), steps,
                                                     r["flip_evals"], dt),
            "host": {"cpu_model": model, "os_cpu_count": os.cpu_count(),
                     "affinity_cpus": len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity")
                     else None, "omp_num_threads_env": os.environ.get("OMP_NUM_THREADS"),
                     "machine": platform.machine()},
            "native_build_s": t_build,
            "definitional_oracle_one_core": {"value": 8 * nf / t_def, "unit": "flip-evals/s",
                                             "sample": "1 walker x 8 steps, energy of every "
                                                       "neighbour from the definition"}}


def step1_configs(a, labs, dev):
    """First-step rates of the other single-length configurations: L = 101 (p = 8,
    65,536 walkers x 10,000 steps, tenure [10, 20], F >= 6 sieve into a 2^20 pool,
    seed 2) and L = 451 / 475 / 527 (p = 16, 16,384 walkers x 50,000 steps, F >= 8,
    walker bests offered, seed 4; L = 501 is the headline run)."""
    import torch
    out = {}
    runs = [(101, 8, 65536, 10000, 6, 2, False)] + [(x, 16, 16384, 50000, 8, 4, True)
                                                    for x in (451, 475, 527)]
    for (Lx, px, n, steps, tau, seed, wb) in runs:
        log("first step at L=%d" % Lx)
        pool = labs.PoolBuffers.empty(Lx, 1 << 20, device=dev)
        e_max = (Lx * Lx) // (2 * tau)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = labs.walk_step1(Lx, px, steps, Lx // 10, Lx // 5, seed, n, e_max=e_max, pool=pool,
                            pool_walker_best=wb, device=dev)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        fe = int(r.flip_evals.item())
        out[str(Lx)] = {"p": px, "walkers": n, "steps": steps, "tau": tau, "flip_evals": fe,
                        "seconds": dt, "flip_evals_per_s": fe / dt,
                        "pool_count": int(pool.count.item()),
                        "best_F": Lx * Lx / (2.0 * int(r.best_E.min().item()))}
        del pool, r
    return out


def batched_measure(a, labs, dev, walkers=4096, steps=None, tune=True):
    """Uneven lengths in one launch: every odd L in [301, 449] (75 lengths), `walkers`
    walkers each, p = 12, tenure [L/10, L/5], seed 3.  Tiles come from the
    autotuner (short trials first); the batched call (hipGraph capture included)
    and its replay are timed against one walk_step1 launch per length."""
    import torch
    sync = torch.cuda.synchronize
    steps = steps or a.batched_steps
    Ls = list(range(301, 450, 2))
    cfgs = [dict(L=x, p=12, steps=steps, tenure_lo=x // 10, tenure_hi=x // 5, seed=3,
                 n_walkers=walkers) for x in Ls]
    t_tune = 0.0
    if tune:
        sync()
        t0 = time.perf_counter()
        labs.autotune_step1(Ls, 12, 4096, 1000, device=dev)
        sync()
        t_tune = time.perf_counter() - t0
    t0 = time.perf_counter()
    res, ws = labs.walk_step1_batch(cfgs, device=dev)
    sync()
    t_b = time.perf_counter() - t0
    evals = sum(int(r.flip_evals.item()) for r in res)
    t0 = time.perf_counter()
    labs.walk_step1_batch(cfgs, device=dev, workspace=ws, results=res)
    sync()
    t_replay = time.perf_counter() - t0
    del res, ws
    per_L = {}
    t_s = 0.0
    for c in cfgs:
        sync()
        t0 = time.perf_counter()
        r = labs.walk_step1(c["L"], c["p"], c["steps"], c["tenure_lo"], c["tenure_hi"], c["seed"],
                            c["n_walkers"], device=dev)
        sync()
        dt = time.perf_counter() - t0
        t_s += dt
        per_L[c["L"]] = int(r.flip_evals.item()) / dt
    return {"lengths": len(Ls), "L_range": [Ls[0], Ls[-1]], "walkers_per_L": walkers, "p": 12,
            "steps": steps, "flip_evals": evals, "autotune_s": t_tune,
            "batched_s": t_b, "batched_flip_evals_per_s": evals / t_b,
            "replay_s": t_replay, "replay_flip_evals_per_s": evals / t_replay,
            "per_length_launches_s": t_s, "per_length_flip_evals_per_s": evals / t_s,
            "speedup": t_s / t_b, "speedup_replay": t_s / t_replay,
            "per_L_flip_evals_per_s": {str(k): round(v, -6) for k, v in per_L.items()}}


def bloom_measure(a, labs, dev):
    """The first step with the Bloom filter of Algorithm 1 at the bench's shape
    (L = 501, p = 16, the bench's walker count, T_i = 4(L+1) steps, 2^15 bits and
    8 probes per walker) beside the tabu walker for the same steps: kernel rate,
    its ALU fraction on the nominal count, and the best F reached."""
    import torch
    T_i = 4 * (L + 1)
    out = {"L": L, "p": P, "walkers": a.walkers, "steps": T_i,
           "bloom": {"log2_bits": BLOOM[0], "n_hash": BLOOM[1]}}
    for name, kw, kern in (("tabu", dict(tenure_lo=L // 10, tenure_hi=L // 5), "walk"),
                           ("bloom", dict(tenure_lo=0, tenure_hi=0, bloom=BLOOM), "walk_bloom")):
        for rep in range(2):
            labs.timing_reset()
            labs.timing_enable(True)
            r = labs.walk_step1(L, P, T_i, kw["tenure_lo"], kw["tenure_hi"], 31 + rep, a.walkers,
                                bloom=kw.get("bloom"), device=dev)
            torch.cuda.synchronize()
            labs.timing_enable(False)
        ms, _ = labs.timing_read(kern)
        fe = int(r.flip_evals.item())
        ach = fe * W_OPS / (ms / 1e3) / 1e12
        out[name] = {"kernel_ms": ms, "flip_evals": fe, "flip_evals_per_s": fe / (ms / 1e3),
                     "alu_frac": ach / (PEAK_INT_OPS / 1e12),
                     "best_F": L * L / (2.0 * int(r.best_E.min().item())),
                     "mean_best_F": float((L * L / (2.0 * r.best_E.double())).mean().item())}
    log("bloom walk: %.3e flip-evals/s, best F %.3f (tabu %.3f)"
        % (out["bloom"]["flip_evals_per_s"], out["bloom"]["best_F"], out["tabu"]["best_F"]))
    return out


# The paper's own results, quoted with the hardware it names (context, not targets):
# it reports solution quality only, no throughput.
PAPER_CONTEXT = {
    "highest_F": {"F": 7.7835, "L": 455, "section": "Sec. 4"},
    "largest_gain": {"F": 7.7791, "L": 493, "gain": 0.6980, "section": "Sec. 4"},
    "mean_gain_450_527": 0.2543,
    "hardware": "step 1: NVIDIA A100-SXM4-40GB (CUDA 12.2, C++); step 2: Rust on a 4-core "
                "ARM Neoverse-N1; all skew-symmetric lengths 450..527 in a few hours",
    "walk_length": "T_i = 4(L+1)",
}

# Sec. 4.1 table: merit factor of the best construction and after the second step
# ("DFS") seeded with the constructions, at four lengths (the paper's numbers).
LEGENDRE_TABLE = {450: (6.1976, 6.3088), 471: (6.2332, 6.2998), 491: (6.4292, 6.4292),
                  526: (6.3240, 6.3240)}


def legendre_step2(a, labs, dev):
    """The second step seeded with the Legendre-construction sweep (Sec. 4.1) at the
    four tabulated lengths: the sweep's sequences and energies are built on the
    device, then the second step runs from all of them (batch 1024, queue 2^20,
    --legendre-expansions pops)."""
    import torch
    out = {"expansions": a.legendre_expansions, "batch": 1024, "queue": 1 << 20, "lengths": {}}
    for Lq, (f_con, f_dfs) in LEGENDRE_TABLE.items():
        n, o = labs.legendre_pairs(Lq)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        seqs, E = labs.legendre_build(Lq, n, o, device=dev)
        torch.cuda.synchronize()
        t_build = time.perf_counter() - t0
        e0 = int(E.min().item())
        t0 = time.perf_counter()
        r = labs.refine_step2(Lq, seqs, 1024, 1 << 20, a.legendre_expansions, 1 << 62)
        torch.cuda.synchronize()
        t_s2 = time.perf_counter() - t0
        out["lengths"][str(Lq)] = {
            "pairs": int(len(n)), "build_s": t_build, "construction_F": Lq * Lq / (2.0 * e0),
            "second_step_F": Lq * Lq / (2.0 * r["best_E"]), "second_step_s": t_s2,
            "paper_construction_F": f_con, "paper_dfs_F": f_dfs,
            "neighbour_evals_per_s": r["expansions"] * Lq / t_s2,
            "rounds_to_best": r["best_round"] + 1}
        log("legendre L=%d: construction F %.4f -> second step F %.4f (paper %.4f -> %.4f)"
            % (Lq, Lq * Lq / (2.0 * e0), Lq * Lq / (2.0 * r["best_E"]), f_con, f_dfs))
    return out


def even_lengths(a, labs, dev, top_seqs, best_seq):
    """The end operators carry the dual-step result to the even lengths L - 1 and
    L + 1 (Sec. 3): the second step's best and the first step's top-k, each with
    its first or last element removed (L - 1) or with +1 / -1 put at either end
    (L + 1), seed the second step at that length (batch 1024, queue 2^20,
    --even-expansions pops)."""
    import torch
    seqs = torch.cat([best_seq.view(1, -1), top_seqs]).contiguous()
    minus, Em, plus, Ep = labs.length_operators(L, seqs)
    out = {"inputs": int(seqs.shape[0]), "expansions": a.even_expansions}
    for Lq, cand, Ec in ((L - 1, minus, Em), (L + 1, plus, Ep)):
        e0 = int(Ec.min().item())
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = labs.refine_step2(Lq, cand.contiguous(), 1024, 1 << 20, a.even_expansions, 1 << 62)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out[str(Lq)] = {"candidates": int(cand.shape[0]), "candidate_F": Lq * Lq / (2.0 * e0),
                        "second_step_F": Lq * Lq / (2.0 * r["best_E"]), "second_step_s": dt}
        log("even lengths: L=%d candidates F %.4f -> second step F %.4f"
            % (Lq, Lq * Lq / (2.0 * e0), Lq * Lq / (2.0 * r["best_E"])))
    return out


def rotations_measure(a, labs, dev, top_seqs):
    """MAKE_ROTATIONS in the second step at L = 501: from the first step's top-k,
    the second step at each T_r of --rot-values (default 0, 1, 4, 16; batch 1024,
    queue 2^20, --rot-expansions pops): time per round and best F."""
    import torch
    out = {"expansions": a.rot_expansions, "runs": {}}
    for T_r in [int(x) for x in a.rot_values.split(",")]:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = labs.refine_step2(L, top_seqs.contiguous(), 1024, 1 << 20, a.rot_expansions, 1 << 62, T_r=T_r)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out["runs"][str(T_r)] = {"seconds": dt, "rounds": r["rounds"], "us_per_round": dt / max(1, r["rounds"]) * 1e6,
                                 "pushes": r["pushes"], "best_F": L * L / (2.0 * r["best_E"])}
        log("rotations T_r=%d: %.1f us per round, best F %.4f" % (T_r, dt / max(1, r["rounds"]) * 1e6,
                                                                 L * L / (2.0 * r["best_E"])))
    return out


def learned_ab(a, labs, dev):
    """Learned proposal against the plain walker at equal wall budgets (L = 501,
    p = 16, the bench's walker count): log plain-walker pairs (seed 5), train the
    network (init seed 55, Adam lr 1e-3, batch 4096), fix tau* from a plain run of
    half the budget (seed 999, best F rounded down to 0.05), then run each arm for
    the budget from seeds 1001.. (--ab-seeds): the plain walker, the trained
    network (top-8, a full scan every 64 steps), the untrained network and a
    random top-8.  The time to reach F >= tau* (and each ladder level) is read
    from the device's real-time counter: the walker kernels stamp the first step
    at which any walker reaches the level, against the stamp of the walker-init
    kernel that starts the arm.  A further arm runs the paper's own first step,
    the Bloom-filter walk of T_i = 4(L+1) steps, in batches of fresh walkers for
    the same budget (times from the first batch's start)."""
    import numpy as np
    import torch
    import labs_inputs as li
    from paper_2409_07222_amd import learn
    lo, hi = L // 10, L // 5
    n = a.walkers
    sync = torch.cuda.synchronize
    res = {"L": L, "p": P, "walkers": n, "top_m": 8, "fallback_every": 64, "hidden": 256,
           "budget_s": a.ab_budget}
    # training data and held-out states
    log_every = max(1, (n * a.ab_log_steps) // max(1, a.ab_pairs))
    sync()
    t0 = time.perf_counter()
    seqs, mask, lab = learn.log_plain(L, P, a.ab_log_steps, lo, hi, 5, n, log_every, device=dev)
    sync()
    res["log"] = {"pairs": int(seqs.shape[0]), "steps": a.ab_log_steps, "log_every": log_every,
                  "seconds": time.perf_counter() - t0}
    hs, hm, hl = learn.log_plain(L, P, 2000, lo, hi, 6, 1024, 100, device=dev)
    lay = labs.mlp_layout(L, 256)
    net = learn.Network(L, li.mlp_init(55, lay.d_in, 256, lay.d_out), 256, device=dev)
    untrained = net.clone()
    log("comparison: %d logged pairs" % int(seqs.shape[0]))
    sync()
    t0 = time.perf_counter()
    hist = learn.train(net, seqs, mask, lab, batch=4096, epochs=a.ab_epochs, lr=1e-3)
    sync()
    t_train = time.perf_counter() - t0
    res["train"] = {"steps": net.t, "seconds": t_train, "loss_first": hist[0][1],
                    "loss_last": hist[-1][1],
                    "samples_per_s": net.t * 4096 / t_train,
                    "tflops": net.t * 4096 * 3 * 644096 / t_train / 1e12}
    del seqs, mask, lab
    # recall of the logged move among the top-8 admissible scores, held-out states
    mk = hm.cpu().numpy().view(np.uint32)
    adm = np.zeros((mk.shape[0], lay.d_out), bool)
    for j in range(lay.d_out):
        adm[:, j] = (mk[:, j // 32] >> np.uint32(j % 32)) & 1
    labels = hl.cpu().numpy()

    def recall(z):
        z = np.where(adm, z[:, :lay.d_out], -np.inf)
        top = np.argsort(-z, axis=1, kind="stable")[:, :8]
        return float(np.mean([labels[i] in top[i] for i in range(len(labels))]))
    res["recall_at_8"] = {"trained": recall(net.logits(hs).cpu().numpy()),
                          "untrained": recall(untrained.logits(hs).cpu().numpy()),
                          "random": recall(np.random.default_rng(0).random(adm.shape))}

    ladder = [5.2, 5.3, 5.4, 6.0, 6.5, 7.0, 7.5, 8.0]

    def stamps_for(e_max):
        # first-hit stamps of the device real-time counter: tau* first, then the ladder
        lv = ([e_max] if e_max >= 0 else []) + [int(np.floor(L * L / (2.0 * tl))) for tl in ladder]
        return labs.Stamps(lv[:labs.MAX_LEVELS], device=dev)

    def stamp_times(st, e_max):
        sec = st.seconds()
        off = 1 if e_max >= 0 else 0
        return (sec[0] if e_max >= 0 else None), {str(tl): sec[off + i] for i, tl in enumerate(ladder)
                                                  if off + i < len(sec)}

    def plain_run(steps, seed, e_max, tau_star=None):
        # device stamps give the times; the pool (sieve at the lowest ladder level)
        # gives each level's first hit step as a cross-check
        e_pool = max(e_max, int(np.floor(L * L / (2.0 * ladder[0])))) if e_max >= 0 else -1
        pool = labs.PoolBuffers.empty(L, 1 << 20, device=dev)
        st = stamps_for(e_max)
        sync()
        t0 = time.perf_counter()
        r = labs.walk_step1(L, P, steps, lo, hi, seed, n, e_max=e_pool, pool=pool, device=dev, stamps=st)
        sync()
        dt = time.perf_counter() - t0
        c = int(pool.count.item())
        pE = pool.E[:c].cpu().numpy()
        pS = pool.step[:c].cpu().numpy()

        def first(em):
            sel = pS[pE <= em]
            return int(sel.min()) if sel.size else None
        hits = {str(tl): first(int(np.floor(L * L / (2.0 * tl)))) for tl in ladder}
        tt, lt = stamp_times(st, e_max)
        return {"seconds": dt, "steps": steps, "best_E": int(r.best_E.min().item()),
                "hit_step": first(e_max) if e_max >= 0 else None, "ladder_hit_steps": hits,
                "time_to_tau_s": tt, "ladder_time_s": lt,
                "flip_evals": int(r.flip_evals.item()), "pool_dropped": int(pool.dropped.item())}

    T_i = 4 * (L + 1)

    def bloom_run(budget_s, seed, e_max):
        # Algorithm 1 as the paper runs it: every walker stops after T_i = 4(L+1)
        # steps, so fresh batches of walkers (new ids) are launched until the
        # budget is spent; a level's hit time is the start of the batch that first
        # reaches it plus the fraction of that batch up to its earliest hit step
        # one set of stamps over every batch: times from the first batch's start
        st = stamps_for(e_max)
        t_total, b, best, flips = 0.0, 0, None, 0
        while t_total < budget_s:
            sync()
            t0 = time.perf_counter()
            r = labs.walk_step1(L, P, T_i, 0, 0, seed, n, walker_begin=b * n, bloom=BLOOM, device=dev,
                                stamps=st)
            sync()
            dt = time.perf_counter() - t0
            e = int(r.best_E.min().item())
            best = e if best is None or e < best else best
            flips += int(r.flip_evals.item())
            t_total += dt
            b += 1
        tt, lt = stamp_times(st, e_max)
        return {"seconds": t_total, "steps": b * T_i, "batches": b, "steps_per_walk": T_i,
                "bloom": {"log2_bits": BLOOM[0], "n_hash": BLOOM[1]}, "best_E": best,
                "time_to_tau_s": tt, "ladder_time_s": lt, "flip_evals": flips}

    def learned_run(steps, seed, e_max, kw):
        st = stamps_for(e_max)
        sync()
        t0 = time.perf_counter()
        r = labs.learned_walk(L, P, steps, lo, hi, seed, n, top_m=8, fallback_every=64, e_max=e_max,
                              device=dev, stamps=st, **kw)
        sync()
        dt = time.perf_counter() - t0
        h = r["hit_step"]
        h = h[h >= 0]
        tt, lt = stamp_times(st, e_max)
        return {"seconds": dt, "steps": steps, "best_E": int(r["best_E"].min().item()),
                "hit_step": int(h.min().item()) if h.numel() else None,
                "time_to_tau_s": tt, "ladder_time_s": lt,
                "flip_evals": int(r["flip_evals"].item())}

    arms = {"learned": net.proposer_args(), "untrained": untrained.proposer_args(),
            "random_top8": dict(mode=labs.PROPOSE_RANDOM, prop_seed=7)}
    # time per step of each arm from short probes (graph capture included in a warm call)
    plain_run(64, 11, -1)
    pr = plain_run(2048, 12, -1)
    rate = {"plain": pr["steps"] / pr["seconds"]}
    for name, kw in arms.items():
        learned_run(128, 11, -1, kw)
        q = learned_run(1024, 12, -1, kw)
        rate[name] = q["steps"] / q["seconds"]
    # measured cost of one walker-step per arm (16,384 walkers in lockstep): the plain
    # step scans every neighbour exactly; a proposal step rescoring m candidates costs
    # the random arm's step without a network, and the network pass adds the rest
    res["step_cost_us"] = {name: 1e6 / r for name, r in rate.items()}
    res["step_cost_us"]["network_per_step"] = \
        1e6 / rate["learned"] - 1e6 / rate["random_top8"]
    # tau* from a plain run of half the budget
    cal = plain_run(max(64, int(rate["plain"] * a.ab_budget / 2)), 999, -1)
    tau = np.floor(L * L / (2.0 * cal["best_E"]) / 0.05) * 0.05
    e_max = int(np.floor(L * L / (2.0 * tau)))
    res["tau_star"] = float(round(tau, 2))
    res["e_max"] = e_max
    log("comparison: tau* = %.2f, %d seed(s) of %.1f s per arm" % (tau, max(1, a.ab_seeds), a.ab_budget))
    per_seed = []
    for seed in range(1001, 1001 + max(1, a.ab_seeds)):
        out = {}
        steps = max(64, int(rate["plain"] * a.ab_budget))
        out["plain"] = plain_run(steps, seed, e_max)
        log("seed %d plain: best E %d" % (seed, out["plain"]["best_E"]))
        out["bloom"] = bloom_run(a.ab_budget, seed, e_max)
        log("seed %d bloom: best E %d" % (seed, out["bloom"]["best_E"]))
        for name, kw in arms.items():
            steps = max(64, int(rate[name] * a.ab_budget))
            steps -= steps % 64
            out[name] = learned_run(steps, seed, e_max, kw)
            log("seed %d %s: best E %d" % (seed, name, out[name]["best_E"]))
        for name, o in out.items():
            o["best_F"] = L * L / (2.0 * o["best_E"])
            if o.get("hit_step") is not None:
                # the older estimate (hit step x mean time per step), beside the stamps
                o["time_to_tau_from_steps_s"] = o["hit_step"] / o["steps"] * o["seconds"]
            o["walker_steps_per_s"] = n * o["steps"] / o["seconds"]
            o["flip_evals_per_s"] = o["flip_evals"] / o["seconds"]
        per_seed.append(out)
    res["arms"] = per_seed[0]
    if len(per_seed) > 1:
        # time to tau* per seed; runs that never reach it count as censored at the budget
        summary = {}
        for name in per_seed[0]:
            tt = [s[name]["time_to_tau_s"] for s in per_seed]
            vals = np.array([x if x is not None else a.ab_budget for x in tt])
            bf = np.array([s[name]["best_F"] for s in per_seed])
            summary[name] = {"time_to_tau_median_s": float(np.median(vals)),
                             "time_to_tau_iqr_s": [float(np.percentile(vals, 25)),
                                                   float(np.percentile(vals, 75))],
                             "censored": int(sum(x is None for x in tt)),
                             "best_F_median": float(np.median(bf)),
                             "best_F_iqr": [float(np.percentile(bf, 25)), float(np.percentile(bf, 75))]}
        res["seeds"] = [1001, 1000 + len(per_seed)]
        res["summary"] = summary
    return res


def main():
    a = parse()
    if a.copy_calibration:
        copy_calibration(a.copy_calibration)
        return
    if a.counter_probe == "step2":
        counter_probe_step2(a)
        return
    if a.counter_probe:
        counter_probe(a)
        return
    if a.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(walkers would shard across GPUs by walker-id range)", file=sys.stderr)
        sys.exit(2)
    # the counter pass runs in child processes before this one touches the GPU
    counters = None
    if not a.no_counters and not a.no_roofline_pass:
        log("counter pass of the walk kernel (rocprofv3)")
        counters = walk_counters(a)
        log("counter pass: %s" % ({k: counters[k] for k in ("valu_insts_per_walker_step",
                                                            "lds_bytes_per_walker_step")
                                   if k in counters} or counters))
    import torch
    from paper_2409_07222_amd import labs
    import labs_inputs  # noqa: F401  (seeded inputs live in the library's own RNG streams)

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    k = (L - 1) // 2
    nf = k + 1 - P
    lo, hi = L // 10, L // 5
    e_max = (L * L * TAU_DEN) // (2 * TAU_NUM)
    cap, topk = 1 << 20, 1024
    pool = labs.PoolBuffers.empty(L, cap, device=dev)
    cfg_ws = None

    s2_ws = None

    top = {}

    def one(seed):
        nonlocal cfg_ws, s2_ws
        pool.count.zero_()
        pool.dropped.zero_()
        r = labs.walk_step1(L, P, a.walk_steps, lo, hi, seed, a.walkers, e_max=e_max, pool=pool,
                            pool_walker_best=True, device=dev, workspace=cfg_ws)
        s, E = labs.pool_topk(pool, topk)
        top["seqs"] = s
        if a.s2_expansions > 0:
            if s2_ws is None:
                cfg2 = labs.Step2Cfg(L, a.s2_batch, 0, 0, a.s2_capacity, a.s2_expansions, 1 << 62)
                sz2 = ctypes.c_size_t(0)
                labs._check(labs.lib().labs_refine_step2_workspace(ctypes.byref(cfg2), topk,
                                                                   ctypes.byref(sz2)))
                s2_ws = torch.empty(int(sz2.value), dtype=torch.uint8, device=dev)
            r2 = labs.refine_step2(L, s.contiguous(), a.s2_batch, a.s2_capacity, a.s2_expansions,
                                   1 << 62, workspace=s2_ws)
        else:
            r2 = {"expansions": 0, "best_E": int(E[0].item())}
        top["best"] = r2.get("best_seq")
        return r, E, r2

    # workspace reuse across steps
    import ctypes
    cfg = labs.Step1Cfg(L, P, a.walk_steps, lo, hi, e_max, 0, a.walkers, 0, 1, 0)
    sz = ctypes.c_size_t(0)
    labs._check(labs.lib().labs_walk_step1_workspace(ctypes.byref(cfg), 1, cap, ctypes.byref(sz)))
    cfg_ws = torch.empty(int(sz.value), dtype=torch.uint8, device=dev)

    for i in range(a.warmup):
        one(1000 + i)
    torch.cuda.synchronize()
    evals = evals1 = evals2 = 0
    best_E = best1_E = None
    t0 = time.perf_counter()
    for i in range(a.steps):
        r, E, r2 = one(4 + i)
        e1 = int(r.flip_evals.item())
        e2 = int(r2["expansions"]) * L
        evals1 += e1
        evals2 += e2
        evals += e1 + e2
        e = int(E[0].item()) if E.numel() else None
        if e is not None and (best1_E is None or e < best1_E):
            best1_E = e
        e = int(r2["best_E"])
        if best_E is None or e < best_E:
            best_E = e
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0

    roof = None
    if not a.no_roofline_pass:
        labs.timing_reset()
        labs.timing_enable(True)
        tr0 = time.perf_counter()
        r, _, r2 = one(2000)
        torch.cuda.synchronize()
        t_pass = time.perf_counter() - tr0
        labs.timing_enable(False)
        ms, launches = labs.timing_read("walk")
        ms2, launches2 = labs.timing_read("expand")
        fe = int(r.flip_evals.item())
        wsteps = fe / nf                       # walker-steps over the pass's walk launches
        peak = PEAK_INT_OPS / 1e12
        nominal = fe * W_OPS / (ms / 1e3) / 1e12
        roof = {"bound": "alu", "achieved": None, "peak": peak, "unit": "Tops/s", "frac": None,
                "traffic": None, "kernel": "k_walk<8,4,4> (walk)", "launches": launches,
                "avg_launch_ms": ms / max(launches, 1), "kernel_share_of_pass": ms / 1e3 / t_pass,
                "nominal": {"ops_per_flip_eval": W_OPS, "achieved_Tops": nominal,
                            "ratio_to_peak": nominal / peak,
                            "note": "direct-formula op count; the bit-sliced scan does fewer"}}
        if counters and "valu_insts_per_walker_step" in counters:
            lane_ops = counters["valu_insts_per_walker_step"] * 64.0 * wsteps
            achieved = lane_ops / (ms / 1e3) / 1e12
            lds_bps = counters["lds_bytes_per_walker_step"] * wsteps / (ms / 1e3)
            roof.update({"achieved": achieved, "frac": max(achieved / peak, lds_bps / PEAK_LDS_BYTES),
                         "valu_frac": achieved / peak,
                         "lds": {"achieved_TBps": lds_bps / 1e12, "peak_TBps": PEAK_LDS_BYTES / 1e12,
                                 "frac": lds_bps / PEAK_LDS_BYTES},
                         "per_walker_step": {"valu_insts": counters["valu_insts_per_walker_step"],
                                             "lds_bytes": counters["lds_bytes_per_walker_step"]}})
            if "hbm_bytes_per_launch" in counters:
                roof["traffic"] = counters["hbm_bytes_per_launch"]
        roof["counters"] = counters
        if launches2:
            ops2 = int(r2["expansions"]) * L * W2_OPS
            a2 = ops2 / (ms2 / 1e3) / 1e12
            roof["step2_expand"] = {"nominal_Tops": a2, "nominal_ratio_to_peak": a2 / peak,
                                    "launches": launches2, "avg_launch_ms": ms2 / launches2,
                                    "ops_per_neighbour_eval": W2_OPS,
                                    "kernel_share_of_pass": ms2 / 1e3 / t_pass}

    log("dual-step passes done: %.3e flip-evals/s" % (evals / dt))
    batched = batched_small = None
    if not a.no_batched:
        batched = batched_measure(a, labs, dev)
        # small work per length: 256 walkers x 4000 steps, where one launch per length
        # leaves most of the GPU idle
        batched_small = batched_measure(a, labs, dev, walkers=256, steps=4000, tune=False)
        log("batched: %.2fx at 4096 walkers per length, %.2fx at 256 (replay %.2fx)"
            % (batched["speedup"], batched_small["speedup"], batched_small["speedup_replay"]))
    configs = None if a.no_configs else step1_configs(a, labs, dev)
    bloom = None if a.no_bloom else bloom_measure(a, labs, dev)
    legendre = None if a.no_legendre else legendre_step2(a, labs, dev)
    even = None
    if not a.no_even and top.get("best") is not None:
        even = even_lengths(a, labs, dev, top["seqs"], top["best"])
    rot = None if a.no_rotations else rotations_measure(a, labs, dev, top["seqs"])
    ab = None
    if not a.no_ab:
        s2_ws = None
        torch.cuda.empty_cache()
        ab = learned_ab(a, labs, dev)
    cpu = None if a.no_cpu_baseline else cpu_baseline(a.cpu_seconds, a.cpu_threads or host_threads())
    value = evals / dt
    line = {
        "metric": METRIC, "value": value, "unit": "flip-evals/s", "n_gpus": 1,
        "steps": a.steps, "warmup": a.warmup, "ms_per_step": dt * 1e3 / a.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": "dual step at L=501: first step p=16, tenure [50,100], %d walkers x "
                               "%d steps, F>=8 sieve into a 2^20 pool with walker bests, top-1024; "
                               "second step from the top-1024, batch %d, queue %d, %d expansions"
                               % (a.walkers, a.walk_steps, a.s2_batch, a.s2_capacity,
                                  a.s2_expansions),
                   "L": L, "p": P, "walkers": a.walkers, "walk_steps": a.walk_steps,
                   "tau": TAU_NUM / TAU_DEN, "pool_capacity": cap, "topk": topk,
                   "s2_batch": a.s2_batch, "s2_capacity": a.s2_capacity,
                   "s2_expansions": a.s2_expansions,
                   "parallelism": "single GPU"},
        "best_F": (L * L / (2.0 * best_E)) if best_E else None,
        "best_F_step1": (L * L / (2.0 * best1_E)) if best1_E else None,
        "step1_flip_evals_per_s": evals1 / dt, "step2_neighbour_evals_per_s": evals2 / dt,
        "time_to_tau_s": ({k: v["time_to_tau_s"] for k, v in ab["arms"].items()} if ab else None),
        "tau_star": ab["tau_star"] if ab else None,
        "learned_ab": ab,
        "batched_uneven_L": batched,
        "batched_uneven_L_small": batched_small,
        "step1_configs": configs,
        "bloom_walk": bloom,
        "legendre_seeded_step2": legendre,
        "even_lengths": even,
        "step2_rotations": rot,
        "paper_context": PAPER_CONTEXT,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
