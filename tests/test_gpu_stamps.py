"""First-hit stamps of the device real-time counter (labs_step1_out and
labs_learned_out n_levels / level_E / first_hit_ticks / start_ticks).  Which
levels are hit is exact: a level is stamped iff some walker's energy (the
initial one included) reaches it, decided against the oracle's walker.  The
stamps' values are times, checked for what holds on any run: every stamp lies
between the call's start stamp and the host-timed end of the call, a lower
level is never stamped before a higher one, and the stamps accumulate over
calls that share them."""
import time

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

NEVER = (1 << 64) - 1


@pytest.fixture(scope="module")
def lb():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2409_07222_amd import labs
    labs.lib()
    return labs


def _u64(t):
    return [x & NEVER for x in t.cpu().tolist()]


def _check_times(lb, st, elapsed_s):
    hz = lb.realtime_hz()
    assert 1e6 <= hz <= 1e10
    start = _u64(st.start)[0]
    assert start != NEVER
    ticks = _u64(st.ticks)
    # levels in decreasing energy order: reaching a lower level reaches the higher ones
    order = np.argsort([-e for e in st.level_E], kind="stable")
    prev = 0
    for l in order:
        if ticks[l] == NEVER:
            prev = NEVER
            continue
        assert start <= ticks[l] <= start + int((elapsed_s + 0.05) * hz), (l, ticks[l] - start, hz)
        assert ticks[l] >= prev
        prev = ticks[l]
    return ticks


def test_walk_stamps_levels(lb, orc):
    import torch
    L, p, steps, n = 101, 8, 1500, 32
    o = orc.baseline_walk(L, p, steps, 10, 20, 5, 0, n, threads=4, want_traj=True)
    lowest = int(o["traj"].min())
    levels = [lowest - 4, lowest, lowest + 40, 10 ** 7]   # never / at the minimum / above it / at init
    st = lb.Stamps(levels)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = lb.walk_step1(L, p, steps, 10, 20, 5, n, stamps=st)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    best = int(o["best_E"].min())         # the oracle's, initial sequences included
    assert int(r.best_E.min().item()) == best
    ticks = _check_times(lb, st, el)
    for l, e in enumerate(levels):
        assert (ticks[l] != NEVER) == (best <= e), (l, e, best)
    assert ticks[0] == NEVER and ticks[1] != NEVER and ticks[3] != NEVER


def test_walk_stamps_accumulate_and_pool_mode(lb, orc):
    """Two calls (pool mode: segments and compactions) share one Stamps: the
    start is the first call's, the levels only the first walk reaches stay at
    its times, and a level only the second walk reaches is stamped after the
    first call's end."""
    import torch
    L, p, steps, n = 63, 4, 600, 16
    a = orc.baseline_walk(L, p, steps, 4, 9, 11, 0, n, threads=4, want_traj=True)
    b = orc.baseline_walk(L, p, steps, 4, 9, 12, 0, n, threads=4, want_traj=True)
    la, lbb = int(a["best_E"].min()), int(b["best_E"].min())
    levels = [max(la, lbb), min(la, lbb)]
    st = lb.Stamps(levels)
    pool = lb.PoolBuffers.empty(L, 1024)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lb.walk_step1(L, p, steps, 4, 9, 11, n, e_max=orc.e_max_for_tau(L, 3, 1), pool=pool, stamps=st)
    torch.cuda.synchronize()
    s_after_first = _u64(st.ticks)
    start_first = _u64(st.start)[0]
    lb.walk_step1(L, p, steps, 4, 9, 12, n, e_max=orc.e_max_for_tau(L, 3, 1), pool=pool, stamps=st)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ticks = _check_times(lb, st, el)
    assert _u64(st.start)[0] == start_first
    for l, e in enumerate(levels):
        if la <= e:
            assert ticks[l] == s_after_first[l] != NEVER
        else:
            assert s_after_first[l] == NEVER and ticks[l] != NEVER


def test_bloom_walk_stamps(lb, orc):
    import torch
    L, p, steps, n = 63, 4, 300, 16
    o = orc.walk_bloom(L, p, steps, 10, 3, 2, range(n))
    lowest = int(o["best_E"].min())
    levels = [lowest - 4, lowest]
    st = lb.Stamps(levels)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lb.walk_step1(L, p, steps, 0, 0, 2, n, bloom=(10, 3), stamps=st)
    torch.cuda.synchronize()
    ticks = _check_times(lb, st, time.perf_counter() - t0)
    assert ticks[0] == NEVER and ticks[1] != NEVER


@pytest.mark.parametrize("mode", ["random", "mlp"])
def test_learned_walk_stamps(lb, mode):
    """The proposer walk stamps its levels at the moves it takes (its trajectory
    decides which levels are reached)."""
    import torch
    import labs_inputs as li
    L, p, steps, n = 101, 8, 256, 32
    kw = dict(mode=lb.PROPOSE_RANDOM, prop_seed=3)
    if mode == "mlp":
        lay = lb.mlp_layout(L, 64)
        P = li.mlp_init(55, lay.d_in, 64, lay.d_out)
        blob = torch.from_numpy(lb.mlp_blob_from_dict(lay, P)).cuda()
        pb = torch.empty(lay.n_params, dtype=torch.bfloat16, device="cuda")
        lb.mlp_cast(lay, blob, pb)
        kw = dict(mode=lb.PROPOSE_MLP, hidden=64, params=blob, params_bf16=pb)
    r = lb.learned_walk(L, p, steps, 10, 20, 9, n, top_m=8, fallback_every=16, want_traj=True, **kw)
    torch.cuda.synchronize()
    lowest = int(r["traj_E"].min().item())
    levels = [lowest - 4, lowest, lowest + 24]
    st = lb.Stamps(levels)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r2 = lb.learned_walk(L, p, steps, 10, 20, 9, n, top_m=8, fallback_every=16, want_traj=True, stamps=st, **kw)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    assert torch.equal(r["traj_E"], r2["traj_E"])
    ticks = _check_times(lb, st, el)
    best = min(lowest, int(r2["best_E"].min().item()))
    for l, e in enumerate(levels):
        assert (ticks[l] != NEVER) == (best <= e)
