"""The no-allocation top-k (labs_pool_topk_noalloc) against labs_pool_topk,
through the C ABI: two calls in a row on one GPU, the second on a smaller pool,
each bit-equal to the workspace entry point; and the size limit of its fixed
scratch, rejected on the host before any launch."""
import numpy as np
import pytest

import labs_inputs as li

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lb():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2409_07222_amd import labs
    labs.lib()
    return labs


def _pool_from(lb, L, seqs, E, cap):
    import torch
    pool = lb.PoolBuffers.empty(L, cap)
    n = len(E)
    pool.seqs[:n] = torch.from_numpy(li.pack(seqs).view(np.int32)).cuda()
    pool.E[:n] = torch.from_numpy(np.asarray(E, dtype=np.int32)).cuda()
    pool.count[0] = n
    return pool


def _random_pool(lb, orc, L, n, seed, cap):
    """n random sequences with repeats (every third one is a copy of an earlier one)."""
    S = li.random_pm1(seed, n, L)
    S[2::3] = S[0::3][: len(S[2::3])]
    E = orc.energy_batch(S)
    return _pool_from(lb, L, S, E, cap)


def _same(a, b):
    return all(x.shape == y.shape and bool((x == y).all()) for x, y in zip(a, b))


def test_noalloc_topk_matches_workspace_topk_twice(lb, orc):
    big = _random_pool(lb, orc, 501, 6000, 11, 8192)
    small = _random_pool(lb, orc, 63, 300, 12, 512)
    for pool, k in ((big, 1024), (small, 100)):
        ref = lb.pool_topk(pool, k)
        got = lb.pool_topk_noalloc(pool, k)
        assert _same(got, ref)
        assert len(got[1]) == k
    # k beyond the distinct count: everything, in key order
    ref = lb.pool_topk(small, 400)
    got = lb.pool_topk_noalloc(small, 400)
    assert _same(got, ref) and len(got[1]) < 300


def test_noalloc_topk_empty_pool(lb):
    s, E = lb.pool_topk_noalloc(lb.PoolBuffers.empty(101, 16), 4)
    assert len(E) == 0 and len(s) == 0


def test_noalloc_topk_rejects_beyond_its_scratch(lb):
    """A pool of 800,000 entries at L = 501 needs more than the 64 MiB scratch:
    rejected before any launch, with the limit in the message."""
    pool = lb.PoolBuffers.empty(501, 800_000)
    pool.count[0] = 800_000
    with pytest.raises(lb.LabsError, match="scratch"):
        lb.pool_topk_noalloc(pool, 10)
