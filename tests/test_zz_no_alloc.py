"""bp_run_noalloc (static per-GPU scratch, no events) against bp_run.

The two entry points launch the same kernels with the same arguments; only
the device memory holding the run's iteration state, counters and top-k tie
counts differs.  So messages, beliefs, iteration state and statistics must be
bitwise equal.  Each case makes two calls in a row, the second on a smaller
graph, so the second call starts from whatever the first left in the shared
array (stale counters, histogram copies, tie counts).
"""
import numpy as np
import pytest

from paper_1909_11469_amd import inputs

pytestmark = pytest.mark.gpu

STAT_KEYS = ("iterations", "converged", "last_active", "last_max_residual", "evaluated",
             "committed", "final_t", "status")


@pytest.fixture(scope="module")
def bp():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1909_11469_amd import bp as mod
    return mod


def _solve(bp, prob, noalloc, **kw):
    with bp.Graph(prob) as g:
        r = g.run(noalloc=noalloc, **kw)
        m, st = g.get_state()
        b = g.marginals()
    return r, m, st, b


def _same(bp, prob, **kw):
    ra, ma, sa, ba = _solve(bp, prob, False, **kw)
    rb, mb, sb, bb = _solve(bp, prob, True, **kw)
    for k in STAT_KEYS:
        assert ra[k] == rb[k], (k, ra[k], rb[k])
    assert rb["device_ms"] == 0.0
    assert sa == sb
    assert np.array_equal(ma, mb)
    assert np.array_equal(ba, bb)
    return ra


CASES = [
    # (schedule, p, max_iters, sparse)
    ("rnbp", 0.5, 300, 0),   # dynamic p: both outputs, the four counter sets
    ("rbp", 0.05, 40, 0),    # top-k: histogram copies and tie counts in the scratch
    ("lbp", 1.0, 200, 0),
    ("rnbp", 0.3, 300, 2),   # switches to sparse re-evaluation (graph-held buffers)
    ("rbp", 1 / 256, 30, 1),
    ("rs", 1 / 64, 20, 0),     # residual splash: graph-held splash buffers, ties over variables
]


@pytest.mark.parametrize("schedule,p,max_iters,sparse", CASES)
def test_noalloc_matches_bp_run_two_calls(bp, schedule, p, max_iters, sparse):
    for side, C, seed in ((96, 1.0, 3), (40, 2.5, 4)):  # second call smaller
        prob = inputs.ising_grid(side, side, C, seed)
        _same(bp, prob, schedule=schedule, eps=1e-4, p=p, seed=11, max_iters=max_iters,
              check_every=7, sparse=sparse)


def test_noalloc_generic_layout_two_calls(bp):
    for prob in (inputs.potts_grid(24, 20, 8, 1.0, 5), inputs.potts_grid(9, 7, 8, 1.0, 6)):
        _same(bp, prob, schedule="rnbp", eps=1e-5, p=0.5, seed=2, max_iters=60, check_every=5)


def test_noalloc_warm_start_continues_like_bp_run(bp):
    prob = inputs.ising_grid(50, 50, 2.5, 8)
    res = []
    for noalloc in (False, True):
        with bp.Graph(prob) as g:
            g.run("rnbp", eps=1e-4, p=0.5, seed=1, max_iters=25, noalloc=noalloc)
            r = g.run("rnbp", eps=1e-4, p=0.5, seed=1, max_iters=25, warm_start=True,
                      noalloc=noalloc)
            res.append((r, g.get_state(), g.marginals()))
    (ra, (ma, sa), ba), (rb, (mb, sb), bb) = res
    assert all(ra[k] == rb[k] for k in STAT_KEYS)
    assert sa == sb and np.array_equal(ma, mb) and np.array_equal(ba, bb)


def test_noalloc_rejects_profile_and_unreserved_sparse(bp):
    prob = inputs.ising_grid(12, 12, 1.0, 0)
    with bp.Graph(prob) as g:
        with pytest.raises(bp.BpError) as e:
            g.run("rnbp", eps=1e-4, p=0.5, max_iters=3, profile=1, noalloc=True)
        assert e.value.code == bp.BP_EINVAL
    with bp.Graph(prob, sparse_buffers=False) as g:
        with pytest.raises(bp.BpError) as e:
            g.run("rnbp", eps=1e-4, p=0.5, max_iters=3, sparse=1, noalloc=True)
        assert e.value.code == bp.BP_EINVAL
        # the graph is still usable afterwards
        r = g.run("rnbp", eps=1e-4, p=0.5, max_iters=3, noalloc=True)
        assert r["iterations"] == 3
