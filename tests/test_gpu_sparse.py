"""Sparse re-evaluation (bp_run_opts.sparse) against the full evaluation.

An iteration of the sparse path evaluates again only the messages out of
nodes that received a committed message; every other candidate and residual is
kept from the iteration that computed it.  The re-evaluated messages use the
same arithmetic on the same inputs as the full evaluation, so a sparse run must
give bitwise the same messages, beliefs, iteration and commit counts, n_t and
R_t as the full evaluation, while evaluating fewer messages.  Parity with the
oracle follows from that of the full evaluation; one sparse RnBP iteration is
also checked against the oracle directly.
"""
import numpy as np
import pytest

import oracle
from paper_1909_11469_amd import inputs

pytestmark = pytest.mark.gpu

SWEEP_TOL = 1e-6
BAND = 1e-6
SAME = ("iterations", "converged", "last_active", "last_max_residual", "committed", "final_t",
        "status")


@pytest.fixture(scope="module")
def bp():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1909_11469_amd import bp as mod
    return mod


def _run(bp, prob, sparse, schedule="rnbp", **kw):
    with bp.Graph(prob) as g:
        r = g.run(schedule, sparse=sparse, **kw)
        m, st = g.get_state()
        marg = g.marginals()
    return r, m, st, marg


def _assert_same(a, b):
    ra, ma, sa, ga = a
    rb, mb, sb, gb = b
    for k in SAME:
        assert ra[k] == rb[k], (k, ra[k], rb[k])
    assert np.array_equal(ma, mb)
    assert np.array_equal(ga, gb)
    assert sa == sb


PROBS = {
    "grid_C1": lambda: inputs.ising_grid(37, 45, 1.0, 3),
    "grid_C2.5": lambda: inputs.ising_grid(40, 40, 2.5, 4),
    "er": lambda: inputs.er_graph(3000, 6.0, 2.5, 1),
    "chain": lambda: inputs.chain(5000, 2.0, 2),
}


@pytest.mark.parametrize("name", sorted(PROBS))
@pytest.mark.parametrize("dynamic_p,p", [(True, 0.3), (True, 0.7), (False, 0.5)])
def test_sparse_bitwise_equals_full(bp, name, dynamic_p, p):
    prob = PROBS[name]()
    kw = dict(eps=1e-4, p=p, seed=9, max_iters=150, check_every=4, dynamic_p=dynamic_p)
    full = _run(bp, prob, 0, **kw)
    for sparse in (1, 2):
        got = _run(bp, prob, sparse, **kw)
        _assert_same(full, got)
        assert got[0]["evaluated"] <= full[0]["evaluated"]
    if name in ("grid_C1", "chain"):
        # converging: after the first iteration only the out-messages of nodes
        # that received a commit are evaluated
        assert _run(bp, prob, 1, **kw)[0]["evaluated"] < full[0]["evaluated"]


@pytest.mark.parametrize("name", ["grid_C1", "grid_C2.5", "er"])
@pytest.mark.parametrize("p", [1 / 256, 0.05, 0.5, 1.0])
def test_sparse_rbp_bitwise_equals_full(bp, name, p):
    # frontier residual BP: the top-k reads every stored residual, which the
    # sparse path keeps equal to what the full evaluation recomputes
    prob = PROBS[name]()
    kw = dict(eps=1e-4, p=p, max_iters=60, check_every=4)
    full = _run(bp, prob, 0, "rbp", **kw)
    for sparse in (1, 2):
        got = _run(bp, prob, sparse, "rbp", **kw)
        _assert_same(full, got)
        assert got[0]["evaluated"] <= full[0]["evaluated"]


def test_sparse_switch_happens_and_saves(bp):
    # a converging grid: n_t falls below E / 16, the run switches to the sparse
    # path and evaluates fewer messages than the full evaluation
    prob = inputs.ising_grid(60, 50, 1.0, 7)
    kw = dict(eps=1e-5, p=0.3, seed=4, max_iters=2000, check_every=2)
    full = _run(bp, prob, 0, **kw)
    auto = _run(bp, prob, 2, **kw)
    assert full[0]["converged"]
    _assert_same(full, auto)
    assert auto[0]["evaluated"] < full[0]["evaluated"]


@pytest.mark.parametrize("schedule", ["rnbp", "rbp"])
@pytest.mark.parametrize("first,second", [(0, 1), (1, 0), (1, 1), (2, 2)])
def test_sparse_warm_start_continuation(bp, schedule, first, second):
    prob = inputs.ising_grid(33, 29, 2.5, 5)
    kw = dict(eps=1e-4, p=0.4, seed=21, check_every=3)
    ref = _run(bp, prob, 0, schedule, max_iters=80, **kw)
    with bp.Graph(prob) as g:
        r1 = g.run(schedule, sparse=first, max_iters=35, **kw)
        r2 = g.run(schedule, sparse=second, max_iters=45, warm_start=True, **kw)
        m, st = g.get_state()
        marg = g.marginals()
    assert r1["iterations"] + r2["iterations"] == ref[0]["iterations"]
    assert r1["committed"] + r2["committed"] == ref[0]["committed"]
    assert r2["last_active"] == ref[0]["last_active"]
    assert r2["last_max_residual"] == ref[0]["last_max_residual"]
    assert np.array_equal(m, ref[1]) and np.array_equal(marg, ref[3]) and st == ref[2]


def test_sparse_one_iteration_against_oracle(bp):
    prob = inputs.ising_grid(30, 30, 2.5, 2)
    E = 2 * len(prob["edges"])
    rng = np.random.default_rng(5)
    m = rng.uniform(0.3, 1.0, size=(E, 2))
    state = (m / m.sum(1, keepdims=True)).astype(np.float32)
    eps, p, seed, t, prev = 0.05, 0.4, 1234, 7, 10 ** 6
    with bp.Graph(prob) as g:
        g.set_state(state, t=t, prev_active=prev)
        start, _ = g.get_state()
        r = g.run("rnbp", eps=eps, p=p, seed=seed, max_iters=1, warm_start=True, sparse=1)
        got, st = g.get_state()
    changed = np.any(got != start, axis=1)
    cand, res = oracle.evaluate(prob, start.astype(np.float64))
    src, _ = oracle.canonical_src_dst(prob)
    rank = oracle.neighbour_rank(prob)
    u = np.array([oracle.uniform(seed, src[e], rank[e], t) for e in range(E)])
    n_t = int((res > eps).sum())
    p_t = p if n_t / prev > 0.9 else 1.0
    want = (res > eps) & (u < p_t)
    band = np.abs(res - eps) < BAND
    assert np.array_equal(changed[~band], want[~band])
    assert band.sum() <= 3
    sel = want & ~band
    d = np.max(np.abs(got[sel].astype(np.float64) - cand[sel]), axis=1)
    assert (d / np.max(np.abs(cand[sel]), axis=1)).max() <= SWEEP_TOL
    assert r["committed"] == changed.sum()
    assert st["t"] == t + 1


def test_sparse_degenerate_cases(bp):
    # no edges: n_0 = 0, converged at once
    prob = dict(N=5, K=2, edges=np.zeros((0, 2), np.int32),
                log_unary=np.array([[0.1, -0.1]] * 5), pair_kind=inputs.PAIR_ISING,
                coupling=np.zeros(0))
    with bp.Graph(prob) as g:
        r = g.run("rnbp", p=0.5, sparse=1)
        assert r["converged"] and r["iterations"] == 0 and r["evaluated"] == 0
    # max_iters = 0: one evaluation, no commit, same as the full path
    prob = inputs.ising_grid(10, 10, 1.0, 0)
    a = _run(bp, prob, 0, p=0.5, max_iters=0)
    b = _run(bp, prob, 1, p=0.5, max_iters=0)
    _assert_same(a, b)
    assert b[0]["iterations"] == 0 and b[0]["evaluated"] == 360
    # zero field: uniform messages are a fixed point, converged at t = 0
    prob = inputs.ising_grid(12, 9, 2.0, 1)
    prob["log_unary"] = np.zeros_like(prob["log_unary"])
    r = _run(bp, prob, 1, p=0.5)[0]
    assert r["converged"] and r["iterations"] == 0


def test_sparse_rejected_where_not_built(bp):
    prob = inputs.ising_grid(8, 8, 1.0, 0)
    with bp.Graph(prob) as g:
        with pytest.raises(bp.BpError):
            g.run("lbp", p=0.5, sparse=1)
        with pytest.raises(bp.BpError):
            g.run("rnbp", p=0.5, sparse=3)
    with bp.Graph(inputs.potts_grid(6, 6, 3, 1.0, 0)) as g:
        with pytest.raises(bp.BpError):
            g.run("rnbp", p=0.5, sparse=1)
    # a star whose centre has more messages than one tile holds
    n = 700
    edges = np.stack([np.zeros(n - 1, np.int32), np.arange(1, n, dtype=np.int32)], 1)
    rng = np.random.default_rng(0)
    star = dict(N=n, K=2, edges=edges, log_unary=np.stack([-np.ones(n), np.ones(n)], 1) * 0.1,
                pair_kind=inputs.PAIR_ISING, coupling=rng.uniform(-1, 1, n - 1))
    with bp.Graph(star) as g:
        with pytest.raises(bp.BpError):
            g.run("rnbp", p=0.5, sparse=1)


def test_sparse_ising_1000_full_size(bp):
    # the 1000 x 1000 grid at C = 1 to convergence: switching to the sparse path
    # changes nothing but the number of evaluated messages
    prob = inputs.ising_grid(1000, 1000, 1.0, 100)
    kw = dict(eps=1e-4, p=0.5, seed=0, max_iters=3000, check_every=16)
    full = _run(bp, prob, 0, **kw)
    auto = _run(bp, prob, 2, **kw)
    _assert_same(full, auto)
    assert full[0]["converged"]
    assert auto[0]["evaluated"] < full[0]["evaluated"]
