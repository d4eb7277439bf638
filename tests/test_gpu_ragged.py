"""Variables with their own numbers of states (bp_graph_desc.var_states; the
ragged layout) on the GPU against the oracle.

The message i -> j holds K_j values and Eq. (2) sums over the K_i states of i
(Sec. II-A); the synthetic stand-in for the side-chain models of Sec. IV-E
(2 to 81 states per variable, a contact graph) is inputs.protein_like_graph.
Bars as for the uniform layouts: one LBP sweep from the same FP32 state within
1e-6 relative per message; converged beliefs within 1e-4 where the fixed point
is unique (trees, weak coupling); RnBP and RBP frontiers equal outside the
band of residuals within 1e-6 of the decision threshold.
"""
import numpy as np
import pytest

import oracle
from paper_1909_11469_amd import inputs

pytestmark = pytest.mark.gpu

SWEEP_TOL = 1e-6
BAND = 1e-6


@pytest.fixture(scope="module")
def bp():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1909_11469_amd import bp as mod
    return mod


def _rows(prob):
    off = oracle.message_offsets(prob)
    return off[:-1], off[1:]


def _random_state(prob, seed, lo=0.2):
    """A positive ragged message set, each row normalised, rounded to FP32."""
    a, b = _rows(prob)
    rng = np.random.default_rng(seed)
    m = rng.uniform(lo, 1.0, size=int(b[-1]))
    for x, y in zip(a, b):
        m[x:y] /= m[x:y].sum()
    return m.astype(np.float32)


def _row_rel_err(m_gpu, m_ref, prob):
    a, b = _rows(prob)
    d = np.abs(m_gpu.astype(np.float64) - m_ref)
    return np.array([d[x:y].max() / np.abs(m_ref[x:y]).max() for x, y in zip(a, b)])


def _row_changed(m1, m0, prob):
    a, b = _rows(prob)
    ne = (m1 != m0)
    return np.array([ne[x:y].any() for x, y in zip(a, b)])


PROBLEMS = {
    "vark60": lambda: inputs.vark_graph(60, 150, 9, 1),
    "vark_tree_k128": lambda: inputs.vark_graph(40, 0, 128, 2, tree=True),
    "protein300": lambda: inputs.protein_like_graph(300, 8.0, 3),
    "vark_dense_deg": lambda: inputs.vark_graph(30, 300, 6, 4),
    # most variables heavy: up to 128 states and about 14 neighbours
    "vark_heavy_k128": lambda: inputs.vark_graph(30, 200, 128, 7),
}


def _heavy_slots(prob):
    """Messages out of variables that the evaluation kernel gives a wave per
    slot: more than 64 neighbours, more than 1024 cavity or output entries, or
    more than 16384 multiply-adds (output entries times K_i)."""
    K = np.asarray(prob["var_states"], dtype=np.int64)
    e = np.asarray(prob["edges"], dtype=np.int64).reshape(-1, 2)
    deg = np.bincount(e.ravel(), minlength=len(K))
    P = np.zeros(len(K), np.int64)
    np.add.at(P, e[:, 0], K[e[:, 1]])
    np.add.at(P, e[:, 1], K[e[:, 0]])
    flat = (deg <= 64) & (deg * K <= 1024) & (P <= 1024) & (P * K <= 16384)
    return int(deg[~flat].sum())


@pytest.mark.parametrize("name", list(PROBLEMS))
def test_ragged_single_lbp_sweep(bp, name):
    prob = PROBLEMS[name]()
    S = _random_state(prob, 7)
    with bp.Graph(prob) as g:
        assert g.info()["layout"] == 2
        assert g.info()["heavy_slots"] == _heavy_slots(prob)
        g.set_state(S, t=0)
        S, _ = g.get_state()
        g.run("lbp", eps=0.0, max_iters=1, warm_start=True)
        m, _ = g.get_state()
    cand, _ = oracle.evaluate(prob, S.astype(np.float64))
    err = _row_rel_err(m, cand, prob)
    print(f"{name}: {len(err)} messages ({_heavy_slots(prob)} heavy), max rel err {err.max():.2e}")
    assert err.max() <= SWEEP_TOL


def test_ragged_heavy_slots_cover_both_product_forms():
    # the sweep problems reach the per-slot path with K_j <= 64 (rows of the
    # table several at a time) and K_j > 64 (two target states per lane)
    for name in ("vark_tree_k128", "protein300", "vark_heavy_k128"):
        assert _heavy_slots(PROBLEMS[name]()) > 0, name
    prob = PROBLEMS["vark_heavy_k128"]()
    K = np.asarray(prob["var_states"])
    assert K.max() > 64 and K.min() <= 64


@pytest.mark.parametrize("schedule,p", [("lbp", 1.0), ("rnbp", 0.5), ("rbp", 0.1)])
def test_ragged_tree_converged_marginals(bp, schedule, p):
    # BP is exact on trees: every schedule converges to the oracle's beliefs
    prob = inputs.vark_graph(80, 0, 20, 5, tree=True)
    ref = oracle.run(prob, oracle.LBP, eps=1e-12, max_iters=1000)
    assert ref["converged"]
    with bp.Graph(prob) as g:
        r = g.run(schedule, eps=1e-7, p=p, seed=3, max_iters=20000)
        b = g.marginals()
    assert r["converged"]
    assert b.shape == ref["marginals"].shape
    assert np.max(np.abs(b - ref["marginals"])) <= 1e-4


def test_ragged_protein_like_converged_marginals(bp):
    # weak coupling on the contact graph: a unique fixed point
    prob = inputs.protein_like_graph(200, 6.0, 6, coupling_scale=0.15)
    ref = oracle.run(prob, oracle.LBP, eps=1e-10, max_iters=5000)
    assert ref["converged"]
    with bp.Graph(prob) as g:
        r = g.run("rnbp", eps=1e-6, p=0.5, seed=1, max_iters=5000)
        b = g.marginals()
    assert r["converged"]
    print(f"protein-like 200: {r['iterations']} iterations, "
          f"max |b - oracle| {np.max(np.abs(b - ref['marginals'])):.2e}")
    assert np.max(np.abs(b - ref["marginals"])) <= 1e-4


@pytest.mark.parametrize("dynamic,prev", [(True, -1), (True, 400), (False, -1)])
def test_ragged_rnbp_iterations_against_oracle(bp, dynamic, prev):
    prob = inputs.protein_like_graph(250, 7.0, 8)
    E = 2 * len(prob["edges"])
    S0 = _random_state(prob, 9, lo=0.3)
    eps, p, seed, t0 = 2e-3, 0.5, 13, 5
    with bp.Graph(prob) as g:
        g.set_state(S0, t=t0, prev_active=prev)
        # the stored state (rows renormalised in FP32), continued on the
        # device one iteration at a time
        m_prev, st_prev = g.get_state()
        for k in range(1, 5):
            r = g.run("rnbp", eps=eps, p=p, seed=seed, max_iters=1, warm_start=True,
                      dynamic_p=dynamic)
            m_now, st_now = g.get_state()
            ref = oracle.run(prob, oracle.RNBP, eps=eps, p=p, seed=seed, dynamic_p=dynamic,
                             max_iters=1, init_msgs=m_prev.astype(np.float64),
                             t0=st_prev["t"], prev_active=st_prev["prev_active"], trace=True)
            cand, res = oracle.evaluate(prob, m_prev.astype(np.float64))
            want = _row_changed(ref["msgs"], m_prev.astype(np.float64), prob)
            got = _row_changed(m_now, m_prev, prob)
            band = np.abs(res - eps) < BAND
            assert band.sum() <= 6
            assert np.array_equal(got[~band], want[~band]), k
            sel = want & ~band
            a, b = _rows(prob)
            for e in np.flatnonzero(sel):
                x, y = a[e], b[e]
                assert np.max(np.abs(m_now[x:y] - cand[x:y])) <= SWEEP_TOL * np.max(cand[x:y])
            assert st_now["t"] == st_prev["t"] + 1
            assert abs(st_now["prev_active"] - int(ref["trace"]["active"][0])) <= band.sum()
            assert r["iterations"] == 1
            m_prev, st_prev = m_now, st_now
    assert E > 0


def test_ragged_rbp_one_iteration(bp):
    prob = inputs.protein_like_graph(250, 7.0, 10)
    E = 2 * len(prob["edges"])
    S0 = _random_state(prob, 11, lo=0.3)
    p = 0.05
    with bp.Graph(prob) as g:
        g.set_state(S0, t=0)
        S0, _ = g.get_state()
        r = g.run("rbp", eps=1e-4, p=p, max_iters=1, warm_start=True)
        m, _ = g.get_state()
    cand, res = oracle.evaluate(prob, S0.astype(np.float64))
    k = max(1, int(np.ceil(p * E)))
    thr = np.sort(res)[::-1][k - 1]
    band = np.abs(res - thr) < BAND
    assert band.sum() <= 2
    ref = oracle.run(prob, oracle.RBP, eps=1e-4, p=p, max_iters=1,
                     init_msgs=S0.astype(np.float64))
    want = _row_changed(ref["msgs"], S0.astype(np.float64), prob)
    got = _row_changed(m, S0, prob)
    assert np.array_equal(got[~band], want[~band])
    assert r["committed"] == k


def test_ragged_state_round_trip_and_rejects(bp):
    prob = inputs.vark_graph(20, 40, 7, 12)
    S = _random_state(prob, 1)
    with bp.Graph(prob) as g:
        g.set_state(S, t=3)
        m, st = g.get_state()
        assert st["t"] == 3
        a, b = _rows(prob)
        for x, y in zip(a, b):
            assert np.allclose(m[x:y], S[x:y] / S[x:y].sum(), rtol=5e-7, atol=0)
        # ragged graphs take no sparse re-evaluation and no residual splash
        for kw in ({"schedule": "rs"}, {"schedule": "rnbp", "sparse": 1}):
            sched = kw.pop("schedule")
            with pytest.raises(bp.BpError):
                g.run(sched, eps=1e-4, p=0.5, max_iters=2, **kw)
        # fresh runs start from the uniform 1 / K_j messages
        g.run("lbp", eps=1e-4, max_iters=0)
        m0, _ = g.get_state()
        for x, y in zip(a, b):
            assert np.all(m0[x:y] == np.float32(1.0 / (y - x)))
