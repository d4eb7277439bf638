"""Residual splash (BP_RS, Sec. II-B, Sec. III-A) on the GPU against the oracle.

One iteration from the same FP32 state: the roots are the k variables of
largest residual (largest incoming message residual, ties by id); FP32 and
FP64 residuals can order differently only where two variable residuals lie
within 1e-6 of each other around the k-th, so every case asserts a gap there
(or has exactly tied residuals, decided by id alone).  With the same roots the
levels are the same, so the same messages are committed (the commit count is
compared exactly and every other message must keep its bits) and the committed
values must agree with the oracle.  A splash iteration chains 2h + 1 level
updates, each one sweep over its messages from the state the previous level
left, so the FP32 error of one sweep (1e-6 relative) can accumulate once per
level: the bar is (2h + 1) * 1e-6 relative per message.
"""
import numpy as np
import pytest

import oracle
from paper_1909_11469_amd import inputs

pytestmark = pytest.mark.gpu

SWEEP_TOL = 1e-6
GAP = 1e-6


@pytest.fixture(scope="module")
def bp():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1909_11469_amd import bp as mod
    return mod


def _random_state(E, seed, lo):
    m = np.random.default_rng(seed).uniform(lo, 1.0, size=(E, 2))
    m /= m.sum(1, keepdims=True)
    return m.astype(np.float32)


def _rel_err(a, ref):
    d = np.max(np.abs(a.astype(np.float64) - ref), axis=1)
    return d / np.max(np.abs(ref), axis=1)


def _roots_gap(prob, m, p):
    """The oracle's variable residuals around the k-th largest: the smallest
    distance between the k-th and its neighbours in the sorted order (inf when
    every variable is a root)."""
    N = int(prob["N"])
    _, dst = oracle.canonical_src_dst(prob)
    _, res = oracle.evaluate(prob, m.astype(np.float64))
    vres = np.zeros(N)
    np.maximum.at(vres, dst, res)
    k = min(N, max(1, int(np.ceil(p * len(dst)))))
    if k >= N:
        return np.inf
    s = np.sort(vres)[::-1]
    return float(s[k - 1] - s[k])


def _gpu_iterations(bp, prob, S0, kmax, p, h, eps):
    """States and stats after max_iters = 0 .. kmax from S0 (each a fresh run
    from S0: the runs are deterministic, so run k is run k - 1 plus one
    iteration)."""
    out = []
    with bp.Graph(prob) as g:
        for k in range(kmax + 1):
            g.set_state(S0, t=0, prev_active=-1)
            r = g.run("rs", eps=eps, p=p, max_iters=k, warm_start=True, splash_depth=h,
                      check_every=2)
            m, _ = g.get_state()
            out.append((m, r))
    return out


def _check_one(prob, m_prev, m_now, r_now, r_prev, p, h, eps):
    ref = oracle.rs(prob, eps=eps, p=p, splash_depth=h, max_iters=1,
                    init_msgs=m_prev.astype(np.float64), trace=True)
    assert r_now["committed"] - r_prev["committed"] == ref["committed"]
    want = ref["msgs"]
    changed = np.any(want != m_prev.astype(np.float64), axis=1)
    assert _rel_err(m_now[changed], want[changed]).max() <= (2 * h + 1) * SWEEP_TOL
    # messages out of no level variable keep their bits (a committed message
    # can also equal its old value, so only the unchanged set is checked)
    src, _ = oracle.canonical_src_dst(prob)
    touched = np.zeros(int(prob["N"]), bool)
    touched[src[changed]] = True
    untouched = ~touched[src]
    assert np.array_equal(m_now[untouched], m_prev[untouched])
    return ref


CASES = [  # problem, p, h, eps, start-state floor
    ("grid20_C1", 0.02, 2, 1e-4, 0.3),
    ("grid20_C2.5", 0.05, 2, 1e-4, 0.3),
    ("grid23x31_C4", 0.01, 2, 1e-4, 0.2),
    ("grid20_C2.5", 0.05, 1, 1e-4, 0.3),
    ("grid20_C2.5", 0.05, 0, 1e-4, 0.3),
    ("er600_C2.5", 0.03, 2, 1e-4, 0.3),
    ("tree300_C2", 0.04, 2, 1e-4, 0.3),
]


def _problem(name):
    return {"grid20_C1": lambda: inputs.ising_grid(20, 20, 1.0, 3),
            "grid20_C2.5": lambda: inputs.ising_grid(20, 20, 2.5, 4),
            "grid23x31_C4": lambda: inputs.ising_grid(23, 31, 4.0, 5),
            "er600_C2.5": lambda: inputs.er_graph(600, 6.0, 2.5, 6),
            "tree300_C2": lambda: inputs.ising_tree(300, 2.0, 7)}[name]()


@pytest.mark.parametrize("name,p,h,eps,lo", CASES)
def test_rs_iterations_against_oracle(bp, name, p, h, eps, lo):
    prob = _problem(name)
    E = 2 * len(prob["edges"])
    S0 = _random_state(E, 11, lo)
    runs = _gpu_iterations(bp, prob, S0, 4, p, h, eps)
    for k in range(1, len(runs)):
        m_prev, r_prev = runs[k - 1]
        m_now, r_now = runs[k]
        if r_prev["converged"]:
            break
        gap = _roots_gap(prob, m_prev, p)
        assert gap > GAP, f"roots not separated at iteration {k}: gap {gap:.2e}"
        assert r_now["iterations"] == k
        ref = _check_one(prob, m_prev, m_now, r_now, r_prev, p, h, eps)
        # n_t of the evaluation of m_prev, as the oracle counts it, up to
        # residuals within the band around eps
        _, res = oracle.evaluate(prob, m_prev.astype(np.float64))
        band = int(np.sum(np.abs(res - eps) < GAP))
        assert abs(r_prev["last_active"] - int(ref["trace"]["active"][0])) <= band


def test_rs_exact_ties_taken_by_id(bp):
    # equal fields and couplings from uniform messages: every message residual,
    # hence every variable residual of equal degree, is bitwise equal, and the
    # roots are decided by id alone
    prob = inputs.ising_grid(17, 19, 1.0, 0)
    prob["log_unary"] = np.tile([-0.4, 0.4], (prob["N"], 1))
    prob["coupling"] = np.full(len(prob["edges"]), 0.7)
    E = 2 * len(prob["edges"])
    U = np.full((E, 2), 0.5, np.float32)
    for p, h in ((0.01, 2), (0.03, 1), (0.05, 0)):
        with bp.Graph(prob) as g:
            r = g.run("rs", eps=1e-6, p=p, max_iters=1, splash_depth=h)
            m, _ = g.get_state()
        ref = oracle.rs(prob, eps=1e-6, p=p, splash_depth=h, max_iters=1, trace=True)
        assert r["committed"] == ref["committed"]
        changed_ref = np.any(ref["msgs"] != 0.5, axis=1)
        changed_gpu = np.any(m != U, axis=1)
        assert np.array_equal(changed_ref, changed_gpu)
        assert _rel_err(m[changed_ref], ref["msgs"][changed_ref]).max() <= (2 * h + 1) * SWEEP_TOL


def test_rs_depth_zero_all_roots_equals_lbp_bitwise(bp):
    # p = 1 makes every variable a root; depth 0 updates every message from m^t
    prob = inputs.ising_grid(33, 29, 2.5, 8)
    with bp.Graph(prob) as g:
        a = g.run("lbp", eps=1e-5, max_iters=40)
        ma, _ = g.get_state()
        b = g.run("rs", eps=1e-5, p=1.0, max_iters=40, splash_depth=0)
        mb, _ = g.get_state()
    assert np.array_equal(ma, mb)
    for k in ("iterations", "committed", "last_active", "final_t"):
        assert a[k] == b[k], k


@pytest.mark.parametrize("name,C", [("grid", 0.3), ("tree", 2.0), ("er", 0.3)])
def test_rs_converged_marginals(bp, name, C):
    # unique fixed point (weak coupling, or a tree): the splash converges to the
    # marginals of the oracle's LBP
    prob = {"grid": lambda: inputs.ising_grid(24, 24, C, 2),
            "tree": lambda: inputs.ising_tree(500, C, 3),
            "er": lambda: inputs.er_graph(1000, 5.0, C, 4)}[name]()
    ref = oracle.run(prob, oracle.LBP, eps=1e-9, max_iters=10000)
    assert ref["converged"]
    with bp.Graph(prob) as g:
        r = g.run("rs", eps=1e-6, p=1 / 32, max_iters=20000, splash_depth=2)
        b = g.marginals()
    assert r["converged"]
    assert np.max(np.abs(b - ref["marginals"])) <= 1e-4


def test_rs_degenerate_cases(bp):
    # h = 0 fields: uniform messages are a fixed point, converged at t = 0
    prob = inputs.ising_grid(10, 10, 2.0, 1)
    prob["log_unary"] = np.zeros((prob["N"], 2))
    with bp.Graph(prob) as g:
        r = g.run("rs", eps=1e-6, p=0.1, max_iters=50)
        assert r["converged"] and r["iterations"] == 0 and r["committed"] == 0
        r = g.run("rs", eps=1e-6, p=0.1, max_iters=0)
        assert r["iterations"] == 0
    # isolated variables (no incoming messages: residual exactly 0) among the
    # roots, tied at 0 and taken by id on both sides
    prob = inputs.er_graph(400, 1.0, 1.0, 2)
    N, E = prob["N"], 2 * len(prob["edges"])
    _, dst = oracle.canonical_src_dst(prob)
    _, res = oracle.evaluate(prob, np.full((E, 2), 0.5))
    vres = np.zeros(N)
    np.maximum.at(vres, dst, res)
    k = int(np.ceil(0.8 * E))
    assert k < N and np.sort(vres)[::-1][k - 1] == 0.0
    assert not np.any((vres > 0) & (vres < GAP))
    ref = oracle.rs(prob, eps=1e-5, p=0.8, splash_depth=2, max_iters=1, trace=True)
    with bp.Graph(prob) as g:
        r = g.run("rs", eps=1e-5, p=0.8, max_iters=1)
    assert r["committed"] == ref["committed"]


def test_rs_rejects(bp):
    prob = inputs.ising_grid(6, 6, 1.0, 0)
    with bp.Graph(prob) as g:
        for kw in ({"splash_depth": 3}, {"splash_depth": -1}, {"sparse": 1}, {"p": 0.0}):
            args = dict(eps=1e-4, p=0.1, max_iters=3)
            args.update(kw)
            with pytest.raises(bp.BpError) as e:
                g.run("rs", **args)
            assert e.value.code == bp.BP_EINVAL
    with bp.Graph(inputs.potts_grid(5, 5, 3, 1.0, 0)) as g:
        with pytest.raises(bp.BpError) as e:
            g.run("rs", eps=1e-4, p=0.1, max_iters=3)
        assert e.value.code == bp.BP_EINVAL


def _levels_sparse(N, src, dst, roots, h):
    """Level membership for h <= 2 with sparse products: level 1 = neighbours of
    a root; level 2 = vertices w with a root r at distance exactly 2 (a common
    neighbour, w != r, w not adjacent to r)."""
    from scipy.sparse import csr_matrix
    E = len(src)
    A = csr_matrix((np.ones(E, np.int32), (src, dst)), shape=(N, N))
    lv = [np.zeros(N, bool) for _ in range(h + 1)]
    lv[0][roots] = True
    if h >= 1:
        lv[1] = np.asarray(A[:, roots].sum(axis=1)).ravel() > 0
    if h >= 2:
        Ar = A[:, roots].tocsc()
        P = (A @ Ar).tocoo()  # P[w, j]: paths of length 2 from roots[j] to w
        w, j = P.row, P.col
        r = roots[j]
        keep = (w != r) & (np.asarray(A[w, r]).ravel() == 0)
        lv[2][w[keep]] = True
    return lv


def test_rs_ising_1000_one_iteration_full_size(bp):
    # 1000 x 1000, C = 2.5, p = 1/256 (15,610 roots), depth 2, from a random
    # state: every message compared with a replay over the oracle's evaluation
    prob = inputs.ising_grid(1000, 1000, 2.5, 0)
    N = prob["N"]
    E = 2 * len(prob["edges"])
    src, dst = oracle.canonical_src_dst(prob)
    S0 = _random_state(E, 9, 0.3)
    p, h = 1 / 256, 2
    with bp.Graph(prob) as g:
        g.set_state(S0, t=0, prev_active=-1)
        # the state as stored (K = 2 messages are kept as FP32 log-odds, so
        # the probabilities read back may differ from S0 in the last bit)
        S0, _ = g.get_state()
        r = g.run("rs", eps=1e-4, p=p, max_iters=1, warm_start=True, splash_depth=h)
        m, _ = g.get_state()
    m0 = S0.astype(np.float64)
    cand, res = oracle.evaluate(prob, m0)
    vres = np.zeros(N)
    np.maximum.at(vres, dst, res)
    k = min(N, int(np.ceil(p * E)))
    order = np.lexsort((np.arange(N), -vres))
    s = vres[order]
    assert s[k - 1] - s[k] > GAP
    roots = order[:k]
    lv = _levels_sparse(N, src, dst, roots, h)
    cur = m0.copy()
    committed = 0
    for q, d in enumerate(list(range(h, -1, -1)) + list(range(1, h + 1))):
        # the first level starts from m^t, whose candidates are already known
        c = cand if q == 0 else oracle.evaluate(prob, cur)[0]
        sel = lv[d][src]
        cur[sel] = c[sel]
        committed += int(sel.sum())
    assert r["committed"] == committed
    touched = np.zeros(N, bool)
    for d in range(h + 1):
        touched |= lv[d]
    upd = touched[src]
    assert np.array_equal(m[~upd], S0[~upd])
    err = _rel_err(m[upd], cur[upd])
    print(f"1000x1000 splash iteration: {upd.sum()} messages updated, max rel err {err.max():.2e}")
    assert err.max() <= (2 * h + 1) * SWEEP_TOL
