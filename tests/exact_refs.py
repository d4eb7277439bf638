"""Exact inference routines used to pin the FP64 oracle.

Each routine is a different algorithm from belief propagation, written
independently of ``oracle/``:

* ``brute_force_marginals``: enumerate every joint state of Eq. (1);
* ``chain_marginals``: the textbook forward-backward recursion on a chain;
* ``grid_marginals_transfer``: exact marginals of a small-width Ising grid by
  variable elimination one row at a time (transfer matrices over 2^W row states),
  the check the paper uses for its 10 x 10 correctness test (Sec. IV-E);
* ``ising_message_closed_form``: Eq. (2) for binary spins with psi_i = exp(h s),
  psi_ij = exp(J s_i s_j), solved in closed form with hyperbolic functions.
"""
import itertools

import numpy as np


def _states(problem):
    """States of every variable."""
    vs = problem.get("var_states")
    N = int(problem["N"])
    return np.full(N, int(problem["K"])) if vs is None else np.asarray(vs, int)


def _unary(problem):
    """Log-unaries as a list of per-variable arrays (ragged or [N, K])."""
    ks = _states(problem)
    lu = np.asarray(problem["log_unary"], float).reshape(-1)
    off = np.concatenate([[0], np.cumsum(ks)])
    return [lu[off[i]:off[i + 1]] for i in range(len(ks))]


def _pair_table(problem, u):
    """Table psi_u[x_a, x_b] of undirected edge u = (a, b) (K_a x K_b)."""
    kind = int(problem["pair_kind"])
    K = int(problem["K"])
    if problem.get("var_states") is not None:
        ks = _states(problem)
        edges = np.asarray(problem["edges"]).reshape(-1, 2)
        sizes = ks[edges[:, 0]] * ks[edges[:, 1]]
        o = int(np.sum(sizes[:u]))
        a, b = int(edges[u, 0]), int(edges[u, 1])
        return np.asarray(problem["pair"], float)[o:o + ks[a] * ks[b]].reshape(ks[a], ks[b])
    if kind == 0:
        J = float(problem["coupling"][u])
        s = np.array([-1.0, 1.0])
        return np.exp(J * np.outer(s, s))
    if kind == 1:
        return float(problem["edge_scale"][u]) * np.asarray(problem["shared"], float).reshape(K, K)
    return np.asarray(problem["pair"], float)[u]


def brute_force_marginals(problem):
    """Exact marginals by summing Eq. (1) over every joint state ([N, K], or
    ragged [sum K_i] for a problem with per-variable state counts)."""
    N, K = int(problem["N"]), int(problem["K"])
    ks = _states(problem)
    if np.prod(ks.astype(float)) > 1 << 20:
        raise ValueError("too large for enumeration")
    edges = np.asarray(problem["edges"]).reshape(-1, 2)
    lu = _unary(problem)
    tables = [np.log(_pair_table(problem, u)) for u in range(len(edges))]
    states = np.array(list(itertools.product(*[range(k) for k in ks])), dtype=np.int64)
    logp = np.zeros(len(states))
    for i in range(N):
        logp += lu[i][states[:, i]]
    for u, (a, b) in enumerate(edges):
        logp += tables[u][states[:, a], states[:, b]]
    w = np.exp(logp - logp.max())
    w /= w.sum()
    rows = [np.array([w[states[:, i] == x].sum() for x in range(ks[i])]) for i in range(N)]
    if problem.get("var_states") is not None:
        return np.concatenate(rows)
    return np.stack(rows)


def chain_marginals(problem):
    """Forward-backward on a chain whose edges are (i, i + 1) in order ([N, K],
    or ragged [sum K_i] with per-variable state counts)."""
    N = int(problem["N"])
    edges = np.asarray(problem["edges"]).reshape(-1, 2)
    assert len(edges) == N - 1 and all(int(a) == i and int(b) == i + 1
                                       for i, (a, b) in enumerate(edges))
    phi = [np.exp(u) for u in _unary(problem)]
    T = [_pair_table(problem, u) for u in range(N - 1)]
    alpha, beta = [None] * N, [None] * N
    alpha[0] = phi[0] / phi[0].sum()
    for i in range(1, N):
        a = (alpha[i - 1] @ T[i - 1]) * phi[i]
        alpha[i] = a / a.sum()
    beta[N - 1] = np.ones(len(phi[N - 1]))
    for i in range(N - 2, -1, -1):
        b = T[i] @ (phi[i + 1] * beta[i + 1])
        beta[i] = b / b.sum()
    rows = [alpha[i] * beta[i] / np.sum(alpha[i] * beta[i]) for i in range(N)]
    if problem.get("var_states") is not None:
        return np.concatenate(rows)
    return np.stack(rows)


def grid_marginals_transfer(problem, H, W):
    """Exact marginals of an H x W binary grid (node r*W + c, right/down edges) by
    eliminating one row at a time.  Handles any pairwise table kind with K = 2."""
    assert int(problem["K"]) == 2 and H * W == int(problem["N"])
    edges = np.asarray(problem["edges"]).reshape(-1, 2)
    lu = np.asarray(problem["log_unary"], float)
    S = 1 << W
    bits = (np.arange(S)[:, None] >> np.arange(W)[None, :]) & 1  # [S, W]: state of column c
    horiz, vert = {}, {}
    for u, (a, b) in enumerate(edges):
        a, b = int(a), int(b)
        t = np.log(_pair_table(problem, u))
        if b == a + 1:
            horiz[a] = t
        else:
            assert b == a + W
            vert[a] = t
    # log row potentials: unaries + horizontal couplings inside the row
    row_lp = np.zeros((H, S))
    for r in range(H):
        for c in range(W):
            i = r * W + c
            row_lp[r] += lu[i, bits[:, c]]
            if c < W - 1:
                row_lp[r] += horiz[i][bits[:, c], bits[:, c + 1]]
    # log vertical transfer between row r and r+1: [S, S]
    vt = []
    for r in range(H - 1):
        L = np.zeros((S, S))
        for c in range(W):
            i = r * W + c
            L += vert[i][bits[:, c][:, None], bits[:, c][None, :]]
        vt.append(L)
    # forward / backward in log space
    la = np.zeros((H, S))
    lb = np.zeros((H, S))
    la[0] = row_lp[0]
    for r in range(1, H):
        x = la[r - 1][:, None] + vt[r - 1]
        mx = x.max(axis=0)
        la[r] = mx + np.log(np.exp(x - mx).sum(axis=0)) + row_lp[r]
    lb[H - 1] = 0.0
    for r in range(H - 2, -1, -1):
        x = vt[r] + (row_lp[r + 1] + lb[r + 1])[None, :]
        mx = x.max(axis=1)
        lb[r] = mx + np.log(np.exp(x - mx[:, None]).sum(axis=1))
    out = np.zeros((H * W, 2))
    for r in range(H):
        lp = la[r] + lb[r]
        w = np.exp(lp - lp.max())
        w /= w.sum()
        for c in range(W):
            out[r * W + c, 1] = w[bits[:, c] == 1].sum()
            out[r * W + c, 0] = 1.0 - out[r * W + c, 1]
    return out


def star_marginals(problem, center=0):
    """Exact marginals of a star (every edge joins ``center`` to a leaf), summed in
    log space: the centre's marginal is psi_c(x) prod_l sum_y psi(x, y) psi_l(y); a
    leaf's is psi_l(y) sum_x psi(x, y) psi_c(x) prod_{l' != l} (...)."""
    N, K = int(problem["N"]), int(problem["K"])
    edges = np.asarray(problem["edges"]).reshape(-1, 2)
    lu = np.asarray(problem["log_unary"], float)
    leaf_terms = np.zeros((len(edges), K))  # log sum_y psi(x_c = x, y) psi_l(y)
    tabs = []
    for u, (a, b) in enumerate(edges):
        T = _pair_table(problem, u)
        if int(a) == center:
            leaf, Tcl = int(b), T
        else:
            assert int(b) == center
            leaf, Tcl = int(a), T.T
        tabs.append((leaf, Tcl))
        leaf_terms[u] = np.log(Tcl @ np.exp(lu[leaf]))
    total = lu[center] + leaf_terms.sum(axis=0)
    out = np.zeros((N, K))
    w = np.exp(total - total.max())
    out[center] = w / w.sum()
    for u, (leaf, Tcl) in enumerate(tabs):
        lc = total - leaf_terms[u]  # centre without this leaf
        c = np.exp(lc - lc.max())
        b = np.exp(lu[leaf]) * (Tcl.T @ c)
        out[leaf] = b / b.sum()
    return out


def ising_message_closed_form(h_i, J, u_in):
    """Eq. (2) for psi_i = exp(h_i s_i), psi_ij = exp(J s_i s_j), with incoming
    messages written as fields u_k = 0.5 log(m(+1) / m(-1)) over Gamma_i \\ j.
    The sum over s_i of exp(J s_i s_j + H s_i) is 2 cosh(J s_j + H), H = h_i + sum u_k,
    so the outgoing field is atanh(tanh J tanh H).  Returns (m(-1), m(+1))."""
    H = h_i + float(np.sum(u_in))
    u = np.arctanh(np.tanh(J) * np.tanh(H))
    mp = 0.5 * (1.0 + np.tanh(u))
    return np.array([1.0 - mp, mp])


def kl_divergence(p, q):
    """Mean over variables of KL(p_i || q_i)."""
    p = np.clip(np.asarray(p, float), 1e-300, None)
    q = np.clip(np.asarray(q, float), 1e-300, None)
    return float(np.mean(np.sum(p * (np.log(p) - np.log(q)), axis=1)))
