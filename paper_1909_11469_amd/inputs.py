"""Seeded synthetic pairwise-MRF generators.

This module draws random problem instances and nothing else: it holds none of
the belief-propagation arithmetic, so both the HIP path and the FP64 oracle can
be fed from it.  Every generator uses numpy's PCG64 (``default_rng(seed)``) and
a fixed draw order, so a (generator, arguments, seed) triple names one problem.

A problem is a plain dict:
    N, K        number of variables, states per variable
    edges       int32 [M, 2] undirected edges (a, b), no self-loops, no duplicates
    log_unary   float64 [N, K]: psi_i(x) = exp(log_unary[i, x])
    pair_kind   PAIR_ISING  : coupling float64 [M], psi = exp(J * s_a * s_b),
                              spins s = -1 (state 0) and +1 (state 1)
                PAIR_SHARED : shared float64 [K, K] > 0, edge_scale float64 [M] > 0,
                              psi_u = edge_scale[u] * shared
                PAIR_DENSE  : pair float64 [M, K, K] > 0, first index is the state
                              of edges[u, 0]
    name        short description

Grid node ids are r * W + c; undirected grid edges are listed per node in id
order: (id, id + 1) if c < W - 1, then (id, id + W) if r < H - 1.
"""
import numpy as np

PAIR_ISING, PAIR_SHARED, PAIR_DENSE = 0, 1, 2


def grid_edges(H: int, W: int) -> np.ndarray:
    ids = np.arange(H * W, dtype=np.int64).reshape(H, W)
    out = []
    for r in range(H):
        for c in range(W):
            i = ids[r, c]
            if c < W - 1:
                out.append((i, i + 1))
            if r < H - 1:
                out.append((i, i + W))
    return np.asarray(out, dtype=np.int32).reshape(-1, 2)


def _grid_edges_fast(H: int, W: int) -> np.ndarray:
    """Same list as grid_edges, vectorised for large grids: every node has a
    (right, down) pair of candidate edges, masked at the last column and row."""
    ids = np.arange(H * W, dtype=np.int32).reshape(H, W)
    e = np.empty((H, W, 2, 2), dtype=np.int32)
    e[:, :, 0, 0] = ids
    e[:, :, 0, 1] = ids + 1
    e[:, :, 1, 0] = ids
    e[:, :, 1, 1] = ids + W
    keep = np.empty((H, W, 2), dtype=bool)
    keep[:, :, 0] = np.arange(W) < W - 1
    keep[:, :, 1] = (np.arange(H) < H - 1)[:, None]
    return e[keep]


def ising_grid(H: int, W: int, C: float, seed: int) -> dict:
    """Ising grid: h ~ U[-1, 1]^N, then J ~ U[-C, C]^M; psi_i(x) = exp(h_i s_x),
    psi_ij = exp(J_ij s_i s_j)."""
    rng = np.random.default_rng(seed)
    N = H * W
    edges = _grid_edges_fast(H, W) if N > 4096 else grid_edges(H, W)
    h = rng.uniform(-1.0, 1.0, size=N)
    J = rng.uniform(-C, C, size=edges.shape[0])
    lu = np.stack([-h, h], axis=1)
    return dict(N=N, K=2, edges=edges, log_unary=lu, pair_kind=PAIR_ISING, coupling=J,
                name=f"ising{H}x{W}_C{C}_s{seed}", h=h)


def chain(N: int, C: float, seed: int) -> dict:
    """A chain of N binary variables drawn like the Ising grid (one row)."""
    p = ising_grid(1, N, C, seed)
    p["name"] = f"chain{N}_C{C}_s{seed}"
    return p


def ising_tree(n: int, C: float, seed: int) -> dict:
    """A random tree of n binary variables (vertex i > 0 joined to a parent drawn
    uniformly from 0 .. i-1), then h ~ U[-1, 1]^n and J ~ U[-C, C]^(n-1) as for
    the Ising grid."""
    rng = np.random.default_rng(seed)
    parent = np.array([rng.integers(0, i) for i in range(1, n)], dtype=np.int64)
    edges = np.stack([parent, np.arange(1, n)], axis=1).astype(np.int32).reshape(-1, 2)
    h = rng.uniform(-1.0, 1.0, size=n)
    J = rng.uniform(-C, C, size=edges.shape[0])
    lu = np.stack([-h, h], axis=1)
    return dict(N=n, K=2, edges=edges, log_unary=lu, pair_kind=PAIR_ISING, coupling=J,
                name=f"ising_tree{n}_C{C}_s{seed}", h=h)


def paper_ising_grid(H: int, W: int, C: float, seed: int) -> dict:
    """The paper's Ising parameterisation: one U(0, 1] value per state for psi_i,
    psi_ij = e^{lambda C} when x_i = x_j else e^{-lambda C}, lambda ~ U[-0.5, 0.5].
    In spin form this is J = lambda * C."""
    rng = np.random.default_rng(seed)
    N = H * W
    edges = _grid_edges_fast(H, W) if N > 4096 else grid_edges(H, W)
    u = 1.0 - rng.random(size=(N, 2))  # (0, 1]
    lam = rng.uniform(-0.5, 0.5, size=edges.shape[0])
    return dict(N=N, K=2, edges=edges, log_unary=np.log(u), pair_kind=PAIR_ISING,
                coupling=lam * C, name=f"paper_ising{H}x{W}_C{C}_s{seed}")


def er_edges(n: int, M: int, rng) -> np.ndarray:
    """G(n, M): M distinct undirected edges drawn uniformly, no self-loops.
    Candidate pairs are drawn in batches; duplicates and self-loops are dropped,
    first occurrence kept, until M edges exist."""
    if M > n * (n - 1) // 2:
        raise ValueError("too many edges")
    keys = np.empty(0, dtype=np.int64)
    pairs = np.empty((0, 2), dtype=np.int64)
    while len(keys) < M:
        need = M - len(keys)
        cand = rng.integers(0, n, size=(int(need * 1.2) + 16, 2), dtype=np.int64)
        cand = cand[cand[:, 0] != cand[:, 1]]
        a = np.minimum(cand[:, 0], cand[:, 1])
        b = np.maximum(cand[:, 0], cand[:, 1])
        k = a * n + b
        allk = np.concatenate([keys, k])
        allp = np.concatenate([pairs, np.stack([a, b], 1)])
        _, first = np.unique(allk, return_index=True)
        first.sort()
        keys, pairs = allk[first], allp[first]
    return pairs[:M].astype(np.int32)


def er_graph(n: int, avg_degree: float, C: float, seed: int) -> dict:
    """Erdos-Renyi G(n, M) with M = n * avg_degree / 2, then h ~ U[-1, 1]^n and
    J ~ U[-C, C]^M as for the Ising grid."""
    rng = np.random.default_rng(seed)
    M = int(round(n * avg_degree / 2))
    edges = er_edges(n, M, rng)
    h = rng.uniform(-1.0, 1.0, size=n)
    J = rng.uniform(-C, C, size=M)
    lu = np.stack([-h, h], axis=1)
    return dict(N=n, K=2, edges=edges, log_unary=lu, pair_kind=PAIR_ISING, coupling=J,
                name=f"er{n}_d{avg_degree}_C{C}_s{seed}", h=h)


def potts_grid(H: int, W: int, K: int, beta: float, seed: int) -> dict:
    """Potts grid: log-unary ~ N(0, 1)^{N x K}; one shared K x K matrix
    exp(beta [a == b]); per-edge scale ~ U[0.5, 1.5]."""
    rng = np.random.default_rng(seed)
    N = H * W
    edges = _grid_edges_fast(H, W) if N > 4096 else grid_edges(H, W)
    lu = rng.standard_normal(size=(N, K))
    scale = rng.uniform(0.5, 1.5, size=edges.shape[0])
    shared = np.exp(beta * np.eye(K))
    return dict(N=N, K=K, edges=edges, log_unary=lu, pair_kind=PAIR_SHARED, shared=shared,
                edge_scale=scale, name=f"potts{H}x{W}_K{K}_b{beta}_s{seed}")


def random_tree(n: int, K: int, seed: int, coupling_scale: float = 1.0) -> dict:
    """A random labelled tree (node i > 0 attaches to a uniform earlier node) with
    dense positive pairwise tables exp(N(0, coupling_scale)) and N(0, 1) log-unaries."""
    rng = np.random.default_rng(seed)
    parent = np.array([rng.integers(0, i) for i in range(1, n)], dtype=np.int64)
    edges = np.stack([parent, np.arange(1, n)], axis=1).astype(np.int32)
    lu = rng.standard_normal(size=(n, K))
    pair = np.exp(coupling_scale * rng.standard_normal(size=(n - 1, K, K)))
    return dict(N=n, K=K, edges=edges, log_unary=lu, pair_kind=PAIR_DENSE, pair=pair,
                name=f"tree{n}_K{K}_s{seed}")


def random_dense_graph(n: int, m: int, K: int, seed: int, coupling_scale: float = 1.0):
    """Small loopy graph with dense positive tables (for brute-force checks)."""
    rng = np.random.default_rng(seed)
    edges = er_edges(n, m, rng)
    lu = rng.standard_normal(size=(n, K))
    pair = np.exp(coupling_scale * rng.standard_normal(size=(m, K, K)))
    return dict(N=n, K=K, edges=edges, log_unary=lu, pair_kind=PAIR_DENSE, pair=pair,
                name=f"dense{n}_{m}_K{K}_s{seed}")


def shared_table_graph(n: int, m: int, K: int, seed: int, tree: bool = False) -> dict:
    """Small graph with one shared K x K table exp(N(0, 1)) (not symmetric) and a
    per-edge scale ~ U[0.5, 1.5]: a random labelled tree on n nodes when `tree`,
    else G(n, m).  Log-unaries ~ N(0, 1)."""
    rng = np.random.default_rng(seed)
    if tree:
        parent = np.array([rng.integers(0, i) for i in range(1, n)], dtype=np.int64)
        edges = np.stack([parent, np.arange(1, n)], axis=1).astype(np.int32)
    else:
        edges = er_edges(n, m, rng)
    lu = rng.standard_normal(size=(n, K))
    shared = np.exp(rng.standard_normal(size=(K, K)))
    scale = rng.uniform(0.5, 1.5, size=edges.shape[0])
    return dict(N=n, K=K, edges=edges, log_unary=lu, pair_kind=PAIR_SHARED, shared=shared,
                edge_scale=scale, name=f"shared{n}_K{K}_{'tree' if tree else m}_s{seed}")


def _ragged_tables(rng, Kv, edges, coupling_scale):
    """Dense tables exp(coupling_scale * N(0, 1)) of every edge, K_a x K_b with
    the state of edges[u, 0] first, concatenated."""
    return np.concatenate([np.exp(coupling_scale * rng.standard_normal(int(Kv[a]) * int(Kv[b])))
                           for a, b in edges]) if len(edges) else np.zeros(0)


def vark_graph(n: int, m: int, kmax: int, seed: int, tree: bool = False,
               coupling_scale: float = 1.0) -> dict:
    """Small graph whose variables have 2..kmax states each (uniform draw):
    a random labelled tree on n nodes when `tree`, else G(n, m).  Ragged arrays:
    log_unary [sum K_i] ~ N(0, 1), pair [sum_u K_a K_b] (dense tables)."""
    rng = np.random.default_rng(seed)
    Kv = rng.integers(2, kmax + 1, size=n).astype(np.int32)
    if tree:
        parent = np.array([rng.integers(0, i) for i in range(1, n)], dtype=np.int64)
        edges = np.stack([parent, np.arange(1, n)], axis=1).astype(np.int32)
    else:
        edges = er_edges(n, m, rng)
    lu = rng.standard_normal(size=int(Kv.sum()))
    pair = _ragged_tables(rng, Kv, edges, coupling_scale)
    return dict(N=n, K=int(Kv.max()), var_states=Kv, edges=edges, log_unary=lu,
                pair_kind=PAIR_DENSE, pair=pair, name=f"vark{n}_{'tree' if tree else m}_s{seed}")


def protein_like_graph(n: int, avg_degree: float, seed: int, kmin: int = 2, kmax: int = 81,
                       coupling_scale: float = 0.5) -> dict:
    """Synthetic stand-in for side-chain (protein folding) models with 2..81
    states per variable: n points uniform in a unit cube, an edge between every
    pair closer than the radius that gives the requested average degree (a
    contact graph: irregular degrees, spatial structure); K_i log-uniform on
    [kmin, kmax]; log-unaries ~ N(0, 1); dense tables
    exp(coupling_scale * N(0, 1)) per edge (ragged, state of edges[u, 0] first)."""
    rng = np.random.default_rng(seed)
    pts = rng.random(size=(n, 3))
    # radius for the expected degree of a Poisson process in a unit cube
    r = (3.0 * avg_degree / (4.0 * np.pi * n)) ** (1.0 / 3.0)
    cells = np.floor(pts / r).astype(np.int64)
    ncell = int(np.ceil(1.0 / r)) + 1
    key = (cells[:, 0] * ncell + cells[:, 1]) * ncell + cells[:, 2]
    order = np.argsort(key, kind="stable")
    skey = key[order]
    edges = []
    for dx in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dz in (-1, 0, 1):
                nb = ((cells[:, 0] + dx) * ncell + (cells[:, 1] + dy)) * ncell + cells[:, 2] + dz
                lo = np.searchsorted(skey, nb, side="left")
                hi = np.searchsorted(skey, nb, side="right")
                for i in range(n):
                    for j in order[lo[i]:hi[i]]:
                        if j > i and np.sum((pts[i] - pts[j]) ** 2) < r * r:
                            edges.append((i, j))
    edges = np.array(sorted(set(edges)), dtype=np.int32).reshape(-1, 2)
    Kv = np.exp(rng.uniform(np.log(kmin), np.log(kmax + 1), size=n)).astype(np.int32)
    Kv = np.clip(Kv, kmin, kmax).astype(np.int32)
    lu = rng.standard_normal(size=int(Kv.sum()))
    pair = _ragged_tables(rng, Kv, edges, coupling_scale)
    return dict(N=n, K=int(Kv.max()), var_states=Kv, edges=edges, log_unary=lu,
                pair_kind=PAIR_DENSE, pair=pair, name=f"protein_like{n}_d{avg_degree}_s{seed}")
