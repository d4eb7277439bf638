"""FP64 CPU oracle for frontier-based sum-product belief propagation.

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  The product path (the HIP library and
its Python binding) never imports this package, and this package imports
nothing from the product path.

The arithmetic lives in ``oracle.c`` (literal Eq. (2) and Eq. (3), Alg. 1 with
the LBP / frontier-RBP / RnBP frontier rules, Philox4x32-10).  This module only
marshals numpy arrays through ctypes.

A problem is a plain dict:
    N, K            number of variables, states per variable
    edges           int32 [M, 2] undirected edges (a, b)
    log_unary       float64 [N, K], psi_i(x) = exp(log_unary[i, x])
    pair_kind       0 Ising (coupling [M]: psi = exp(J s_a s_b), s = -1/+1 for
                    states 0/1), 1 shared (shared [K, K] > 0 times edge_scale [M]),
                    2 dense (pair [M, K, K] > 0, first index = state of edges[u, 0])
Messages are in canonical order: row 2u is edges[u,0] -> edges[u,1], row 2u+1 the
reverse.

A problem with "var_states" (int32 [N], the states K_i of each variable; K is
then the largest) has ragged arrays: log_unary float64 [sum_i K_i], pair_kind 2
with pair float64 [sum_u K_a K_b] (the K_a x K_b table of edge u = (a, b),
state of a first, row after row); messages are then 1-D [sum_e K_dst(e)] in
canonical order (message e a distribution over its target's states) and
marginals 1-D [sum_i K_i].
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

LBP, RBP, RNBP = 0, 1, 2
PAIR_ISING, PAIR_SHARED, PAIR_DENSE = 0, 1, 2


class OracleStats(ctypes.Structure):
    _fields_ = [
        ("iterations", ctypes.c_int64),
        ("converged", ctypes.c_int32),
        ("pad0", ctypes.c_int32),
        ("last_active", ctypes.c_int64),
        ("last_max_residual", ctypes.c_double),
        ("evaluated", ctypes.c_int64),
        ("committed", ctypes.c_int64),
        ("final_t", ctypes.c_int64),
        ("last_prev_active", ctypes.c_int64),
    ]


def _configure(lib):
    P = ctypes.c_void_p
    lib.oracle_philox4x32_10.argtypes = [P, P, P]
    lib.oracle_philox4x32_10.restype = None
    lib.oracle_uniform.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                                   ctypes.c_uint32]
    lib.oracle_uniform.restype = ctypes.c_double
    lib.oracle_bp_run.argtypes = [
        ctypes.c_int, ctypes.c_int, ctypes.c_int64, P, P, ctypes.c_int, P, P, P, P,
        ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double,
        ctypes.c_int, ctypes.c_uint64, ctypes.c_int64, P, ctypes.c_int64, ctypes.c_int64,
        P, P, P, P, P, P, P]
    lib.oracle_bp_run.restype = ctypes.c_int
    lib.oracle_bp_evaluate.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int64, P, P,
                                       ctypes.c_int, P, P, P, P, P, P, P]
    lib.oracle_bp_evaluate.restype = ctypes.c_int
    lib.oracle_bp_beliefs.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int64, P, P, P, P]
    lib.oracle_bp_beliefs.restype = ctypes.c_int
    lib.oracle_bp_run_v.argtypes = lib.oracle_bp_run.argtypes[:4] + [P] + \
        lib.oracle_bp_run.argtypes[4:]
    lib.oracle_bp_run_v.restype = ctypes.c_int
    lib.oracle_bp_evaluate_v.argtypes = lib.oracle_bp_evaluate.argtypes[:4] + [P] + \
        lib.oracle_bp_evaluate.argtypes[4:]
    lib.oracle_bp_evaluate_v.restype = ctypes.c_int
    lib.oracle_bp_beliefs_v.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int64, P, P, P, P, P]
    lib.oracle_bp_beliefs_v.restype = ctypes.c_int
    lib.oracle_num_threads.argtypes = []
    lib.oracle_num_threads.restype = ctypes.c_int
    lib.oracle_srbp_run.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int64, P, P, ctypes.c_int,
                                    P, P, P, P, ctypes.c_double, ctypes.c_int64, P, P, P, P]
    lib.oracle_srbp_run.restype = ctypes.c_int
    lib.oracle_rs_run.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int64, P, P, ctypes.c_int,
                                  P, P, P, P, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                  ctypes.c_int64, P, P, P, P, P, P, P]
    lib.oracle_rs_run.restype = ctypes.c_int
    return lib


def load_library(path):
    """Load an oracle build from ``path`` (the tests load deliberately broken
    builds this way to show that the pins catch them)."""
    return _configure(ctypes.CDLL(path))


def _load(lib=None):
    global _lib
    if lib is not None:
        return lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build_oracle
        build_oracle.build()
    _lib = load_library(_LIB_PATH)
    return _lib


def load_openmp():
    """The timing build: the same oracle with its evaluation loop split over
    OpenMP threads (the benchmark's multi-core CPU baseline)."""
    from . import build_oracle
    if not os.path.exists(build_oracle.LIB_OMP):
        build_oracle.build()
    return load_library(build_oracle.LIB_OMP)


def num_threads(lib=None):
    return int(_load(lib).oracle_num_threads())


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _prep(problem):
    N = int(problem["N"])
    K = int(problem["K"])
    edges = np.ascontiguousarray(problem["edges"], dtype=np.int32).reshape(-1, 2)
    M = edges.shape[0]
    if problem.get("var_states") is not None:
        lu = np.ascontiguousarray(problem["log_unary"], dtype=np.float64).reshape(-1)
    else:
        lu = np.ascontiguousarray(problem["log_unary"], dtype=np.float64).reshape(N, K)
    kind = int(problem["pair_kind"])

    def f64(name):
        v = problem.get(name)
        return None if v is None else np.ascontiguousarray(v, dtype=np.float64)

    return N, K, M, edges, lu, kind, f64("coupling"), f64("shared"), f64("edge_scale"), \
        f64("pair")


def philox4x32_10(ctr, key, lib=None):
    """Philox4x32-10 bijection: 4 counter words, 2 key words -> 4 output words."""
    lib = _load(lib)
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib.oracle_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def uniform(seed, src, rank, t, lib=None):
    """U in [0, 1) of the random frontier filter for the message src -> j at
    iteration t, where j is the neighbour of rank `rank` of src (neighbours in
    ascending id order)."""
    return _load(lib).oracle_uniform(int(seed), int(src), int(rank), int(t))


def neighbour_rank(problem):
    """Rank of the target among the source's neighbours (ascending ids) for
    every canonical message id."""
    src, dst = canonical_src_dst(problem)
    order = np.lexsort((dst, src))
    rank = np.empty(len(src), np.int64)
    first = np.searchsorted(src[order], src[order], side="left")
    rank[order] = np.arange(len(src)) - first
    return rank


def _var_states(problem):
    v = problem.get("var_states")
    return None if v is None else np.ascontiguousarray(v, dtype=np.int32)


def message_offsets(problem):
    """Offsets [E + 1] of the canonical messages in a ragged message array (the
    states of each message's target)."""
    vs = _var_states(problem)
    _, dst = canonical_src_dst(problem)
    if vs is None:
        ks = np.full(len(dst), int(problem["K"]), np.int64)
    else:
        ks = vs[dst].astype(np.int64)
    return np.concatenate([[0], np.cumsum(ks)])


def _shapes(problem, N, K, E):
    """Shapes of the message and marginal arrays."""
    vs = _var_states(problem)
    if vs is None:
        return (E, K), (N, K)
    return (int(message_offsets(problem)[-1]),), (int(vs.sum()),)


def run(problem, schedule=LBP, eps=1e-4, p=1.0, high_p=1.0, ratio_threshold=0.9,
        dynamic_p=True, seed=0, max_iters=10000, init_msgs=None, t0=0, prev_active=-1,
        trace=False, lib=None):
    """Alg. 1 in FP64.  Returns a dict with msgs [E,K] (ragged: 1-D), marginals
    [N,K] (ragged: 1-D), stats and (if trace) per-evaluation arrays active /
    frontier / p / maxres."""
    lib = _load(lib)
    N, K, M, edges, lu, kind, cp, sh, sc, pr = _prep(problem)
    E = 2 * M
    vs = _var_states(problem)
    mshape, bshape = _shapes(problem, N, K, E)
    out_m = np.zeros(mshape, dtype=np.float64)
    out_b = np.zeros(bshape, dtype=np.float64)
    init = None
    if init_msgs is not None:
        init = np.ascontiguousarray(init_msgs, dtype=np.float64).reshape(mshape)
    st = OracleStats()
    tr = None
    if trace:
        L = int(max_iters) + 1
        tr = dict(active=np.zeros(L, np.int64), frontier=np.zeros(L, np.int64),
                  p=np.zeros(L, np.float64), maxres=np.zeros(L, np.float64))
    rc = lib.oracle_bp_run_v(
        N, K, M, _ptr(edges), _ptr(vs), _ptr(lu), kind, _ptr(cp), _ptr(sh), _ptr(sc), _ptr(pr),
        int(schedule), float(eps), float(p), float(high_p), float(ratio_threshold),
        int(bool(dynamic_p)), int(seed), int(max_iters), _ptr(init), int(t0),
        int(prev_active), _ptr(out_m), _ptr(out_b), ctypes.byref(st),
        _ptr(tr["active"]) if tr else None, _ptr(tr["frontier"]) if tr else None,
        _ptr(tr["p"]) if tr else None, _ptr(tr["maxres"]) if tr else None)
    if rc < 0:
        raise ValueError(f"oracle_bp_run failed with {rc}")
    res = dict(msgs=out_m, marginals=out_b, converged=bool(st.converged),
               iterations=st.iterations, last_active=st.last_active,
               last_max_residual=st.last_max_residual, evaluated=st.evaluated,
               committed=st.committed, final_t=st.final_t,
               last_prev_active=st.last_prev_active)
    if tr is not None:
        n = st.final_t - int(t0) + 1
        res["trace"] = {k: v[:n] for k, v in tr.items()}
    return res


def rs(problem, eps=1e-4, p=1.0 / 256, splash_depth=2, max_iters=10000, init_msgs=None,
       trace=False, lib=None):
    """Residual splash in frontier form: roots = the k = min(N, max(1, ceil(p E)))
    vertices of largest vertex residual (largest incoming residual), splash
    levels by BFS distance <= splash_depth, updates through the levels h..0..h.
    Returns msgs, marginals, stats and (if trace) active / committed / maxres."""
    lib = _load(lib)
    N, K, M, edges, lu, kind, cp, sh, sc, pr = _prep(problem)
    E = 2 * M
    out_m = np.zeros((E, K), np.float64)
    out_b = np.zeros((N, K), np.float64)
    init = None
    if init_msgs is not None:
        init = np.ascontiguousarray(init_msgs, dtype=np.float64).reshape(E, K)
    st = OracleStats()
    L = int(max_iters) + 1
    tr = dict(active=np.zeros(L, np.int64), committed=np.zeros(L, np.int64),
              maxres=np.zeros(L, np.float64)) if trace else None
    rc = lib.oracle_rs_run(N, K, M, _ptr(edges), _ptr(lu), kind, _ptr(cp), _ptr(sh), _ptr(sc),
                           _ptr(pr), float(eps), float(p), int(splash_depth), int(max_iters),
                           _ptr(init), _ptr(out_m), _ptr(out_b), ctypes.byref(st),
                           _ptr(tr["active"]) if tr else None,
                           _ptr(tr["committed"]) if tr else None,
                           _ptr(tr["maxres"]) if tr else None)
    if rc < 0:
        raise ValueError(f"oracle_rs_run failed with {rc}")
    res = dict(msgs=out_m, marginals=out_b, converged=bool(st.converged),
               iterations=st.iterations, last_active=st.last_active,
               last_max_residual=st.last_max_residual, evaluated=st.evaluated,
               committed=st.committed, final_t=st.final_t)
    if tr is not None:
        res["trace"] = {k: v[:st.final_t + 1] for k, v in tr.items()}
    return res


def srbp(problem, eps=1e-4, max_updates=100000, trace=False, lib=None):
    """Serial residual BP (one message at a time, largest residual first, ties
    by (target, source)).  Returns msgs, marginals, converged, updates and (if
    trace) the message id of every commit."""
    lib = _load(lib)
    N, K, M, edges, lu, kind, cp, sh, sc, pr = _prep(problem)
    E = 2 * M
    out_m = np.zeros((E, K), np.float64)
    out_b = np.zeros((N, K), np.float64)
    n = ctypes.c_int64()
    tr = np.zeros(max(int(max_updates), 1), np.int64) if trace else None
    rc = lib.oracle_srbp_run(N, K, M, _ptr(edges), _ptr(lu), kind, _ptr(cp), _ptr(sh), _ptr(sc),
                             _ptr(pr), float(eps), int(max_updates), _ptr(out_m), _ptr(out_b),
                             ctypes.byref(n), _ptr(tr))
    if rc < 0:
        raise ValueError(f"oracle_srbp_run failed with {rc}")
    out = dict(msgs=out_m, marginals=out_b, converged=rc == 0, updates=int(n.value))
    if trace:
        out["trace"] = tr[:n.value]
    return out


def evaluate(problem, msgs, lib=None):
    """f_BP(msgs) and the L-infinity residual of every message (no commit)."""
    lib = _load(lib)
    N, K, M, edges, lu, kind, cp, sh, sc, pr = _prep(problem)
    E = 2 * M
    vs = _var_states(problem)
    mshape, _ = _shapes(problem, N, K, E)
    m = np.ascontiguousarray(msgs, dtype=np.float64).reshape(mshape)
    cand = np.zeros(mshape, np.float64)
    res = np.zeros(E, np.float64)
    rc = lib.oracle_bp_evaluate_v(N, K, M, _ptr(edges), _ptr(vs), _ptr(lu), kind, _ptr(cp),
                                  _ptr(sh), _ptr(sc), _ptr(pr), _ptr(m), _ptr(cand), _ptr(res))
    if rc < 0:
        raise ValueError(f"oracle_bp_evaluate failed with {rc}")
    return cand, res


def beliefs(problem, msgs, lib=None):
    """Eq. (3) marginals [N, K] from a canonical message set."""
    lib = _load(lib)
    N, K, M, edges, lu, kind, cp, sh, sc, pr = _prep(problem)
    vs = _var_states(problem)
    mshape, bshape = _shapes(problem, N, K, 2 * M)
    m = np.ascontiguousarray(msgs, dtype=np.float64).reshape(mshape)
    out = np.zeros(bshape, np.float64)
    rc = lib.oracle_bp_beliefs_v(N, K, M, _ptr(edges), _ptr(vs), _ptr(lu), _ptr(m), _ptr(out))
    if rc < 0:
        raise ValueError(f"oracle_bp_beliefs failed with {rc}")
    return out


def canonical_src_dst(problem):
    """(src, dst) node ids of every canonical message id."""
    edges = np.asarray(problem["edges"], dtype=np.int64).reshape(-1, 2)
    src = np.empty(2 * len(edges), np.int64)
    dst = np.empty(2 * len(edges), np.int64)
    src[0::2], dst[0::2] = edges[:, 0], edges[:, 1]
    src[1::2], dst[1::2] = edges[:, 1], edges[:, 0]
    return src, dst
