"""ctypes binding of libbp (include/bp.h) with the same entry-point names.

Argument marshalling only: every step of belief propagation runs in the HIP
library.  When PyTorch with a GPU is present, the graph's device memory is a
torch tensor (the library's workspace) and its work is ordered on torch's
current stream; otherwise the library allocates and uses the null stream.

Importing this module loads ``libbp.so`` from the package directory and raises
if it is missing: there is no fallback implementation.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbp.so")

BP_OK, BP_NOT_CONVERGED = 0, 1
BP_EINVAL, BP_ENOMEM, BP_EDEVICE, BP_ESTATE = -1, -2, -3, -4
BP_PAIR_ISING, BP_PAIR_SHARED, BP_PAIR_DENSE = 0, 1, 2
BP_LBP, BP_RBP, BP_RNBP, BP_RS = 0, 1, 2, 3
BP_FLAG_GENERIC_LAYOUT = 1
BP_FLAG_NO_MATRIX_CORES = 2
BP_FLAG_SPARSE_BUFFERS = 4
BP_FLAG_BF16_MATRIX_CORES = 16
BP_FLAG_SPLASH_BUFFERS = 8
BP_SERVER_GRAPHS = 1
BP_SERVER_AUTOTUNE = 2

SCHEDULES = {"lbp": BP_LBP, "rbp": BP_RBP, "rnbp": BP_RNBP, "rs": BP_RS}

# Every symbol include/bp.h declares.
EXPORTED = ["bp_default_opts", "bp_workspace_bytes", "bp_create_graph", "bp_run",
            "bp_run_noalloc", "bp_marginals", "bp_marginals_device", "bp_get_state", "bp_set_state",
            "bp_graph_info_get", "bp_destroy_graph", "bp_last_error",
            "bp_server_create", "bp_server_submit", "bp_server_step", "bp_server_result",
            "bp_server_counts", "bp_server_config", "bp_server_destroy",
            "bp_server_inject_failures"]


class BpError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libbp error {code}: {msg}")
        self.code = code


class bp_graph_desc(ctypes.Structure):
    _fields_ = [("num_vars", ctypes.c_int32), ("num_states", ctypes.c_int32),
                ("num_edges", ctypes.c_int64), ("edges", ctypes.c_void_p),
                ("log_unary", ctypes.c_void_p), ("pair_kind", ctypes.c_int32),
                ("flags", ctypes.c_uint32), ("coupling", ctypes.c_void_p),
                ("shared", ctypes.c_void_p), ("edge_scale", ctypes.c_void_p),
                ("pair", ctypes.c_void_p), ("stream", ctypes.c_void_p),
                ("workspace", ctypes.c_void_p), ("workspace_bytes", ctypes.c_uint64),
                ("var_states", ctypes.c_void_p)]


class bp_run_opts(ctypes.Structure):
    _fields_ = [("max_iters", ctypes.c_int64), ("check_every", ctypes.c_int32),
                ("dynamic_p", ctypes.c_int32), ("high_p", ctypes.c_double),
                ("ratio_threshold", ctypes.c_double), ("warm_start", ctypes.c_int32),
                ("profile", ctypes.c_int32), ("sparse", ctypes.c_int32),
                ("splash_depth", ctypes.c_int32)]


class bp_run_stats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int64), ("converged", ctypes.c_int32),
                ("reserved0", ctypes.c_int32), ("last_active", ctypes.c_int64),
                ("last_max_residual", ctypes.c_double), ("evaluated", ctypes.c_int64),
                ("committed", ctypes.c_int64), ("final_t", ctypes.c_int64),
                ("device_ms", ctypes.c_double), ("eval_kernel_ms", ctypes.c_double),
                ("eval_kernel_launches", ctypes.c_int64)]


class bp_iter_state(ctypes.Structure):
    _fields_ = [("t", ctypes.c_int64), ("prev_active", ctypes.c_int64)]


class bp_graph_info(ctypes.Structure):
    _fields_ = [("num_vars", ctypes.c_int32), ("num_states", ctypes.c_int32),
                ("num_edges", ctypes.c_int64), ("num_messages", ctypes.c_int64),
                ("layout", ctypes.c_int32), ("num_tiles", ctypes.c_int32),
                ("device_bytes", ctypes.c_uint64), ("eval_blocks", ctypes.c_int32),
                ("heavy_slots", ctypes.c_int32)]


class bp_server_desc(ctypes.Structure):
    _fields_ = [("arena_bytes", ctypes.c_uint64), ("arena", ctypes.c_void_p),
                ("stream", ctypes.c_void_p), ("max_graphs", ctypes.c_int32),
                ("options", ctypes.c_uint32)]


class bp_request(ctypes.Structure):
    _fields_ = [("schedule", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("eps", ctypes.c_double), ("p", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("opts", bp_run_opts)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                          "(hipcc --offload-arch=gfx950)")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    lib.bp_default_opts.argtypes = [ctypes.POINTER(bp_run_opts)]
    lib.bp_default_opts.restype = None
    lib.bp_workspace_bytes.argtypes = [ctypes.POINTER(bp_graph_desc),
                                       ctypes.POINTER(ctypes.c_uint64)]
    lib.bp_workspace_bytes.restype = ctypes.c_int
    lib.bp_create_graph.argtypes = [ctypes.POINTER(bp_graph_desc), ctypes.POINTER(P)]
    lib.bp_create_graph.restype = ctypes.c_int
    lib.bp_run.argtypes = [P, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_uint64,
                           ctypes.POINTER(bp_run_opts), ctypes.POINTER(bp_run_stats)]
    lib.bp_run.restype = ctypes.c_int
    lib.bp_run_noalloc.argtypes = lib.bp_run.argtypes
    lib.bp_run_noalloc.restype = ctypes.c_int
    lib.bp_marginals.argtypes = [P, P]
    lib.bp_marginals.restype = ctypes.c_int
    lib.bp_marginals_device.argtypes = [P, P]
    lib.bp_marginals_device.restype = ctypes.c_int
    lib.bp_get_state.argtypes = [P, P, ctypes.POINTER(bp_iter_state)]
    lib.bp_get_state.restype = ctypes.c_int
    lib.bp_set_state.argtypes = [P, P, ctypes.POINTER(bp_iter_state)]
    lib.bp_set_state.restype = ctypes.c_int
    lib.bp_graph_info_get.argtypes = [P, ctypes.POINTER(bp_graph_info)]
    lib.bp_graph_info_get.restype = ctypes.c_int
    lib.bp_destroy_graph.argtypes = [P]
    lib.bp_destroy_graph.restype = None
    lib.bp_last_error.argtypes = []
    lib.bp_last_error.restype = ctypes.c_char_p
    I64P = ctypes.POINTER(ctypes.c_int64)
    lib.bp_server_create.argtypes = [ctypes.POINTER(bp_server_desc), ctypes.POINTER(P)]
    lib.bp_server_create.restype = ctypes.c_int
    lib.bp_server_submit.argtypes = [P, ctypes.POINTER(bp_graph_desc), ctypes.POINTER(bp_request),
                                     I64P]
    lib.bp_server_submit.restype = ctypes.c_int
    lib.bp_server_step.argtypes = [P, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]
    lib.bp_server_step.restype = ctypes.c_int
    lib.bp_server_result.argtypes = [P, ctypes.c_int64, P, ctypes.POINTER(bp_run_stats)]
    lib.bp_server_result.restype = ctypes.c_int
    lib.bp_server_counts.argtypes = [P, I64P, I64P, I64P]
    lib.bp_server_counts.restype = ctypes.c_int
    lib.bp_server_destroy.argtypes = [P]
    lib.bp_server_destroy.restype = None
    I32P = ctypes.POINTER(ctypes.c_int32)
    lib.bp_server_config.argtypes = [P, I32P, I32P, I32P, ctypes.POINTER(ctypes.c_double),
                                     ctypes.c_int32, I32P]
    lib.bp_server_config.restype = ctypes.c_int
    lib.bp_server_inject_failures.argtypes = [P, ctypes.c_int32]
    lib.bp_server_inject_failures.restype = ctypes.c_int
    return lib


lib = _load()


def bp_last_error():
    return lib.bp_last_error().decode()


def _check(rc):
    if rc < 0:
        raise BpError(rc, bp_last_error())
    return rc


def bp_default_opts():
    o = bp_run_opts()
    lib.bp_default_opts(ctypes.byref(o))
    return o


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _make_desc(problem, flags=0):
    """Host arrays (kept alive in the returned tuple) and the descriptor.
    A problem with "var_states" (K_i per variable) passes ragged log_unary
    [sum K_i] and pair [sum_u K_a K_b] arrays."""
    N, K = int(problem["N"]), int(problem["K"])
    edges = np.ascontiguousarray(problem["edges"], dtype=np.int32).reshape(-1, 2)
    vs = problem.get("var_states")
    if vs is not None:
        vs = np.ascontiguousarray(vs, dtype=np.int32).reshape(N)
        lu = np.ascontiguousarray(problem["log_unary"], dtype=np.float64).reshape(-1)
    else:
        lu = np.ascontiguousarray(problem["log_unary"], dtype=np.float64).reshape(N, K)
    keep = [edges, lu, vs]

    def f64(name):
        v = problem.get(name)
        if v is None:
            return None
        a = np.ascontiguousarray(v, dtype=np.float64)
        keep.append(a)
        return a

    d = bp_graph_desc()
    d.num_vars, d.num_states, d.num_edges = N, K, edges.shape[0]
    d.edges, d.log_unary = _ptr(edges), _ptr(lu)
    d.pair_kind = int(problem["pair_kind"])
    d.flags = int(flags)
    d.coupling = _ptr(f64("coupling"))
    d.shared = _ptr(f64("shared"))
    d.edge_scale = _ptr(f64("edge_scale"))
    d.pair = _ptr(f64("pair"))
    d.var_states = _ptr(vs)
    return d, keep


def bp_workspace_bytes(problem, flags=0):
    d, _keep = _make_desc(problem, flags)
    n = ctypes.c_uint64()
    _check(lib.bp_workspace_bytes(ctypes.byref(d), ctypes.byref(n)))
    return int(n.value)


def _torch_cuda():
    try:
        import torch
    except ImportError:
        return None
    return torch if torch.cuda.is_available() else None


class Graph:
    """A problem resident on the GPU (bp_create_graph ... bp_destroy_graph).

    Binary Ising graphs are created with BP_FLAG_SPARSE_BUFFERS and
    BP_FLAG_SPLASH_BUFFERS unless sparse_buffers is False, so that all of their
    device memory is the one workspace tensor."""

    def __init__(self, problem, flags=0, use_torch=True, sparse_buffers=True):
        self.N, self.K = int(problem["N"]), int(problem["K"])
        self.M = int(np.asarray(problem["edges"]).reshape(-1, 2).shape[0])
        self.E = 2 * self.M
        # ragged problems (K_i per variable): flat message and belief arrays
        self._ragged = None
        if problem.get("var_states") is not None:
            vs = np.asarray(problem["var_states"], dtype=np.int64)
            ed = np.asarray(problem["edges"], dtype=np.int64).reshape(-1, 2)
            kdst = np.empty(self.E, np.int64)
            kdst[0::2], kdst[1::2] = vs[ed[:, 1]], vs[ed[:, 0]]
            self._ragged = (int(kdst.sum()), int(vs.sum()))
        if sparse_buffers and int(problem["pair_kind"]) == BP_PAIR_ISING:
            flags = int(flags) | BP_FLAG_SPARSE_BUFFERS | BP_FLAG_SPLASH_BUFFERS
        d, keep = _make_desc(problem, flags)
        self._workspace = None
        torch = _torch_cuda() if use_torch else None
        if torch is not None:
            n = ctypes.c_uint64()
            _check(lib.bp_workspace_bytes(ctypes.byref(d), ctypes.byref(n)))
            # torch's caching allocator owns the device memory; 256-byte alignment
            self._workspace = torch.empty(int(n.value) + 256, dtype=torch.uint8, device="cuda")
            base = self._workspace.data_ptr()
            d.workspace = base + (-base) % 256
            d.workspace_bytes = int(n.value)
            d.stream = torch.cuda.current_stream().cuda_stream
        h = ctypes.c_void_p()
        _check(lib.bp_create_graph(ctypes.byref(d), ctypes.byref(h)))
        del keep
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            lib.bp_destroy_graph(self.handle)
            self.handle = None
        self._workspace = None

    def __del__(self):
        self.close()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def info(self):
        i = bp_graph_info()
        _check(lib.bp_graph_info_get(self.handle, ctypes.byref(i)))
        return {f: getattr(i, f) for f, _ in i._fields_}

    def run(self, schedule="lbp", eps=1e-4, p=1.0, seed=0, max_iters=10000, check_every=16,
            dynamic_p=True, high_p=1.0, ratio_threshold=0.9, warm_start=False, profile=False,
            sparse=0, noalloc=False, splash_depth=2):
        """sparse: 0 full evaluation, 1 sparse re-evaluation, 2 full until n_t <= E/16
        (RnBP on K = 2 graphs only; see bp_run_opts in include/bp.h).  noalloc: call
        bp_run_noalloc (static per-GPU scratch, no events) instead of bp_run.
        splash_depth: depth h of residual splash ("rs")."""
        o = bp_default_opts()
        o.max_iters, o.check_every = int(max_iters), int(check_every)
        o.dynamic_p, o.high_p, o.ratio_threshold = int(bool(dynamic_p)), float(high_p), \
            float(ratio_threshold)
        o.warm_start, o.profile = int(bool(warm_start)), int(profile)
        o.sparse = int(sparse)
        o.splash_depth = int(splash_depth)
        s = bp_run_stats()
        sched = SCHEDULES[schedule] if isinstance(schedule, str) else int(schedule)
        fn = lib.bp_run_noalloc if noalloc else lib.bp_run
        rc = _check(fn(self.handle, sched, float(eps), float(p), int(seed),
                       ctypes.byref(o), ctypes.byref(s)))
        out = {f: getattr(s, f) for f, _ in s._fields_ if f != "reserved0"}
        out["converged"] = bool(out["converged"])
        out["status"] = rc
        return out

    def marginals(self):
        """[N, K] beliefs, or for a ragged problem [sum K_i] (variable-major)."""
        shape = (self._ragged[1],) if self._ragged else (self.N, self.K)
        out = np.empty(shape, dtype=np.float32)
        _check(lib.bp_marginals(self.handle, _ptr(out)))
        return out

    def marginals_device(self, out_tensor):
        """Write [N, K] FP32 beliefs (ragged: [sum K_i]) into a caller-owned CUDA tensor."""
        n = self._ragged[1] if self._ragged else self.N * self.K
        assert out_tensor.is_cuda and out_tensor.numel() == n
        _check(lib.bp_marginals_device(self.handle, ctypes.c_void_p(out_tensor.data_ptr())))
        return out_tensor

    def get_state(self):
        """Messages in canonical order, [E, K] or ragged [sum K_dst], and the
        iteration state."""
        shape = (self._ragged[0],) if self._ragged else (self.E, self.K)
        m = np.empty(shape, dtype=np.float32)
        st = bp_iter_state()
        _check(lib.bp_get_state(self.handle, _ptr(m), ctypes.byref(st)))
        return m, {"t": st.t, "prev_active": st.prev_active}

    def set_state(self, msgs=None, t=None, prev_active=-1):
        m = None
        if msgs is not None:
            shape = (self._ragged[0],) if self._ragged else (self.E, self.K)
            m = np.ascontiguousarray(msgs, dtype=np.float32).reshape(shape)
        st = None
        if t is not None:
            st = bp_iter_state(int(t), int(prev_active))
        _check(lib.bp_set_state(self.handle, _ptr(m), ctypes.byref(st) if st else None))


def bp_create_graph(problem, flags=0, use_torch=True):
    return Graph(problem, flags=flags, use_torch=use_torch)


def bp_run(graph, schedule, eps, p, seed, **opts):
    return graph.run(schedule, eps=eps, p=p, seed=seed, **opts)


def bp_run_noalloc(graph, schedule, eps, p, seed, **opts):
    return graph.run(schedule, eps=eps, p=p, seed=seed, noalloc=True, **opts)


def bp_marginals(graph):
    return graph.marginals()


def bp_get_state(graph):
    return graph.get_state()


def bp_set_state(graph, msgs=None, t=None, prev_active=-1):
    graph.set_state(msgs, t, prev_active)


def bp_destroy_graph(graph):
    graph.close()


class Server:
    """Batched serving of many K = 2 Ising graphs (bp_server_* in include/bp.h).

    submit() copies a problem and returns a request id; step(n) admits what fits,
    runs n batched iterations and retires finished graphs; result(id) returns
    (marginals, stats) once the request is retired, else None."""

    def __init__(self, arena_bytes, max_graphs=256, use_torch=True, graphs=False,
                 autotune=False):
        """graphs: replay each step's launches as a recorded HIP graph;
        autotune: choose the batched kernel's grid from timed live steps."""
        d = bp_server_desc()
        d.arena_bytes, d.max_graphs = int(arena_bytes), int(max_graphs)
        d.options = (BP_SERVER_GRAPHS if graphs else 0) | (BP_SERVER_AUTOTUNE if autotune else 0)
        self._arena = None
        torch = _torch_cuda() if use_torch else None
        if torch is not None:
            self._arena = torch.empty(int(arena_bytes) + 256, dtype=torch.uint8, device="cuda")
            base = self._arena.data_ptr()
            d.arena = base + (-base) % 256
            d.stream = torch.cuda.current_stream().cuda_stream
        h = ctypes.c_void_p()
        _check(lib.bp_server_create(ctypes.byref(d), ctypes.byref(h)))
        self.handle = h
        self._shapes = {}

    def close(self):
        if getattr(self, "handle", None):
            lib.bp_server_destroy(self.handle)
            self.handle = None
        self._arena = None

    def __del__(self):
        self.close()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def submit(self, problem, schedule="rnbp", eps=1e-4, p=0.5, seed=0, max_iters=10000,
               dynamic_p=True, high_p=1.0, ratio_threshold=0.9, sparse=0):
        d, keep = _make_desc(problem)
        r = bp_request()
        r.schedule = SCHEDULES[schedule] if isinstance(schedule, str) else int(schedule)
        r.eps, r.p, r.seed = float(eps), float(p), int(seed)
        r.opts = bp_default_opts()
        r.opts.max_iters = int(max_iters)
        r.opts.dynamic_p, r.opts.high_p = int(bool(dynamic_p)), float(high_p)
        r.opts.ratio_threshold = float(ratio_threshold)
        r.opts.sparse = int(sparse)  # the server accepts 0 only
        i = ctypes.c_int64()
        _check(lib.bp_server_submit(self.handle, ctypes.byref(d), ctypes.byref(r), ctypes.byref(i)))
        del keep
        self._shapes[i.value] = int(problem["N"])
        return i.value

    def step(self, launches=16):
        n = ctypes.c_int32()
        _check(lib.bp_server_step(self.handle, int(launches), ctypes.byref(n)))
        return n.value

    def result(self, rid):
        m = np.empty((self._shapes[rid], 2), dtype=np.float32)
        s = bp_run_stats()
        rc = lib.bp_server_result(self.handle, int(rid), _ptr(m), ctypes.byref(s))
        if rc == BP_ESTATE:
            return None
        _check(rc)
        del self._shapes[rid]
        out = {f: getattr(s, f) for f, _ in s._fields_ if f != "reserved0"}
        out["converged"] = bool(out["converged"])
        return m, out

    def config(self):
        """{"grid_blocks", "tuned", "candidates": [(blocks, ns per message per launch)]}"""
        g, t, n = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        cb = (ctypes.c_int32 * 16)()
        cn = (ctypes.c_double * 16)()
        _check(lib.bp_server_config(self.handle, ctypes.byref(g), ctypes.byref(t), cb, cn, 16,
                                    ctypes.byref(n)))
        return {"grid_blocks": g.value, "tuned": bool(t.value),
                "candidates": [(cb[i], cn[i]) for i in range(n.value)]}

    def inject_failures(self, admissions):
        """Test hook: the next `admissions` admissions fail (bp_server_inject_failures)."""
        _check(lib.bp_server_inject_failures(self.handle, int(admissions)))

    def counts(self):
        q, a, d = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _check(lib.bp_server_counts(self.handle, ctypes.byref(q), ctypes.byref(a), ctypes.byref(d)))
        return q.value, a.value, d.value
