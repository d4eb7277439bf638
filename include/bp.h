/*
 * bp.h -- C ABI of libbp: frontier-based sum-product belief propagation on
 * pairwise Markov random fields, on one AMD Instinct MI355X (gfx950).
 *
 * Problem (Sec. II-A, Eq. (1)): N discrete variables, variable i with K_i
 * states (K states each, or per-variable counts given by
 * bp_graph_desc.var_states), a positive unary potential psi_i per variable and
 * a positive pairwise potential psi_ij per undirected edge.  Every edge carries
 * two directed messages, so a graph with M edges has E = 2M messages; the
 * message i -> j is a distribution over the K_j states of j.  Messages start
 * uniform, are normalised after every update and are updated with Eq. (2)
 * (a sum over the K_i states of the source); beliefs follow Eq. (3).
 *
 * Solver (Alg. 1): repeat { evaluate f_BP(m^t) and the residual of Eq. (4) for
 * every message; stop if no residual exceeds eps; choose a frontier; commit
 * the frontier's new values }.  Frontier rules:
 *   BP_LBP   every message (synchronous loopy BP, Sec. II-B);
 *   BP_RBP   the k = max(1, ceil(p * E)) messages with the largest residuals,
 *            ties by (target, source) ascending (bulk greedy top-k, Sec. III-A);
 *   BP_RNBP  messages with residual > eps, each then kept with probability p_t
 *            (randomized BP, Sec. IV-A); with dynamic p, p_t is the low
 *            setting p when n_t / n_{t-1} > ratio_threshold, else high_p, where
 *            n_t counts messages with residual > eps (EdgeRatio, Sec. IV-A).
 *   BP_RS    residual splash in frontier form (Sec. II-B, Sec. III-A): the
 *            residual of a variable is the largest residual of its incoming
 *            messages; the k = min(N, max(1, ceil(p * E))) variables with the
 *            largest residuals (ties by id ascending) are the roots; level d
 *            (d = 0 .. h, h = bp_run_opts.splash_depth) holds every variable
 *            at graph distance exactly d from some root; the levels are
 *            updated in the order h, ..., 1, 0, 1, ..., h, each level
 *            recomputing every message out of its variables from the messages
 *            as they stand when the level starts, then committing them.
 *
 * Conventions
 *   - Residual: L-infinity norm of the change of the normalised message.
 *   - Canonical message order (used by bp_get_state / bp_set_state): for the
 *     undirected edge u = edges[u] = (a, b), row 2u is the message a -> b and
 *     row 2u + 1 is b -> a.
 *   - Random filter: for the message i -> j, where j is the neighbour of rank r
 *     of i (the neighbours of i in ascending id order, r = 0, 1, ...),
 *     U = (w >> 8) * 2^-24 where w is word r mod 4 of Philox4x32-10 (Salmon et
 *     al., SC'11) with key (seed & 0xffffffff, seed >> 32) and counter
 *     (i, r div 4, t, 0); a message is kept when U < p_t.  One Philox call
 *     serves four messages of a source.  Results do not depend on the storage
 *     order.
 *   - Messages are FP32 on the device; parameters are given in FP64 and
 *     rounded to FP32 when the graph is created.
 *   - Same inputs on the same device give bitwise identical results.
 *
 * Memory and threads
 *   - Every input array is host memory, read during the call and copied; the
 *     caller keeps ownership.  Output arrays are caller-owned host memory
 *     unless a function says device.
 *   - A graph owns its device memory (allocated at creation, or carved from
 *     the caller's workspace, see bp_graph_desc.workspace) until
 *     bp_destroy_graph.  All device work of a graph is ordered on its stream.
 *   - Calls on one graph must not overlap; different graphs are independent.
 *   - Errors: functions return a bp_status; bp_last_error() gives a
 *     thread-local description of the last failure in the calling thread.
 */
#ifndef BP_H
#define BP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BP_ABI_VERSION 2

typedef enum bp_status {
    BP_OK = 0,              /* success; for bp_run: converged */
    BP_NOT_CONVERGED = 1,   /* bp_run reached max_iters; state and marginals valid */
    BP_EINVAL = -1,         /* invalid argument or problem description */
    BP_ENOMEM = -2,         /* device or host allocation failed, or workspace too small */
    BP_EDEVICE = -3,        /* HIP runtime error (no device, launch failure, ...) */
    BP_ESTATE = -4          /* call not valid for the graph's current state */
} bp_status;

typedef enum bp_pair_kind {
    /* K = 2, psi_ij(x_a, x_b) = exp(J_u s_a s_b), spin s = -1 for state 0 and +1
     * for state 1; coupling[u] = J_u (any finite value). */
    BP_PAIR_ISING = 0,
    /* psi_u(x_a, x_b) = edge_scale[u] * shared[x_a][x_b]; shared [K][K] > 0 and
     * edge_scale [M] > 0.  (A per-edge scale cancels in the normalised Eq. (2);
     * it is validated but does not change any result.) */
    BP_PAIR_SHARED = 1,
    /* psi_u(x_a, x_b) = pair[u][x_a][x_b] > 0, [M][K][K]. */
    BP_PAIR_DENSE = 2
} bp_pair_kind;

typedef enum bp_schedule { BP_LBP = 0, BP_RBP = 1, BP_RNBP = 2, BP_RS = 3 } bp_schedule;

/* bp_graph_desc.flags */
#define BP_FLAG_GENERIC_LAYOUT 1u /* K = 2 Ising: keep [E][2] probabilities instead of
                                    one log-odds value per message */
#define BP_FLAG_NO_MATRIX_CORES 2u /* K = 32 with one symmetric shared table: take the
                                     Eq. (2) product on the FP32 vector units instead of
                                     the matrix cores (FP32 MFMA); same results within
                                     FP32 rounding */
#define BP_FLAG_BF16_MATRIX_CORES 16u /* K = 32 with one symmetric shared table: BF16
                                     operands on the matrix cores (FP32 accumulation):
                                     the cavity distribution and the table are rounded
                                     to 8-bit mantissas, so messages carry relative
                                     errors of order 2^-8 (not within the FP32 sweep
                                     tolerance); ignored with BP_FLAG_NO_MATRIX_CORES */
#define BP_FLAG_SPARSE_BUFFERS 4u  /* one-log-odds-per-message graphs: hold the buffers of
                                     sparse re-evaluation (bp_run_opts.sparse) in the
                                     graph's memory (counted by bp_workspace_bytes) instead
                                     of allocating them at the first sparse run; ignored
                                     for the [E][K] layout */
#define BP_FLAG_SPLASH_BUFFERS 8u  /* one-log-odds-per-message graphs: hold the buffers of
                                     BP_RS (variable residuals, level marks and level
                                     lists, 28 bytes per variable) in the graph's memory
                                     instead of allocating them at the first BP_RS run;
                                     BP_RS also needs the target index of the sparse
                                     buffers (BP_FLAG_SPARSE_BUFFERS); ignored for the
                                     [E][K] layout */

typedef struct bp_graph bp_graph;

typedef struct bp_graph_desc {
    int32_t num_vars;         /* N, 1 <= N < 2^31 */
    int32_t num_states;       /* K, 2 <= K <= 64; with var_states the largest K_i,
                                 2 <= K <= 128 */
    int64_t num_edges;        /* M, 0 <= M, 2M < 2^31 */
    const int32_t* edges;     /* host [M][2]: 0 <= a, b < N, a != b, no duplicate {a, b} */
    const double* log_unary;  /* host [N][K]: psi_i(x) = exp(log_unary[i][x]), finite */
    int32_t pair_kind;        /* bp_pair_kind */
    uint32_t flags;           /* BP_FLAG_* */
    const double* coupling;   /* host [M], BP_PAIR_ISING only, finite */
    const double* shared;     /* host [K][K], BP_PAIR_SHARED only, > 0 and finite */
    const double* edge_scale; /* host [M], BP_PAIR_SHARED only, > 0 and finite */
    const double* pair;       /* host [M][K][K], BP_PAIR_DENSE only, > 0 and finite */
    void* stream;             /* hipStream_t for all device work, NULL = null stream */
    void* workspace;          /* optional caller-owned device memory, 256-byte aligned,
                                 at least bp_workspace_bytes(); NULL = library allocates */
    uint64_t workspace_bytes;
    /* Optional host [N]: K_i, the number of states of each variable,
     * 2 <= K_i <= num_states (variables with their own state sets, e.g. the
     * side-chain models of Sec. IV-E).  NULL: every variable has num_states.
     * With var_states the pairwise potentials must be BP_PAIR_DENSE and the
     * arrays are ragged (rows concatenated in variable / edge order):
     *   log_unary  [sum_i K_i], row i holds log psi_i(0 .. K_i - 1);
     *   pair       [sum_u K_a K_b], edge u = (a, b) = edges[u] holds the
     *              K_a x K_b table psi_u(x_a, x_b), x_a major;
     * and so are the message and belief arrays of bp_get_state, bp_set_state
     * and bp_marginals (see there).  Such graphs keep K_j floats per message
     * (layout 2 of bp_graph_info) and run BP_LBP, BP_RNBP and BP_RBP. */
    const int32_t* var_states;
} bp_graph_desc;

typedef struct bp_run_opts {
    int64_t max_iters;        /* maximum number of commits (sweeps); default 10000 */
    int32_t check_every;      /* host polls the device convergence flag every this
                                 many iterations; default 16; results do not depend on it */
    int32_t dynamic_p;        /* BP_RNBP: 1 = EdgeRatio rule (default), 0 = p_t = p */
    double high_p;            /* BP_RNBP dynamic: high setting, default 1.0 */
    double ratio_threshold;   /* BP_RNBP dynamic: default 0.9 */
    int32_t warm_start;       /* 0 (default): messages reset to uniform 1/K and t = 0;
                                 1: continue from the current messages and iteration state */
    int32_t profile;          /* k > 0: time the evaluation kernel with HIP events on the
                                 graph's stream: whole chunks of back-to-back launches when
                                 it is the only kernel of an iteration, else every k-th
                                 launch */
    int32_t sparse;           /* BP_RNBP, BP_RBP on K = 2 graphs without oversized nodes (a node
                                 whose messages exceed one 512-slot tile): re-evaluate
                                 only the messages out of nodes that received a committed
                                 message (candidates and residuals of the others are kept).
                                 0 (default): full evaluation every iteration;
                                 1: sparse from the first iteration;
                                 2: full evaluation until n_t <= E / 16 at a host poll,
                                    sparse from then on.
                                 A sparse iteration costs about as much as a full one
                                 when n_t is near E / 16 and more when it is larger
                                 (its work is per variable, not tiled), so mode 1 is
                                 slower than the full evaluation while most messages
                                 stay active (strong coupling); mode 2 is the
                                 adaptive choice.
                                 Messages, iteration counts and residuals are bitwise those
                                 of the full evaluation; only `evaluated` differs.  The
                                 buffers (2 bytes per node and 4 per message) are in the
                                 graph's memory when it was created with
                                 BP_FLAG_SPARSE_BUFFERS; otherwise the first sparse run
                                 allocates them outside the workspace, held until
                                 bp_destroy_graph.  Other schedules and layouts:
                                 BP_EINVAL. */
    int32_t splash_depth;     /* BP_RS: depth h of a splash, 0, 1 or 2 (default 2, the
                                 depth the paper fixes); BP_RS runs on K = 2 Ising
                                 graphs in the one-log-odds-per-message layout and
                                 takes its buffers as BP_FLAG_SPLASH_BUFFERS says */
} bp_run_opts;

typedef struct bp_run_stats {
    int64_t iterations;        /* commits performed by this call */
    int32_t converged;         /* 1 if an evaluation found no residual > eps */
    int32_t reserved0;
    int64_t last_active;       /* n_t of the last evaluation */
    double last_max_residual;  /* max residual of the last evaluation */
    int64_t evaluated;         /* Eq. (2) evaluations performed by this call */
    int64_t committed;         /* messages committed by this call */
    int64_t final_t;           /* global iteration number of the last evaluation */
    double device_ms;          /* stream time of the whole call (HIP events) */
    double eval_kernel_ms;     /* profile: summed duration of the timed evaluation launches */
    int64_t eval_kernel_launches; /* profile: number of evaluation launches timed */
} bp_run_stats;

/* Iteration state carried between runs (checkpoint / resume, Alg. 1 loop).
 * p_t is not stored: BP_RNBP with dynamic p derives it when iteration t is
 * evaluated, from n_t (that evaluation's count) and n_{t-1} = prev_active:
 * p_t = p (the low setting) if prev_active > 0 and n_t / prev_active >
 * ratio_threshold, else high_p (EdgeRatio, Sec. IV-A). */
typedef struct bp_iter_state {
    int64_t t;            /* global iteration number of the next evaluation (the
                             RNG counter word of the random filter) */
    int64_t prev_active;  /* n_{t-1}, or -1 if none (then p_t = high_p) */
} bp_iter_state;

typedef struct bp_graph_info {
    int32_t num_vars;
    int32_t num_states;
    int64_t num_edges;
    int64_t num_messages;     /* E = 2M */
    int32_t layout;           /* 0 = one log-odds value per message (K = 2 Ising with
                                 fewer than 2^30 - 512 messages and variables),
                                 1 = [E][K] probabilities,
                                 2 = K_j probabilities per message (var_states) */
    int32_t num_tiles;        /* node tiles of the evaluation kernel */
    uint64_t device_bytes;    /* device memory held by the graph */
    int32_t eval_blocks;      /* one-log-odds-per-message graphs: the persistent grid of
                                 the evaluation kernel chosen by launch-shape tuning (the
                                 first run of at least 32 iterations times 8 launches at
                                 each of 1, 2, 4 blocks per compute unit and every
                                 resident block, and keeps the fastest; results do not
                                 depend on it); 0 until tuned */
    int32_t heavy_slots;      /* layout 2: messages whose source variable has many
                                 states, neighbours or table entries, each evaluated
                                 by a wave of its own (the others share one wave per
                                 variable); 0 for the other layouts */
} bp_graph_info;

/* Fill *opts with the defaults listed in bp_run_opts. */
void bp_default_opts(bp_run_opts* opts);

/* Device bytes bp_create_graph needs for this description (for a caller-owned
 * workspace).  Validates the description; returns BP_OK or BP_EINVAL. */
int bp_workspace_bytes(const bp_graph_desc* desc, uint64_t* bytes);

/* Validate the problem (ranges, self-loops, duplicate edges, positivity and
 * finiteness of potentials, K range), build the device layout (directed
 * messages grouped by source node and sorted by target inside a source,
 * reverse-message index, node tiles), upload it and set messages to uniform.
 * *out receives the handle.
 * Errors: BP_EINVAL, BP_ENOMEM, BP_EDEVICE; *out is NULL on error. */
int bp_create_graph(const bp_graph_desc* desc, bp_graph** out);

/* Run Alg. 1 with the given frontier rule (see top of file).
 *   eps   convergence and filter threshold, >= 0 and finite
 *   p     BP_RBP: fraction of messages per iteration; BP_RNBP: the low setting
 *         (static: the probability); BP_RS: roots = ceil(p * E) capped at N;
 *         in (0, 1]; ignored by BP_LBP
 *   seed  Philox key for BP_RNBP; ignored otherwise
 *   opts  NULL = defaults; stats NULL = not returned.
 * Returns BP_OK if converged, BP_NOT_CONVERGED at max_iters, negative on error.
 * On return the graph holds the final messages and iteration state. */
int bp_run(bp_graph* g, int schedule, double eps, double p, uint64_t seed,
           const bp_run_opts* opts, bp_run_stats* stats);

/* bp_run for callers that cannot allocate device memory or create events at
 * run time: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  Same arguments, results and return codes as bp_run (the
 * messages, statistics and iteration state are bitwise those of bp_run),
 * except:
 *   - the run's scratch (iteration state, per-iteration counters and the
 *     top-k tie counts: about 49 KiB plus 4 bytes per 4096 messages) is taken
 *     from a static device array of 1 MiB that each GPU holds until the
 *     process ends, not from the graph's memory; a graph whose scratch would
 *     not fit (more than about 1.0e9 messages) is rejected with BP_EINVAL;
 *   - no HIP events are created: stats->device_ms and the profile fields are
 *     0, and opts->profile must be 0 (BP_EINVAL otherwise);
 *   - opts->sparse != 0 needs a graph created with BP_FLAG_SPARSE_BUFFERS
 *     (BP_EINVAL otherwise), so that no buffer is allocated.
 * All calls on one GPU share that GPU's array and it keeps the last call's
 * contents (each call clears what must start at zero with a kernel): calls
 * that overlap on one GPU, from other threads or on other streams, race and
 * give wrong results; the caller serialises them.  The graph must exist
 * already (created with a caller workspace if nothing may be allocated). */
int bp_run_noalloc(bp_graph* g, int schedule, double eps, double p, uint64_t seed,
                   const bp_run_opts* opts, bp_run_stats* stats);

/* Eq. (3) beliefs from the current messages into host [N][K] FP32; each row
 * sums to 1 up to rounding.  Graphs with var_states: host [sum_i K_i], the
 * K_i beliefs of variable i after those of variables 0 .. i - 1. */
int bp_marginals(bp_graph* g, float* out);

/* Same, into caller-owned device memory [N][K] FP32, ordered on the graph's
 * stream (no synchronisation). */
int bp_marginals_device(bp_graph* g, float* out_device);

/* Copy the current messages to host [E][K] FP32 in canonical order and the
 * iteration state to *st (either may be NULL).  Graphs with var_states: host
 * [sum_c K_dst(c)], the K_j values of canonical message c (target j) after
 * those of messages 0 .. c - 1. */
int bp_get_state(bp_graph* g, float* msgs, bp_iter_state* st);

/* Replace the messages (host [E][K] FP32, canonical order, each row positive;
 * rows are renormalised to sum 1; ragged as bp_get_state for graphs with
 * var_states) and/or the iteration state (either may be NULL).  Use with
 * bp_run_opts.warm_start = 1. */
int bp_set_state(bp_graph* g, const float* msgs, const bp_iter_state* st);

/* Sizes and layout of a graph. */
int bp_graph_info_get(const bp_graph* g, bp_graph_info* info);

/* Release the graph's device memory (not a caller workspace) and the handle.
 * NULL is ignored. */
void bp_destroy_graph(bp_graph* g);

/* Description of the last error in the calling thread ("" if none). */
const char* bp_last_error(void);

/* ------------------------------------------------------------------------
 * Serving: many independent graphs solved together.
 *
 * A server keeps up to max_graphs graphs resident in one device arena and
 * evaluates one iteration of every resident graph per kernel launch (a
 * persistent grid; each block runs a contiguous range of the graphs' tiles
 * through the same pipelined tile loop as bp_run), so small graphs share the
 * GPU instead of each paying for whole-GPU launches.  Requests wait in FIFO order until
 * the arena has room, join the batch at the next step, and leave it when
 * they converge or reach max_iters.  Every graph advances exactly as bp_run
 * would advance it alone (same tiles, arithmetic, counters and random keys),
 * so a result does not depend on which other graphs shared its launches:
 * it is bitwise identical to bp_run with the same arguments on a fresh graph.
 * Requests must use BP_PAIR_ISING with the one-log-odds-per-message layout
 * (no BP_FLAG_GENERIC_LAYOUT, fewer than 2^30 - 512 messages) and the
 * BP_LBP or BP_RNBP schedule.
 * ------------------------------------------------------------------------ */
typedef struct bp_server bp_server;

/* bp_server_desc.options */
#define BP_SERVER_GRAPHS 1u    /* record the launches of a step once as a HIP graph of
                                  kernel nodes and replay it (re-recorded when the set of
                                  resident graphs or the launch shape changes) */
#define BP_SERVER_AUTOTUNE 2u  /* choose the persistent grid of the batched kernel (blocks
                                  per compute unit) from HIP-event timings of live steps;
                                  results do not depend on the choice */

typedef struct bp_server_desc {
    uint64_t arena_bytes;   /* device memory for resident graphs (> 0) */
    void* arena;            /* optional caller-owned device memory, 256-byte aligned,
                               at least arena_bytes; NULL = library allocates */
    void* stream;           /* hipStream_t for all device work, NULL = null stream */
    int32_t max_graphs;     /* most graphs resident at once, 1 ... 65536 */
    uint32_t options;       /* BP_SERVER_* */
} bp_server_desc;

typedef struct bp_request {
    int32_t schedule;       /* BP_LBP or BP_RNBP */
    int32_t reserved;
    double eps;             /* as bp_run */
    double p;               /* as bp_run (RnBP low setting) */
    uint64_t seed;          /* as bp_run */
    bp_run_opts opts;       /* max_iters, dynamic_p, high_p, ratio_threshold as bp_run;
                               check_every, warm_start and profile are ignored;
                               sparse must be 0 (BP_EINVAL otherwise) */
} bp_request;

/* Create a server.  Errors: BP_EINVAL, BP_ENOMEM, BP_EDEVICE; *out NULL on error. */
int bp_server_create(const bp_server_desc* desc, bp_server** out);

/* Validate and copy a request (the caller keeps ownership of every array in
 * *graph; graph->stream and graph->workspace are ignored).  *id receives the
 * request's id (> 0).  A graph that needs more than the whole arena is
 * rejected with BP_ENOMEM.  Errors: BP_EINVAL, BP_ENOMEM. */
int bp_server_submit(bp_server* s, const bp_graph_desc* graph, const bp_request* req,
                     int64_t* id);

/* Admit queued requests that fit, run `launches` batched iterations, then
 * retire the graphs that converged or reached max_iters (their results become
 * available to bp_server_result).  *finished (may be NULL) receives the number
 * retired by this call.  Synchronises the server's stream. */
int bp_server_step(bp_server* s, int32_t launches, int32_t* finished);

/* Result of a retired request: Eq. (3) beliefs into host [N][2] FP32 and the
 * run statistics as bp_run reports them (device_ms and the profile fields are
 * 0).  Returns BP_OK and forgets the request, BP_ESTATE if the request is
 * still queued or resident, BP_EINVAL for an unknown id.  A request whose
 * admission failed (its graph could not be created in the arena) is retired
 * without a result: this call returns that error (BP_ENOMEM, BP_EDEVICE) and
 * forgets the request; the other requests are not affected. */
int bp_server_result(bp_server* s, int64_t id, float* marginals, bp_run_stats* stats);

/* Requests waiting for room, resident in the batch, and retired but not yet
 * fetched (any pointer may be NULL). */
int bp_server_counts(const bp_server* s, int64_t* queued, int64_t* resident, int64_t* retired);

/* The batched kernel's launch shape: *grid_blocks (persistent blocks per
 * launch), *tuned (1 once the autotuner has chosen), and the autotuner's
 * measurements: for up to max_entries candidates, blocks per launch and
 * device nanoseconds per resident message per launch of the last tuning round
 * (*entries receives the count).  Any pointer may be NULL. */
int bp_server_config(const bp_server* s, int32_t* grid_blocks, int32_t* tuned,
                     int32_t* cand_blocks, double* cand_ns_per_msg, int32_t max_entries,
                     int32_t* entries);

/* Release the server's device memory (not a caller arena) and every request.
 * NULL is ignored. */
void bp_server_destroy(bp_server* s);

/* Test hook for the failure path of admission: the next `admissions`
 * admissions fail as a device error during graph creation would (the request
 * is retired with BP_EDEVICE, its arena room returned).  0 turns it off. */
int bp_server_inject_failures(bp_server* s, int32_t admissions);

#ifdef __cplusplus
}
#endif
#endif /* BP_H */
