/*
 * oracle.c -- plain FP64 CPU reference for frontier-based sum-product belief
 * propagation (LBP, frontier residual BP, randomized BP).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code with the HIP library.
 *
 * Written for obviousness, not speed:
 *   - every message is recomputed with the literal product of Eq. (2), in the
 *     probability domain, over the neighbours of the source except the target
 *     (no log-domain aggregate, no cavity division);
 *   - beliefs follow Eq. (3) literally;
 *   - the loop is Alg. 1 with the lookahead reading of its three steps:
 *     evaluate f_BP(m^t) for every message, test convergence, pick the
 *     frontier, commit (all commits of one iteration read m^t only);
 *   - the random filter draws from Philox4x32-10 (Salmon, Moraes, Dror, Shaw,
 *     "Parallel random numbers: as easy as 1, 2, 3", SC'11), written here from
 *     that paper's definition.
 *
 * Message ids are canonical: for undirected edge u = (a, b) given in input
 * order, id 2u is a->b and id 2u+1 is b->a (two messages per edge, Sec. II-A).
 *
 * Variables may have different numbers of states (the _v entry points take
 * the per-variable counts K_i; the others use one K for every variable).  A
 * message i -> j is a distribution over the K_j states of its target; arrays
 * over variables or messages are stored row after row with these lengths
 * ("ragged": unaries [sum_i K_i], messages [sum_e K_dst(e)] in canonical
 * order, dense tables [sum_u K_a K_b] with the state of edges[u][0] first).
 */
#include <limits.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_PAIR_ISING 0
#define OR_PAIR_SHARED 1
#define OR_PAIR_DENSE 2

#define OR_LBP 0
#define OR_RBP 1
#define OR_RNBP 2

typedef struct {
    int64_t iterations;        /* commits performed (sweeps) */
    int32_t converged;         /* 1 if some evaluation found n_t == 0 */
    int32_t pad0;
    int64_t last_active;       /* n_t of the last evaluation */
    double last_max_residual;  /* R_t of the last evaluation */
    int64_t evaluated;         /* Eq. (2) evaluations, all iterations */
    int64_t committed;         /* messages written, all iterations */
    int64_t final_t;           /* t of the last evaluation (global clock) */
    int64_t last_prev_active;  /* n_{t-1} seen by the last evaluation, -1 if none */
} oracle_stats;

/* ------------------------------------------------------------------ */
/* Philox4x32-10 (SC'11): 10 rounds of the 4x32 Philox bijection.       */
/* ------------------------------------------------------------------ */
void oracle_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2],
                          uint32_t out[4]) {
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;  /* multipliers */
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;  /* Weyl key bumps */
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += W0;
            k1 += W1;
        }
        uint64_t p0 = (uint64_t)M0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)M1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Uniform draw for the random filter of Sec. IV-A.  The message i -> j, where j
 * is the neighbour of rank r of i (neighbours of i in ascending id order,
 * r = 0, 1, ...), takes word r mod 4 of Philox4x32-10 with key = seed split into
 * two 32-bit words and counter = (i, r div 4, t, 0); the top 24 bits of that
 * word give U in [0, 1).  One call serves four messages of one source. */
double oracle_uniform(uint64_t seed, uint32_t src, uint32_t rank, uint32_t t) {
    uint32_t ctr[4] = {src, rank / 4u, t, 0u};
    uint32_t key[2] = {(uint32_t)(seed & 0xFFFFFFFFu), (uint32_t)(seed >> 32)};
    uint32_t out[4];
    oracle_philox4x32_10(ctr, key, out);
    return (double)(out[rank % 4u] >> 8) * (1.0 / 16777216.0);
}

/* ------------------------------------------------------------------ */
/* Model                                                               */
/* ------------------------------------------------------------------ */
typedef struct {
    int N, K;                  /* K: the largest state count */
    int64_t M, E;
    const int32_t* edges;      /* [M][2] */
    int32_t* Kv;               /* [N] states of each variable */
    int64_t* uoff;             /* [N+1] row offsets of per-variable arrays */
    int64_t* moff;             /* [E+1] row offsets of messages (K of the target) */
    int64_t* poff;             /* [M+1] offsets of dense tables (K_a K_b) */
    double* unary;             /* psi_i(x) = exp(log_unary), ragged [sum K_i] */
    int pair_kind;
    const double* coupling;    /* Ising J, [M] */
    const double* shared;      /* [K][K] */
    const double* edge_scale;  /* [M] */
    const double* pair;        /* ragged [sum_u K_a K_b] */
    int64_t* in_ptr;           /* [N+1]: incoming message ids grouped by target */
    int64_t* in_ids;           /* [E] */
    int32_t* rank;             /* [E]: rank of the target among the source's neighbours */
} model_t;

static int msg_src(const model_t* g, int64_t e) {
    int64_t u = e >> 1;
    return (e & 1) ? g->edges[2 * u + 1] : g->edges[2 * u];
}
static int msg_dst(const model_t* g, int64_t e) {
    int64_t u = e >> 1;
    return (e & 1) ? g->edges[2 * u] : g->edges[2 * u + 1];
}

/* Pairwise potential of the undirected edge u, first argument the state of
 * edges[u][0], second the state of edges[u][1] (Eq. (1)). */
static double pair_psi(const model_t* g, int64_t u, int xa, int xb) {
    int K = g->K;
    switch (g->pair_kind) {
    case OR_PAIR_ISING: {
        /* psi = exp(J * s_a * s_b) with spins s = -1 (state 0), +1 (state 1) */
        double sa = xa ? 1.0 : -1.0, sb = xb ? 1.0 : -1.0;
        return exp(g->coupling[u] * sa * sb);
    }
    case OR_PAIR_SHARED:
        return g->edge_scale[u] * g->shared[xa * K + xb];
    default:
        return g->pair[g->poff[u] + xa * g->Kv[g->edges[2 * u + 1]] + xb];
    }
}

/* psi_{i,j}(x_i, x_j) for the directed message e = i -> j. */
static double msg_psi(const model_t* g, int64_t e, int xi, int xj) {
    int64_t u = e >> 1;
    return (e & 1) ? pair_psi(g, u, xj, xi) : pair_psi(g, u, xi, xj);
}

/* var_states: the K_i of every variable, or NULL for K states each.  With
 * var_states only dense tables are accepted; K is then the largest K_i. */
static int build_model(model_t* g, int N, int K, int64_t M, const int32_t* edges,
                       const int32_t* var_states, const double* log_unary, int pair_kind,
                       const double* coupling, const double* shared,
                       const double* edge_scale, const double* pair) {
    memset(g, 0, sizeof(*g));
    g->N = N; g->K = K; g->M = M; g->E = 2 * M;
    g->edges = edges;
    g->pair_kind = pair_kind;
    g->coupling = coupling; g->shared = shared; g->edge_scale = edge_scale;
    g->pair = pair;
    g->Kv = (int32_t*)malloc(sizeof(int32_t) * (size_t)N + 1);
    g->uoff = (int64_t*)malloc(sizeof(int64_t) * ((size_t)N + 1));
    g->moff = (int64_t*)malloc(sizeof(int64_t) * ((size_t)g->E + 1));
    g->poff = (int64_t*)malloc(sizeof(int64_t) * ((size_t)M + 1));
    g->in_ptr = (int64_t*)calloc((size_t)N + 1, sizeof(int64_t));
    g->in_ids = (int64_t*)malloc(sizeof(int64_t) * (size_t)g->E + 1);
    if (!g->Kv || !g->uoff || !g->moff || !g->poff || !g->in_ptr || !g->in_ids) return -2;
    if (var_states && pair_kind != OR_PAIR_DENSE) return -1;
    g->uoff[0] = 0;
    for (int i = 0; i < N; ++i) {
        g->Kv[i] = var_states ? var_states[i] : K;
        if (g->Kv[i] < 2 || g->Kv[i] > K) return -1;
        g->uoff[i + 1] = g->uoff[i] + g->Kv[i];
    }
    g->moff[0] = 0;
    for (int64_t e = 0; e < g->E; ++e) g->moff[e + 1] = g->moff[e] + g->Kv[msg_dst(g, e)];
    g->poff[0] = 0;
    for (int64_t u = 0; u < M; ++u)
        g->poff[u + 1] = g->poff[u] + (int64_t)g->Kv[edges[2 * u]] * g->Kv[edges[2 * u + 1]];
    g->unary = (double*)malloc(sizeof(double) * (size_t)g->uoff[N] + 1);
    if (!g->unary) return -2;
    for (int64_t i = 0; i < g->uoff[N]; ++i) g->unary[i] = exp(log_unary[i]);
    /* neighbour lists Gamma_i, as incoming message ids, in message-id order */
    for (int64_t e = 0; e < g->E; ++e) g->in_ptr[msg_dst(g, e) + 1]++;
    for (int i = 0; i < N; ++i) g->in_ptr[i + 1] += g->in_ptr[i];
    int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * ((size_t)N + 1));
    if (!fill) return -2;
    memcpy(fill, g->in_ptr, sizeof(int64_t) * ((size_t)N + 1));
    for (int64_t e = 0; e < g->E; ++e) g->in_ids[fill[msg_dst(g, e)]++] = e;
    free(fill);
    /* rank of j among the neighbours of i for every message i -> j: the
     * incoming list of i holds the messages k -> i, one per neighbour k, and the
     * message i -> k is the other direction (id ^ 1) of the same edge */
    g->rank = (int32_t*)malloc(sizeof(int32_t) * (size_t)g->E + 1);
    if (!g->rank) return -2;
    for (int i = 0; i < N; ++i) {
        for (int64_t a = g->in_ptr[i]; a < g->in_ptr[i + 1]; ++a) {
            int k = msg_src(g, g->in_ids[a]);
            int32_t r = 0;
            for (int64_t b = g->in_ptr[i]; b < g->in_ptr[i + 1]; ++b)
                if (msg_src(g, g->in_ids[b]) < k) ++r;
            g->rank[g->in_ids[a] ^ 1] = r;
        }
    }
    return 0;
}

static void free_model(model_t* g) {
    free(g->Kv);
    free(g->uoff);
    free(g->moff);
    free(g->poff);
    free(g->unary);
    free(g->in_ptr);
    free(g->in_ids);
    free(g->rank);
}

/* A product of many factors below 1 leaves the double range once a node has a
 * few hundred neighbours; products are therefore kept as mant * 2^ex with
 * mant renormalised by frexp after every factor.  This is the same literal
 * product (one rounding per factor) with a wider exponent. */
typedef struct {
    double mant;
    long ex;
} xprod;

static void xmul(xprod* p, double v) {
    int e;
    p->mant = frexp(p->mant * v, &e);
    p->ex += e;
}

/* Scale the K products by a common power of two so the largest is O(1). */
static void xprod_to_double(const xprod* p, int K, double* out) {
    long top = LONG_MIN;
    for (int x = 0; x < K; ++x)
        if (p[x].mant != 0.0 && p[x].ex > top) top = p[x].ex;
    for (int x = 0; x < K; ++x)
        out[x] = p[x].mant == 0.0 ? 0.0 : ldexp(p[x].mant, (int)(p[x].ex - top));
}

/* Eq. (2) for message e = i -> j, from the message set m (read only):
 *   c(x_j) = sum_{x_i} psi_ij(x_i, x_j) psi_i(x_i) prod_{k in Gamma_i \ j} m_{k->i}(x_i)
 * then normalised to sum 1 (Sec. II-A); x_i ranges over the K_i states of i,
 * x_j over the K_j of j.  pw holds K_i products, work K_i doubles. */
static void eval_message(const model_t* g, const double* m, int64_t e, double* out,
                         double* work, xprod* pw) {
    int i = msg_src(g, e);
    int Ki = g->Kv[i], Kj = g->Kv[msg_dst(g, e)];
    int64_t back = e ^ 1; /* the message j -> i, excluded from the product */
    for (int xi = 0; xi < Ki; ++xi) {
        xprod prod = {1.0, 0};
        xmul(&prod, g->unary[g->uoff[i] + xi]);
        for (int64_t q = g->in_ptr[i]; q < g->in_ptr[i + 1]; ++q) {
            int64_t f = g->in_ids[q];
            if (f == back) continue;
            xmul(&prod, m[g->moff[f] + xi]);
        }
        pw[xi] = prod;
    }
    xprod_to_double(pw, Ki, work);
    double z = 0.0;
    for (int xj = 0; xj < Kj; ++xj) {
        double s = 0.0;
        for (int xi = 0; xi < Ki; ++xi) s += msg_psi(g, e, xi, xj) * work[xi];
        out[xj] = s;
        z += s;
    }
    for (int xj = 0; xj < Kj; ++xj) out[xj] /= z;
}

/* f_BP(m) for every message and its residual (Eq. (4), L-infinity norm).
 * Every candidate reads m only, so the messages are independent: the timing
 * build (liboracle_omp.so, compiled with OpenMP) splits them over threads,
 * the parity build ignores the pragmas.  Each message is computed the same way
 * in both, so both give the same bits. */
static int evaluate_all(const model_t* g, const double* m, double* cand, double* res) {
    int K = g->K;
    int bad = 0;
#pragma omp parallel
    {
        double* work = (double*)malloc(sizeof(double) * (size_t)K);
        xprod* pw = (xprod*)malloc(sizeof(xprod) * (size_t)K);
        int ok = work && pw;
        if (!ok) {
#pragma omp atomic write
            bad = 1;
        }
#pragma omp for schedule(static)
        for (int64_t e = 0; e < g->E; ++e) {
            if (!ok) continue;
            int64_t o = g->moff[e];
            eval_message(g, m, e, cand + o, work, pw);
            double r = 0.0;
            for (int64_t q = o; q < g->moff[e + 1]; ++q) {
                double d = fabs(cand[q] - m[q]);
                if (d > r) r = d;
            }
            res[e] = r;
        }
        free(work);
        free(pw);
    }
    return bad ? -2 : 0;
}

/* Threads the evaluation uses (1 in the parity build). */
int oracle_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Eq. (3): b_i(x) proportional to psi_i(x) prod_{k in Gamma_i} m_{k->i}(x). */
static int beliefs(const model_t* g, const double* m, double* out) {
    xprod* pw = (xprod*)malloc(sizeof(xprod) * (size_t)g->K);
    if (!pw) return -2;
    for (int i = 0; i < g->N; ++i) {
        int Ki = g->Kv[i];
        for (int x = 0; x < Ki; ++x) {
            xprod b = {1.0, 0};
            xmul(&b, g->unary[g->uoff[i] + x]);
            for (int64_t q = g->in_ptr[i]; q < g->in_ptr[i + 1]; ++q)
                xmul(&b, m[g->moff[g->in_ids[q]] + x]);
            pw[x] = b;
        }
        double* row = out + g->uoff[i];
        xprod_to_double(pw, Ki, row);
        double z = 0.0;
        for (int x = 0; x < Ki; ++x) z += row[x];
        for (int x = 0; x < Ki; ++x) row[x] /= z;
    }
    free(pw);
    return 0;
}

/* Uniform messages: 1/K_j for every entry of every message into j (Sec. II-A). */
static void uniform_messages(const model_t* g, double* m) {
    for (int64_t e = 0; e < g->E; ++e)
        for (int64_t q = g->moff[e]; q < g->moff[e + 1]; ++q)
            m[q] = 1.0 / g->Kv[msg_dst(g, e)];
}

/* Commit the candidate of message e. */
static void commit_message(const model_t* g, double* m, const double* cand, int64_t e) {
    for (int64_t q = g->moff[e]; q < g->moff[e + 1]; ++q) m[q] = cand[q];
}

/* Ordering for the greedy frontier of Sec. III-A: larger residual first; equal
 * residuals by (target, source) ascending. */
static const model_t* g_sort_model;
static const double* g_sort_res;
static int cmp_topk(const void* pa, const void* pb) {
    int64_t a = *(const int64_t*)pa, b = *(const int64_t*)pb;
    double ra = g_sort_res[a], rb = g_sort_res[b];
    if (ra > rb) return -1;
    if (ra < rb) return 1;
    int da = msg_dst(g_sort_model, a), db = msg_dst(g_sort_model, b);
    if (da != db) return da < db ? -1 : 1;
    int sa = msg_src(g_sort_model, a), sb = msg_src(g_sort_model, b);
    if (sa != sb) return sa < sb ? -1 : 1;
    return 0;
}

/*
 * Alg. 1 with one of three frontier rules.
 *
 *   schedule  OR_LBP : every message (Sec. II-B, Sec. III-A)
 *             OR_RBP : the k = max(1, ceil(p * E)) largest residuals (Sec. III-A)
 *             OR_RNBP: residual > eps, then each survivor kept with
 *                      probability p_t (Sec. IV-A)
 *   p_t       dynamic_p: p_t = low_p (= p) when n_t / n_{t-1} > ratio_threshold,
 *             else high_p; the first iteration with no n_{t-1} uses high_p.
 *             static: p_t = p.
 *   init_msgs canonical [E][K] start state or NULL for uniform 1/K (Sec. II-A).
 *   t0        global iteration number of the first evaluation (RNG counter).
 *   prev_active n_{t0-1}, or -1 if none.
 *   max_iters maximum number of commits; the state after the last commit is
 *             evaluated once more so convergence within max_iters is seen.
 *   trace_*   optional per-evaluation records, length max_iters + 1:
 *             n_t, |F_t| (0 on the converged/final evaluation), p_t, R_t.
 * Returns 0 if converged, 1 if not, negative on bad input.
 */
int oracle_bp_run_v(int N, int K, int64_t M, const int32_t* edges, const int32_t* var_states,
                    const double* log_unary, int pair_kind, const double* coupling,
                    const double* shared, const double* edge_scale, const double* pair,
                    int schedule, double eps, double p, double high_p, double ratio_threshold,
                    int dynamic_p, uint64_t seed, int64_t max_iters, const double* init_msgs,
                    int64_t t0, int64_t prev_active, double* out_msgs, double* out_marginals,
                    oracle_stats* stats, int64_t* trace_active, int64_t* trace_frontier,
                    double* trace_p, double* trace_maxres) {
    if (N < 0 || K < 2 || M < 0 || max_iters < 0) return -1;
    if (pair_kind == OR_PAIR_ISING && K != 2) return -1;
    model_t g;
    int brc = build_model(&g, N, K, M, edges, var_states, log_unary, pair_kind, coupling,
                          shared, edge_scale, pair);
    if (brc != 0) {
        free_model(&g);
        return brc;
    }
    const int64_t E = g.E;
    const int64_t EK = g.moff[E];  /* message entries */
    size_t msz = sizeof(double) * (size_t)EK + 1;
    double* m = (double*)malloc(msz);       /* m^t */
    double* cand = (double*)malloc(msz);    /* f_BP(m^t) */
    double* res = (double*)malloc(sizeof(double) * (size_t)E + 1);
    unsigned char* sel = (unsigned char*)malloc((size_t)E + 1);
    int64_t* order = (int64_t*)malloc(sizeof(int64_t) * (size_t)E + 1);
    double* work = (double*)malloc(sizeof(double) * (size_t)K);
    xprod* pw = (xprod*)malloc(sizeof(xprod) * (size_t)K);
    if (!m || !cand || !res || !sel || !order || !work || !pw) {
        free(m); free(cand); free(res); free(sel); free(order); free(work); free(pw);
        free_model(&g);
        return -2;
    }
    if (init_msgs)
        memcpy(m, init_msgs, sizeof(double) * (size_t)EK);
    else
        uniform_messages(&g, m);

    oracle_stats st;
    memset(&st, 0, sizeof(st));
    st.last_prev_active = prev_active;
    int64_t n_prev = prev_active;
    int converged = 0;
    for (int64_t it = 0;; ++it) {
        int64_t t = t0 + it;
        /* f_BP(m^t) and the residual of Eq. (4), L-infinity norm */
        if (evaluate_all(&g, m, cand, res) != 0) {
            free(m); free(cand); free(res); free(sel); free(order); free(work); free(pw);
            free_model(&g);
            return -2;
        }
        int64_t n_t = 0;
        double r_max = 0.0;
        for (int64_t e = 0; e < E; ++e) {
            if (res[e] > eps) ++n_t;
            if (res[e] > r_max) r_max = res[e];
        }
        st.evaluated += E;
        st.last_active = n_t;
        st.last_max_residual = r_max;
        st.final_t = t;
        st.last_prev_active = n_prev;
        /* p_t from EdgeRatio = n_t / n_{t-1} (Sec. IV-A) */
        double p_t = p;
        if (schedule == OR_RNBP && dynamic_p) {
            if (n_prev > 0 && (double)n_t / (double)n_prev > ratio_threshold)
                p_t = p;
            else
                p_t = high_p;
        }
        if (trace_active) trace_active[it] = n_t;
        if (trace_p) trace_p[it] = p_t;
        if (trace_maxres) trace_maxres[it] = r_max;
        if (trace_frontier) trace_frontier[it] = 0;
        if (n_t == 0) { /* IsConverged */
            converged = 1;
            break;
        }
        if (it == max_iters) break;

        /* GenerateFrontier */
        int64_t nsel = 0;
        memset(sel, 0, (size_t)E);
        if (schedule == OR_LBP) {
            memset(sel, 1, (size_t)E);
            nsel = E;
        } else if (schedule == OR_RNBP) {
            for (int64_t e = 0; e < E; ++e) {
                if (!(res[e] > eps)) continue;
                double u = oracle_uniform(seed, (uint32_t)msg_src(&g, e),
                                          (uint32_t)g.rank[e], (uint32_t)t);
                if (u < p_t) {
                    sel[e] = 1;
                    ++nsel;
                }
            }
        } else { /* OR_RBP */
            int64_t k = (int64_t)ceil(p * (double)E);
            if (k < 1) k = 1;
            if (k > E) k = E;
            for (int64_t e = 0; e < E; ++e) order[e] = e;
            g_sort_model = &g;
            g_sort_res = res;
            qsort(order, (size_t)E, sizeof(int64_t), cmp_topk);
            for (int64_t q = 0; q < k; ++q) sel[order[q]] = 1;
            nsel = k;
        }
        /* Update: synchronous commit, every candidate was computed from m^t */
        for (int64_t e = 0; e < E; ++e)
            if (sel[e]) commit_message(&g, m, cand, e);
        st.committed += nsel;
        st.iterations += 1;
        if (trace_frontier) trace_frontier[it] = nsel;
        n_prev = n_t;
    }
    st.converged = converged;
    if (out_msgs) memcpy(out_msgs, m, sizeof(double) * (size_t)EK);
    brc = out_marginals ? beliefs(&g, m, out_marginals) : 0;
    if (stats) *stats = st;
    free(m); free(cand); free(res); free(sel); free(order); free(work); free(pw);
    if (brc != 0) {
        free_model(&g);
        return brc;
    }
    free_model(&g);
    return converged ? 0 : 1;
}

/* One evaluation of f_BP and Eq. (4) for a given message set, nothing
 * committed: the candidates [E][K] and residuals [E] in canonical order. */
int oracle_bp_evaluate_v(int N, int K, int64_t M, const int32_t* edges,
                         const int32_t* var_states, const double* log_unary, int pair_kind,
                         const double* coupling, const double* shared,
                         const double* edge_scale, const double* pair, const double* msgs,
                         double* out_cand, double* out_res) {
    if (N < 0 || K < 2 || M < 0) return -1;
    model_t g;
    int brc = build_model(&g, N, K, M, edges, var_states, log_unary, pair_kind, coupling,
                          shared, edge_scale, pair);
    if (brc != 0) {
        free_model(&g);
        return brc;
    }
    double* work = (double*)malloc(sizeof(double) * (size_t)K);
    xprod* pw = (xprod*)malloc(sizeof(xprod) * (size_t)K);
    if (!work || !pw) {
        free(work); free(pw);
        free_model(&g);
        return -2;
    }
    for (int64_t e = 0; e < g.E; ++e) {
        eval_message(&g, msgs, e, out_cand + g.moff[e], work, pw);
        double r = 0.0;
        for (int64_t q = g.moff[e]; q < g.moff[e + 1]; ++q) {
            double d = fabs(out_cand[q] - msgs[q]);
            if (d > r) r = d;
        }
        out_res[e] = r;
    }
    free(work);
    free(pw);
    free_model(&g);
    return 0;
}

/* Eq. (3) for a given message set. */
int oracle_bp_beliefs_v(int N, int K, int64_t M, const int32_t* edges,
                        const int32_t* var_states, const double* log_unary, const double* msgs,
                        double* out_marginals) {
    if (N < 0 || K < 2 || M < 0) return -1;
    model_t g;
    /* the pairwise potentials do not enter Eq. (3) */
    int brc = build_model(&g, N, K, M, edges, var_states, log_unary, OR_PAIR_DENSE, NULL, NULL,
                          NULL, NULL);
    if (brc != 0) {
        free_model(&g);
        return brc;
    }
    int rc = beliefs(&g, msgs, out_marginals);
    free_model(&g);
    return rc;
}

/* The same entry points with K states for every variable. */
int oracle_bp_run(int N, int K, int64_t M, const int32_t* edges, const double* log_unary,
                  int pair_kind, const double* coupling, const double* shared,
                  const double* edge_scale, const double* pair, int schedule, double eps,
                  double p, double high_p, double ratio_threshold, int dynamic_p,
                  uint64_t seed, int64_t max_iters, const double* init_msgs, int64_t t0,
                  int64_t prev_active, double* out_msgs, double* out_marginals,
                  oracle_stats* stats, int64_t* trace_active, int64_t* trace_frontier,
                  double* trace_p, double* trace_maxres) {
    return oracle_bp_run_v(N, K, M, edges, NULL, log_unary, pair_kind, coupling, shared,
                           edge_scale, pair, schedule, eps, p, high_p, ratio_threshold, dynamic_p,
                           seed, max_iters, init_msgs, t0, prev_active, out_msgs, out_marginals,
                           stats, trace_active, trace_frontier, trace_p, trace_maxres);
}

int oracle_bp_evaluate(int N, int K, int64_t M, const int32_t* edges,
                       const double* log_unary, int pair_kind, const double* coupling,
                       const double* shared, const double* edge_scale, const double* pair,
                       const double* msgs, double* out_cand, double* out_res) {
    return oracle_bp_evaluate_v(N, K, M, edges, NULL, log_unary, pair_kind, coupling, shared,
                                edge_scale, pair, msgs, out_cand, out_res);
}

int oracle_bp_beliefs(int N, int K, int64_t M, const int32_t* edges, const double* log_unary,
                      const double* msgs, double* out_marginals) {
    return oracle_bp_beliefs_v(N, K, M, edges, NULL, log_unary, msgs, out_marginals);
}

/*
 * Serial residual BP (Sec. II-B; the paper's serial CPU baseline, Sec. III-B):
 * one message at a time, always the one with the largest residual, using the
 * newest messages.  Written plainly: after every commit every message is
 * evaluated again and the largest residual found by a scan.  Ties are taken
 * in (target, source) ascending order, as for the greedy frontier.
 *   max_updates  cap on commits; converged when the largest residual <= eps
 *   trace        optional, length max_updates: the message id of each commit
 * Returns 0 if converged, 1 if not, negative on bad input.
 */
int oracle_srbp_run(int N, int K, int64_t M, const int32_t* edges, const double* log_unary,
                    int pair_kind, const double* coupling, const double* shared,
                    const double* edge_scale, const double* pair, double eps,
                    int64_t max_updates, double* out_msgs, double* out_marginals,
                    int64_t* out_updates, int64_t* trace) {
    if (N < 0 || K < 2 || M < 0 || max_updates < 0) return -1;
    if (pair_kind == OR_PAIR_ISING && K != 2) return -1;
    model_t g;
    if (build_model(&g, N, K, M, edges, NULL, log_unary, pair_kind, coupling, shared, edge_scale,
                    pair) != 0) {
        free_model(&g);
        return -2;
    }
    const int64_t E = g.E;
    size_t msz = sizeof(double) * (size_t)g.moff[E] + 1;
    double* m = (double*)malloc(msz);
    double* cand = (double*)malloc(msz);
    double* res = (double*)malloc(sizeof(double) * (size_t)E + 1);
    if (!m || !cand || !res) {
        free(m); free(cand); free(res);
        free_model(&g);
        return -2;
    }
    uniform_messages(&g, m);
    int converged = 0;
    int64_t updates = 0;
    int rc = 0;
    for (;;) {
        if (evaluate_all(&g, m, cand, res) != 0) {
            rc = -2;
            break;
        }
        /* the message with the largest residual, ties by (target, source) */
        int64_t best = -1;
        for (int64_t e = 0; e < E; ++e) {
            if (best < 0 || res[e] > res[best]) {
                best = e;
                continue;
            }
            if (res[e] < res[best]) continue;
            int de = msg_dst(&g, e), db = msg_dst(&g, best);
            if (de < db || (de == db && msg_src(&g, e) < msg_src(&g, best))) best = e;
        }
        if (best < 0 || !(res[best] > eps)) {
            converged = 1;
            break;
        }
        if (updates == max_updates) break;
        commit_message(&g, m, cand, best);
        if (trace) trace[updates] = best;
        ++updates;
    }
    if (rc == 0) {
        if (out_msgs) memcpy(out_msgs, m, sizeof(double) * (size_t)g.moff[E]);
        if (out_marginals) rc = beliefs(&g, m, out_marginals);
        if (out_updates) *out_updates = updates;
    }
    free(m); free(cand); free(res);
    free_model(&g);
    if (rc != 0) return rc;
    return converged ? 0 : 1;
}

/*
 * Residual splash in frontier form (Sec. II-B, Sec. III-A): per iteration,
 * evaluate f_BP(m^t) for every message (IsConverged as for the other rules);
 * the residual of a vertex is the largest residual of its incoming messages;
 * the k = min(N, max(1, ceil(p * E))) vertices of largest residual (ties by id
 * ascending) are the roots; a splash of depth h around a root visits its BFS
 * tree, so level L_d holds every vertex at graph distance exactly d from some
 * root (d = 0..h).  The updates move through the levels h, h-1, ..., 1, 0, 1,
 * ..., h: at each level every message out of every vertex of the level is
 * recomputed by Eq. (2) from the messages as they stand when that level
 * starts, and committed.
 *   trace_*  optional, length max_iters + 1: n_t, messages committed, R_t.
 * Returns 0 if converged, 1 if not, negative on bad input.
 */
int oracle_rs_run(int N, int K, int64_t M, const int32_t* edges, const double* log_unary,
                  int pair_kind, const double* coupling, const double* shared,
                  const double* edge_scale, const double* pair, double eps, double p,
                  int splash_depth, int64_t max_iters, const double* init_msgs,
                  double* out_msgs, double* out_marginals, oracle_stats* stats,
                  int64_t* trace_active, int64_t* trace_committed, double* trace_maxres) {
    if (N < 0 || K < 2 || M < 0 || max_iters < 0 || splash_depth < 0) return -1;
    if (pair_kind == OR_PAIR_ISING && K != 2) return -1;
    if (!(p > 0.0 && p <= 1.0)) return -1;
    model_t g;
    if (build_model(&g, N, K, M, edges, NULL, log_unary, pair_kind, coupling, shared, edge_scale,
                    pair) != 0) {
        free_model(&g);
        return -2;
    }
    const int64_t E = g.E;
    const int h = splash_depth;
    size_t msz = sizeof(double) * (size_t)g.moff[E] + 1;
    double* m = (double*)malloc(msz);
    double* cand = (double*)malloc(msz);
    double* res = (double*)malloc(sizeof(double) * (size_t)E + 1);
    double* vres = (double*)malloc(sizeof(double) * (size_t)N + 1);
    int32_t* order = (int32_t*)malloc(sizeof(int32_t) * (size_t)N + 1);
    int32_t* dist = (int32_t*)malloc(sizeof(int32_t) * (size_t)N + 1);
    int32_t* queue = (int32_t*)malloc(sizeof(int32_t) * (size_t)N + 1);
    unsigned char* level = (unsigned char*)malloc((size_t)(h + 1) * (size_t)N + 1);
    double* work = (double*)malloc(sizeof(double) * (size_t)K);
    xprod* pw = (xprod*)malloc(sizeof(xprod) * (size_t)K);
    int rc = 0;
    if (!m || !cand || !res || !vres || !order || !dist || !queue || !level || !work || !pw)
        rc = -2;
    if (rc == 0) {
        if (init_msgs)
            memcpy(m, init_msgs, sizeof(double) * (size_t)g.moff[E]);
        else
            uniform_messages(&g, m);
    }
    oracle_stats st;
    memset(&st, 0, sizeof(st));
    st.last_prev_active = -1;
    int converged = 0;
    int64_t k = (int64_t)ceil(p * (double)E);
    if (k < 1) k = 1;
    if (k > N) k = N;
    for (int64_t it = 0; rc == 0; ++it) {
        if (evaluate_all(&g, m, cand, res) != 0) {
            rc = -2;
            break;
        }
        int64_t n_t = 0;
        double r_max = 0.0;
        for (int64_t e = 0; e < E; ++e) {
            if (res[e] > eps) ++n_t;
            if (res[e] > r_max) r_max = res[e];
        }
        st.evaluated += E;
        st.last_active = n_t;
        st.last_max_residual = r_max;
        st.final_t = it;
        if (trace_active) trace_active[it] = n_t;
        if (trace_maxres) trace_maxres[it] = r_max;
        if (trace_committed) trace_committed[it] = 0;
        if (n_t == 0) {
            converged = 1;
            break;
        }
        if (it == max_iters) break;

        /* vertex residuals and the k roots (largest first, ties by id):
         * a selection by repeated scans, O(k N) */
        for (int v = 0; v < N; ++v) {
            vres[v] = 0.0;
            for (int64_t q = g.in_ptr[v]; q < g.in_ptr[v + 1]; ++q)
                if (res[g.in_ids[q]] > vres[v]) vres[v] = res[g.in_ids[q]];
        }
        memset(level, 0, (size_t)(h + 1) * (size_t)N);
        for (int v = 0; v < N; ++v) order[v] = 0; /* 1 once chosen */
        for (int64_t c = 0; c < k; ++c) {
            int best = -1;
            for (int v = 0; v < N; ++v)
                if (!order[v] && (best < 0 || vres[v] > vres[best])) best = v;
            order[best] = 1;
            level[best] = 1; /* level 0 */
        }
        /* BFS of depth h from every root: level d gets every vertex at
         * distance exactly d from that root */
        for (int r = 0; r < N && h > 0; ++r) {
            if (!level[r]) continue;
            for (int v = 0; v < N; ++v) dist[v] = -1;
            int head = 0, tail = 0;
            dist[r] = 0;
            queue[tail++] = r;
            while (head < tail) {
                int u = queue[head++];
                if (dist[u] == h) continue;
                for (int64_t q = g.in_ptr[u]; q < g.in_ptr[u + 1]; ++q) {
                    int w = msg_src(&g, g.in_ids[q]); /* a neighbour of u */
                    if (dist[w] >= 0) continue;
                    dist[w] = dist[u] + 1;
                    level[(size_t)dist[w] * N + w] = 1;
                    queue[tail++] = w;
                }
            }
        }
        /* the splash updates: levels h, ..., 1, 0, 1, ..., h */
        int64_t committed = 0;
        for (int s = 0; s <= 2 * h; ++s) {
            int d = s <= h ? h - s : s - h;
            const unsigned char* L = level + (size_t)d * N;
            for (int64_t e = 0; e < E; ++e)
                if (L[msg_src(&g, e)]) eval_message(&g, m, e, cand + g.moff[e], work, pw);
            for (int64_t e = 0; e < E; ++e)
                if (L[msg_src(&g, e)]) {
                    commit_message(&g, m, cand, e);
                    ++committed;
                }
        }
        st.evaluated += committed;
        st.committed += committed;
        st.iterations += 1;
        if (trace_committed) trace_committed[it] = committed;
    }
    st.converged = converged;
    if (rc == 0) {
        if (out_msgs) memcpy(out_msgs, m, sizeof(double) * (size_t)g.moff[E]);
        if (out_marginals) rc = beliefs(&g, m, out_marginals);
        if (stats) *stats = st;
    }
    free(m); free(cand); free(res); free(vres); free(order); free(dist); free(queue);
    free(level); free(work); free(pw);
    free_model(&g);
    if (rc != 0) return rc;
    return converged ? 0 : 1;
}
