// Serial residual belief propagation on the host CPU (include/srbp.h): the
// paper's serial baseline (Sec. II-B, Sec. III-B).  One message at a time, the
// largest residual first, from the newest messages; an indexed binary max-heap
// over all messages keyed by (residual, then (target, source) ascending) gives
// the next message, and a commit recomputes only the messages that read it.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <unordered_set>
#include <vector>

#include "../../include/srbp.h"

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

bool finite_all(const double* p, size_t n) {
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(p[i])) return false;
    return true;
}
bool positive_all(const double* p, size_t n) {
    for (size_t i = 0; i < n; ++i)
        if (!(p[i] > 0.0) || !std::isfinite(p[i])) return false;
    return true;
}

// Canonical message e of undirected edge u = e / 2: e even is edges[u][0] ->
// edges[u][1], e odd the reverse.
struct Model {
    int N = 0, K = 0;
    long long M = 0, E = 0;
    int kind = 0;
    std::vector<int> src, dst;        // [E]
    std::vector<long long> in_ptr;    // [N+1] incoming messages of each node
    std::vector<int> in_ids;          // [E] grouped by target, in message-id order
    std::vector<long long> out_ptr;   // [N+1] outgoing messages of each node
    std::vector<int> out_ids;         // [E]
    std::vector<double> unary;        // [N][K] psi_i = exp(log_unary)
    std::vector<double> ising;        // [M][2]: exp(J), exp(-J)
    const double* shared = nullptr;   // [K][K]
    const double* scale = nullptr;    // [M]
    const double* pair = nullptr;     // [M][K][K]

    // psi of undirected edge u at (state of edges[u][0], state of edges[u][1])
    double psi_edge(long long u, int xa, int xb) const {
        if (kind == BP_PAIR_ISING) return (xa == xb) ? ising[2 * u] : ising[2 * u + 1];
        if (kind == BP_PAIR_SHARED) return scale[u] * shared[xa * K + xb];
        return pair[(u * K + xa) * K + xb];
    }
    // psi_{ij}(x_i, x_j) for message e = i -> j
    double psi_msg(long long e, int xi, int xj) const {
        const long long u = e >> 1;
        return (e & 1) ? psi_edge(u, xj, xi) : psi_edge(u, xi, xj);
    }
};

int build(const bp_graph_desc* d, Model& g) {
    if (!d) return fail(BP_EINVAL, "desc is NULL");
    if (d->var_states) return fail(BP_EINVAL, "per-variable state counts are not supported");
    const long long N = d->num_vars, K = d->num_states, M = d->num_edges;
    if (N < 1 || N > 0x7FFFFFFELL) return fail(BP_EINVAL, "num_vars %lld out of range", N);
    if (K < 2 || K > 64) return fail(BP_EINVAL, "num_states %lld not in [2, 64]", K);
    if (M < 0 || 2 * M > 0x7FFFFFFELL) return fail(BP_EINVAL, "num_edges %lld out of range", M);
    if (M > 0 && !d->edges) return fail(BP_EINVAL, "edges is NULL");
    if (!d->log_unary || !finite_all(d->log_unary, (size_t)(N * K)))
        return fail(BP_EINVAL, "log_unary missing or not finite");
    g.kind = d->pair_kind;
    if (g.kind == BP_PAIR_ISING) {
        if (K != 2) return fail(BP_EINVAL, "BP_PAIR_ISING needs num_states == 2");
        if (M > 0 && (!d->coupling || !finite_all(d->coupling, (size_t)M)))
            return fail(BP_EINVAL, "coupling missing or not finite");
    } else if (g.kind == BP_PAIR_SHARED) {
        if (!d->shared || !positive_all(d->shared, (size_t)(K * K)))
            return fail(BP_EINVAL, "shared potential must be positive and finite");
        if (M > 0 && (!d->edge_scale || !positive_all(d->edge_scale, (size_t)M)))
            return fail(BP_EINVAL, "edge_scale must be positive and finite");
    } else if (g.kind == BP_PAIR_DENSE) {
        if (M > 0 && (!d->pair || !positive_all(d->pair, (size_t)(M * K * K))))
            return fail(BP_EINVAL, "pair potential must be positive and finite");
    } else {
        return fail(BP_EINVAL, "unknown pair_kind %d", g.kind);
    }
    std::unordered_set<unsigned long long> seen;
    seen.reserve((size_t)M * 2 + 1);
    for (long long u = 0; u < M; ++u) {
        const long long a = d->edges[2 * u], b = d->edges[2 * u + 1];
        if (a < 0 || a >= N || b < 0 || b >= N)
            return fail(BP_EINVAL, "edge %lld out of range", u);
        if (a == b) return fail(BP_EINVAL, "edge %lld is a self-loop", u);
        const unsigned long long key = (unsigned long long)std::min(a, b) * N + std::max(a, b);
        if (!seen.insert(key).second) return fail(BP_EINVAL, "edge %lld duplicates an earlier edge", u);
    }
    g.N = (int)N;
    g.K = (int)K;
    g.M = M;
    g.E = 2 * M;
    g.src.resize((size_t)g.E);
    g.dst.resize((size_t)g.E);
    for (long long e = 0; e < g.E; ++e) {
        const long long u = e >> 1;
        g.src[e] = d->edges[2 * u + (e & 1)];
        g.dst[e] = d->edges[2 * u + 1 - (e & 1)];
    }
    auto group = [&](const std::vector<int>& key, std::vector<long long>& ptr, std::vector<int>& ids) {
        ptr.assign((size_t)N + 1, 0);
        for (long long e = 0; e < g.E; ++e) ptr[key[e] + 1]++;
        for (long long i = 0; i < N; ++i) ptr[i + 1] += ptr[i];
        ids.resize((size_t)g.E);
        std::vector<long long> fill(ptr.begin(), ptr.end() - 1);
        for (long long e = 0; e < g.E; ++e) ids[fill[key[e]]++] = (int)e;
    };
    group(g.dst, g.in_ptr, g.in_ids);
    group(g.src, g.out_ptr, g.out_ids);
    g.unary.resize((size_t)(N * K));
    for (long long i = 0; i < N * K; ++i) g.unary[i] = std::exp(d->log_unary[i]);
    if (g.kind == BP_PAIR_ISING) {
        g.ising.resize((size_t)(2 * M));
        for (long long u = 0; u < M; ++u) {
            g.ising[2 * u] = std::exp(d->coupling[u]);
            g.ising[2 * u + 1] = std::exp(-d->coupling[u]);
        }
    }
    g.shared = d->shared;
    g.scale = d->edge_scale;
    g.pair = d->pair;
    return BP_OK;
}

// A product kept within the double range: when its largest entry falls below
// 2^-600 the vector is scaled by 2^600 (exact), so a node with any number of
// neighbours neither underflows nor changes the rounding of later factors.
inline void rescale(double* v, int K) {
    double mx = 0.0;
    for (int x = 0; x < K; ++x) mx = std::max(mx, v[x]);
    if (mx < 0x1p-600)
        for (int x = 0; x < K; ++x) v[x] = std::ldexp(v[x], 600);
}

struct Solver {
    const Model& g;
    std::vector<double> m, cand, res;   // [E][K], [E][K], [E]
    std::vector<double> prod;           // [K]
    // indexed binary max-heap of message ids
    std::vector<int> heap;
    std::vector<int> pos;
    long long evals = 0;

    explicit Solver(const Model& model) : g(model) {}

    // Eq. (2) for e = i -> j from the current messages:
    // c(x_j) = sum_{x_i} psi(x_i, x_j) psi_i(x_i) prod_{k in Gamma_i \ j} m_{k->i}(x_i),
    // normalised; then the residual against m_e.
    void evaluate(int e) {
        const int K = g.K;
        const int i = g.src[e];
        const int back = e ^ 1;
        double* p = prod.data();
        for (int x = 0; x < K; ++x) p[x] = g.unary[(size_t)i * K + x];
        for (long long q = g.in_ptr[i]; q < g.in_ptr[i + 1]; ++q) {
            const int f = g.in_ids[q];
            if (f == back) continue;
            const double* mf = &m[(size_t)f * K];
            for (int x = 0; x < K; ++x) p[x] *= mf[x];
            rescale(p, K);
        }
        double* c = &cand[(size_t)e * K];
        double z = 0.0;
        for (int y = 0; y < K; ++y) {
            double s = 0.0;
            for (int x = 0; x < K; ++x) s += g.psi_msg(e, x, y) * p[x];
            c[y] = s;
            z += s;
        }
        double r = 0.0;
        const double* me = &m[(size_t)e * K];
        for (int y = 0; y < K; ++y) {
            c[y] /= z;
            r = std::max(r, std::fabs(c[y] - me[y]));
        }
        res[e] = r;
        ++evals;
    }

    // heap order: larger residual first, then smaller (target, source)
    bool before(int a, int b) const {
        if (res[a] != res[b]) return res[a] > res[b];
        if (g.dst[a] != g.dst[b]) return g.dst[a] < g.dst[b];
        return g.src[a] < g.src[b];
    }
    void place(size_t k, int e) {
        heap[k] = e;
        pos[e] = (int)k;
    }
    void sift_up(size_t k) {
        const int e = heap[k];
        while (k > 0) {
            const size_t parent = (k - 1) / 2;
            if (!before(e, heap[parent])) break;
            place(k, heap[parent]);
            k = parent;
        }
        place(k, e);
    }
    void sift_down(size_t k) {
        const int e = heap[k];
        const size_t n = heap.size();
        for (;;) {
            size_t best = k;
            int be = e;
            const size_t l = 2 * k + 1, r = l + 1;
            if (l < n && before(heap[l], be)) {
                best = l;
                be = heap[l];
            }
            if (r < n && before(heap[r], be)) best = r;
            if (best == k) break;
            place(k, heap[best]);
            k = best;
        }
        place(k, e);
    }
    void reorder(int e) {
        const size_t k = (size_t)pos[e];
        sift_up(k);
        sift_down((size_t)pos[e]);
    }
};

}  // namespace

extern "C" {

const char* srbp_last_error(void) { return g_err.c_str(); }

int srbp_solve(const bp_graph_desc* desc, double eps, int64_t max_updates, double time_limit_s,
               double* out_marginals, double* out_msgs, int64_t* trace, int64_t trace_len,
               srbp_stats* stats) {
    if (!(eps >= 0.0) || !std::isfinite(eps)) return fail(BP_EINVAL, "eps must be finite and >= 0");
    if (max_updates < 0) return fail(BP_EINVAL, "max_updates < 0");
    if (trace_len < 0 || (trace_len > 0 && !trace)) return fail(BP_EINVAL, "bad trace buffer");
    try {
        Model g;
        int rc = build(desc, g);
        if (rc != BP_OK) return rc;
        const int K = g.K;
        const long long E = g.E;
        Solver s(g);
        s.m.assign((size_t)(E * K), 1.0 / K);
        s.cand.assign((size_t)(E * K), 0.0);
        s.res.assign((size_t)E, 0.0);
        s.prod.assign((size_t)K, 0.0);
        const auto t0 = std::chrono::steady_clock::now();
        for (long long e = 0; e < E; ++e) s.evaluate((int)e);
        s.heap.resize((size_t)E);
        s.pos.resize((size_t)E);
        for (long long e = 0; e < E; ++e) s.place((size_t)e, (int)e);
        for (long long k = E / 2 - 1; k >= 0; --k) s.sift_down((size_t)k);

        long long updates = 0;
        bool converged = false, timed_out = false;
        for (;;) {
            const int top = E > 0 ? s.heap[0] : -1;
            if (top < 0 || !(s.res[top] > eps)) {
                converged = true;
                break;
            }
            if (updates == max_updates) break;
            if ((updates & 1023) == 0 && time_limit_s > 0.0 && updates > 0) {
                const double el = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
                if (el >= time_limit_s) {
                    timed_out = true;
                    break;
                }
            }
            // commit the top message: its residual becomes 0 (its candidate does
            // not read it), and the messages out of its target except the
            // reverse one read it
            std::memcpy(&s.m[(size_t)top * K], &s.cand[(size_t)top * K], sizeof(double) * K);
            if (trace && updates < trace_len) trace[updates] = top;
            ++updates;
            s.res[top] = 0.0;
            s.reorder(top);
            const int j = g.dst[top];
            const int back = top ^ 1;
            for (long long q = g.out_ptr[j]; q < g.out_ptr[j + 1]; ++q) {
                const int f = g.out_ids[q];
                if (f == back) continue;
                s.evaluate(f);
                s.reorder(f);
            }
        }
        const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        if (out_msgs) std::memcpy(out_msgs, s.m.data(), sizeof(double) * (size_t)(E * K));
        if (out_marginals) {
            // Eq. (3): b_i(x) proportional to psi_i(x) prod_{k in Gamma_i} m_{k->i}(x)
            std::vector<double> b((size_t)K);
            for (int i = 0; i < g.N; ++i) {
                for (int x = 0; x < K; ++x) b[x] = g.unary[(size_t)i * K + x];
                for (long long q = g.in_ptr[i]; q < g.in_ptr[i + 1]; ++q) {
                    const double* mf = &s.m[(size_t)g.in_ids[q] * K];
                    for (int x = 0; x < K; ++x) b[x] *= mf[x];
                    rescale(b.data(), K);
                }
                double z = 0.0;
                for (int x = 0; x < K; ++x) z += b[x];
                for (int x = 0; x < K; ++x) out_marginals[(size_t)i * K + x] = b[x] / z;
            }
        }
        if (stats) {
            std::memset(stats, 0, sizeof(*stats));
            stats->updates = updates;
            stats->converged = converged ? 1 : 0;
            stats->timed_out = timed_out ? 1 : 0;
            stats->max_residual = E > 0 ? s.res[s.heap[0]] : 0.0;
            stats->seconds = secs;
            stats->evaluations = s.evals;
        }
        return converged ? BP_OK : BP_NOT_CONVERGED;
    } catch (const std::bad_alloc&) {
        return fail(BP_ENOMEM, "host allocation failed");
    }
}

}  // extern "C"
