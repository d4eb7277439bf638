// C ABI of libbp (include/bp.h): validation, device layout, and the host side of
// the Alg. 1 loop.  The loop itself runs on the device: each iteration is a
// fixed sequence of kernel launches whose convergence test and EdgeRatio rule
// read device counters, so the host only enqueues work and polls a flag every
// check_every iterations.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <numeric>
#include <string>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "../../include/bp.h"
#include "bp_internal.h"

using namespace bp;

namespace {

thread_local std::string g_last_error;

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

int hip_fail(hipError_t e, const char* what) {
    return fail(BP_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_OK(expr, what)                                  \
    do {                                                    \
        hipError_t _e = (expr);                             \
        if (_e != hipSuccess) return hip_fail(_e, what);    \
    } while (0)

int kpad(int K) {
    int p = 2;
    while (p < K) p <<= 1;
    return p;
}

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

// Host-side description of the device layout, built once per graph.
struct HostLayout {
    int N = 0, K = 0, layout = 0, pair = 0, row = 1;
    long long M = 0, E = 0;
    std::vector<int> node_ptr;        // [N+1] slot range of each source node
    std::vector<int> rev;             // [E]
    std::vector<short> rev16;         // [E] rev[e] - e (K = 2 log-odds layout, when all fit)
    std::vector<int> slot_of_canon;   // [E]
    std::vector<int> tile_start;      // [T+1]
    std::vector<int> tile_slot;       // [T+1] node_ptr[tile_start]
    int tile_nodes_max = 1;           // most nodes in one regular tile
    int tile_big = 0;                 // 1 if some node's slots exceed the tile limit
    int no_mfma = 0;                  // BP_FLAG_NO_MATRIX_CORES
    int mfma_bf16 = 0;                // BP_FLAG_BF16_MATRIX_CORES
    int sparse_reserved = 0;          // BP_FLAG_SPARSE_BUFFERS on a log-odds graph
    int splash_reserved = 0;          // BP_FLAG_SPLASH_BUFFERS on a log-odds graph
    std::vector<int> tiles4;          // log-odds layout: regular tiles {n0, n1, s0, s1}
    std::vector<int> big4;            // log-odds layout: single-node tiles over the slot limit
    std::vector<float> coupling;      // [E] (Ising)
    std::vector<float> unary;         // [N] log-odds or [N][K] log psi (max-shifted)
    std::vector<float> pair_tab;      // shared (2KK) or dense [E][K][K]
    std::vector<unsigned char> orient;// [E] (asymmetric shared)
    // per-variable state counts (ragged layout)
    std::vector<int> kv;              // [N] K_i
    std::vector<int> uoff;            // [N+1] unary / belief row of each variable
    std::vector<int> moff;            // [E+1] message row of each slot (K_target entries)
    std::vector<int> toff;            // [E+1] table of each slot (K_source x K_target)
    std::vector<int> heavy;           // {slot, source} of the slots of heavy variables
    std::vector<long long> coff;      // [E+1] row of each canonical message in host arrays
    long long msg_floats = 0;         // entries of one message buffer
    long long belief_floats = 0;      // entries of the beliefs (N K, or sum K_i)
};

struct Arena {
    size_t off = 0;
    size_t take(size_t bytes) {
        size_t o = off;
        off += (bytes + 255) & ~size_t(255);
        return o;
    }
};

struct Offsets {
    size_t node_ptr, rev, tile, tile_slot, tiles4, big4, coupling, unary, pair, orient, msg[4], cand, keys, ties, state,
        ctr, marg, kv, uoff, moff, toff, heavy, rev16, sparse, splash, total;
};

// Device bytes of the sparse re-evaluation buffers of a log-odds graph: dirty
// and active-node flags u8 [N] each (256-byte rounded), target node i32 [E].
size_t sparse_bytes(const HostLayout& L) {
    const size_t nb = ((size_t)L.N + 255) / 256 * 256;
    return 2 * nb + sizeof(int) * (size_t)L.E + 256;
}

Offsets plan(const HostLayout& L) {
    Arena a;
    Offsets o;
    const size_t E = (size_t)L.E;
    o.node_ptr = a.take(sizeof(int) * (L.N + 1));
    o.rev = a.take(sizeof(int) * L.rev.size());
    o.tile = a.take(sizeof(int) * L.tile_start.size());
    o.tile_slot = a.take(sizeof(int) * L.tile_slot.size());
    o.tiles4 = a.take(sizeof(int) * L.tiles4.size());
    o.big4 = a.take(sizeof(int) * L.big4.size());
    o.coupling = a.take(sizeof(float) * L.coupling.size());
    o.unary = a.take(sizeof(float) * L.unary.size());
    o.pair = a.take(sizeof(float) * L.pair_tab.size());
    o.orient = a.take(L.orient.size());
    for (int i = 0; i < 4; ++i) o.msg[i] = a.take(sizeof(float) * (size_t)L.msg_floats);
    o.cand = a.take(sizeof(float) * (size_t)L.msg_floats);
    o.keys = a.take(sizeof(unsigned int) * E);
    // per-block tie counts of a top-k over the messages or (residual splash) the variables
    o.ties = a.take(sizeof(unsigned int) * (std::max<size_t>(E, (size_t)L.N) / 4096 + 2));
    o.state = a.take(sizeof(DevState));
    o.ctr = a.take(sizeof(CounterLine) * 4 * kCounterCopies);
    o.marg = a.take(sizeof(float) * (size_t)L.belief_floats);
    o.kv = a.take(sizeof(int) * L.kv.size());
    o.uoff = a.take(sizeof(int) * L.uoff.size());
    o.moff = a.take(sizeof(int) * L.moff.size());
    o.toff = a.take(sizeof(int) * L.toff.size());
    o.heavy = a.take(sizeof(int) * L.heavy.size());
    o.rev16 = a.take(sizeof(short) * L.rev16.size());
    o.sparse = L.sparse_reserved ? a.take(sparse_bytes(L)) : 0;
    o.splash = L.splash_reserved ? a.take(splash_bytes(L.N)) : 0;
    o.total = a.off;
    return o;
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

// Validate the problem (Eq. (1): finite state sets, positive potentials) and
// build the device layout: directed messages sorted by (source, target), the
// reverse-slot index, per-slot parameters and node tiles.
int build_layout(const bp_graph_desc* d, HostLayout& L) {
    if (!d) return fail(BP_EINVAL, "desc is NULL");
    const long long N = d->num_vars, K = d->num_states, M = d->num_edges;
    const bool ragged = d->var_states != nullptr;
    const int kmax = ragged ? kMaxKRagged : kMaxK;
    if (N < 1 || N > 0x7FFFFFFFLL - 1) return fail(BP_EINVAL, "num_vars %lld out of range", N);
    if (K < 2 || K > kmax) return fail(BP_EINVAL, "num_states %lld not in [2, %d]", K, kmax);
    if (M < 0 || 2 * M > 0x7FFFFFFFLL - 1) return fail(BP_EINVAL, "num_edges %lld out of range", M);
    if (M > 0 && !d->edges) return fail(BP_EINVAL, "edges is NULL");
    if (!d->log_unary) return fail(BP_EINVAL, "log_unary is NULL");
    long long unary_n = N * K;
    if (ragged) {
        unary_n = 0;
        for (long long i = 0; i < N; ++i) {
            const long long k = d->var_states[i];
            if (k < 2 || k > K)
                return fail(BP_EINVAL, "var_states[%lld] = %lld not in [2, num_states]", i, k);
            unary_n += k;
        }
        if (d->pair_kind != BP_PAIR_DENSE)
            return fail(BP_EINVAL, "var_states needs BP_PAIR_DENSE tables");
    }
    if (!finite_all(d->log_unary, (size_t)unary_n)) return fail(BP_EINVAL, "log_unary not finite");
    const int kind = d->pair_kind;
    if (ragged) {
        if (M > 0 && !d->pair) return fail(BP_EINVAL, "pair is NULL");
        // edges are range-checked before the table sizes are read
        for (long long u = 0; u < M; ++u) {
            const long long a = d->edges[2 * u], b = d->edges[2 * u + 1];
            if (a < 0 || a >= N || b < 0 || b >= N)
                return fail(BP_EINVAL, "edge %lld = (%lld, %lld) out of range", u, a, b);
        }
        long long pn = 0, mn = 0;
        for (long long u = 0; u < M; ++u) {
            const long long ka = d->var_states[d->edges[2 * u]], kb = d->var_states[d->edges[2 * u + 1]];
            pn += ka * kb;
            mn += ka + kb;
        }
        if (2 * pn > 0x7FFFFFFFLL - 1 || mn > 0x7FFFFFFFLL - 1 || unary_n > 0x7FFFFFFFLL - 1)
            return fail(BP_EINVAL, "ragged tables or messages exceed 2^31 entries");
        if (M > 0 && !positive_all(d->pair, (size_t)pn))
            return fail(BP_EINVAL, "pair potential must be positive and finite");
    } else if (kind == BP_PAIR_ISING) {
        if (K != 2) return fail(BP_EINVAL, "BP_PAIR_ISING needs num_states == 2");
        if (M > 0 && !d->coupling) return fail(BP_EINVAL, "coupling is NULL");
        if (M > 0 && !finite_all(d->coupling, (size_t)M)) return fail(BP_EINVAL, "coupling not finite");
    } else if (kind == BP_PAIR_SHARED) {
        if (!d->shared) return fail(BP_EINVAL, "shared is NULL");
        if (!positive_all(d->shared, (size_t)(K * K)))
            return fail(BP_EINVAL, "shared potential must be positive and finite");
        if (M > 0 && !d->edge_scale) return fail(BP_EINVAL, "edge_scale is NULL");
        if (M > 0 && !positive_all(d->edge_scale, (size_t)M))
            return fail(BP_EINVAL, "edge_scale must be positive and finite");
    } else if (kind == BP_PAIR_DENSE) {
        if (M > 0 && !d->pair) return fail(BP_EINVAL, "pair is NULL");
        if (M > 0 && !positive_all(d->pair, (size_t)(M * K * K)))
            return fail(BP_EINVAL, "pair potential must be positive and finite");
    } else {
        return fail(BP_EINVAL, "unknown pair_kind %d", kind);
    }
    if (d->flags & ~(uint32_t)(BP_FLAG_GENERIC_LAYOUT | BP_FLAG_NO_MATRIX_CORES |
                               BP_FLAG_SPARSE_BUFFERS | BP_FLAG_SPLASH_BUFFERS |
                               BP_FLAG_BF16_MATRIX_CORES))
        return fail(BP_EINVAL, "unknown flags");
    L.no_mfma = (d->flags & BP_FLAG_NO_MATRIX_CORES) ? 1 : 0;
    L.mfma_bf16 = (d->flags & BP_FLAG_BF16_MATRIX_CORES) ? 1 : 0;
    {
        std::unordered_set<unsigned long long> seen;
        seen.reserve((size_t)M * 2 + 1);
        for (long long u = 0; u < M; ++u) {
            const long long a = d->edges[2 * u], b = d->edges[2 * u + 1];
            if (a < 0 || a >= N || b < 0 || b >= N)
                return fail(BP_EINVAL, "edge %lld = (%lld, %lld) out of range", u, a, b);
            if (a == b) return fail(BP_EINVAL, "edge %lld is a self-loop", u);
            const unsigned long long key =
                (unsigned long long)std::min(a, b) * (unsigned long long)N + std::max(a, b);
            if (!seen.insert(key).second) return fail(BP_EINVAL, "edge %lld duplicates an earlier edge", u);
        }
    }

    L.N = (int)N;
    L.K = (int)K;
    L.M = M;
    L.E = 2 * M;
    // The log-odds kernel addresses its arrays with 32-bit byte offsets, so it
    // takes graphs with fewer than 2^30 messages and nodes; larger K = 2 graphs
    // use the [E][K] layout.
    const bool small = 2 * M < (1ll << 30) - kTileSlotsLogOdds && N < (1ll << 30) - kTileSlotsLogOdds;
    L.layout = ragged ? kLayoutRagged
               : (kind == BP_PAIR_ISING && !(d->flags & BP_FLAG_GENERIC_LAYOUT) && small)
                   ? kLayoutLogOdds
                   : kLayoutGeneric;
    L.row = L.layout == kLayoutLogOdds ? 1 : (int)K;  // uniform layouts: entries per slot
    L.sparse_reserved = (L.layout == kLayoutLogOdds && (d->flags & BP_FLAG_SPARSE_BUFFERS)) ? 1 : 0;
    L.splash_reserved = (L.layout == kLayoutLogOdds && (d->flags & BP_FLAG_SPLASH_BUFFERS)) ? 1 : 0;
    const long long E = L.E;
    auto csrc = [&](long long c) { return d->edges[2 * (c >> 1) + ((c & 1) ? 1 : 0)]; };
    auto cdst = [&](long long c) { return d->edges[2 * (c >> 1) + ((c & 1) ? 0 : 1)]; };

    // Counting sort of directed messages by source, then by target inside a
    // source: slot e holds m_{i->k}, the message its thread computes, so the
    // old value, the outputs and the per-slot constants are read and written
    // contiguously; the one gather is the incoming m_{k->i} at rev[e].
    L.node_ptr.assign((size_t)N + 1, 0);
    for (long long c = 0; c < E; ++c) L.node_ptr[csrc(c) + 1]++;
    for (long long i = 0; i < N; ++i) L.node_ptr[i + 1] += L.node_ptr[i];
    std::vector<int> canon_of_slot((size_t)E);
    {
        std::vector<int> fill(L.node_ptr.begin(), L.node_ptr.end() - 1);
        for (long long c = 0; c < E; ++c) canon_of_slot[fill[csrc(c)]++] = (int)c;
    }
    for (long long i = 0; i < N; ++i)
        std::sort(canon_of_slot.begin() + L.node_ptr[i], canon_of_slot.begin() + L.node_ptr[i + 1],
                  [&](int x, int y) { return cdst(x) < cdst(y); });
    L.slot_of_canon.assign((size_t)E, 0);
    for (long long s = 0; s < E; ++s) L.slot_of_canon[canon_of_slot[s]] = (int)s;
    L.rev.resize((size_t)E);
    for (long long s = 0; s < E; ++s) L.rev[s] = L.slot_of_canon[canon_of_slot[s] ^ 1];
    // the K = 2 kernel reads slot 0 of a tile without slots: keep one valid entry
    if (E == 0) L.rev.assign(1, 0);
    // K = 2 log-odds layout: the reverse slot as a 16-bit offset when every
    // one fits (grids: the reverse message is a few rows of slots away), two
    // bytes per message instead of four for the evaluation kernel
    if (L.layout == kLayoutLogOdds && E > 0) {
        bool fits = true;
        for (long long s = 0; s < E && fits; ++s) {
            const long long d = (long long)L.rev[s] - s;
            fits = d >= -32768 && d <= 32767;
        }
        if (fits) {
            L.rev16.resize((size_t)E);
            for (long long s = 0; s < E; ++s) L.rev16[s] = (short)((long long)L.rev[s] - s);
        }
    }

    L.msg_floats = E * L.row;
    L.belief_floats = N * K;
    if (ragged) {
        // per-variable rows: unary (and beliefs) by variable, messages and
        // tables by slot, host message rows by canonical id
        L.kv.assign(d->var_states, d->var_states + N);
        L.uoff.assign((size_t)N + 1, 0);
        for (long long i = 0; i < N; ++i) L.uoff[i + 1] = L.uoff[i] + L.kv[i];
        L.belief_floats = L.uoff[N];
        L.moff.assign((size_t)E + 1, 0);
        L.toff.assign((size_t)E + 1, 0);
        for (long long s = 0; s < E; ++s) {
            const int c = canon_of_slot[s];
            const int ki = L.kv[csrc(c)], kj = L.kv[cdst(c)];
            L.moff[s + 1] = L.moff[s] + kj;
            L.toff[s + 1] = L.toff[s] + ki * kj;
        }
        L.msg_floats = L.moff[E];
        // slots of heavy variables: each is evaluated by a wave of its own
        for (long long i = 0; i < N; ++i) {
            const int s0 = L.node_ptr[i], s1 = L.node_ptr[i + 1];
            if (ragged_flat(s1 - s0, L.kv[i], L.moff[s1] - L.moff[s0])) continue;
            for (int s = s0; s < s1; ++s) {
                L.heavy.push_back(s);
                L.heavy.push_back((int)i);
            }
        }
        L.coff.assign((size_t)E + 1, 0);
        for (long long c = 0; c < E; ++c) L.coff[c + 1] = L.coff[c] + L.kv[cdst(c)];
        L.unary.resize((size_t)L.belief_floats);
        for (long long i = 0; i < N; ++i) {
            double mx = -INFINITY;
            const double* lu = d->log_unary + L.uoff[i];
            for (int x = 0; x < L.kv[i]; ++x) mx = std::max(mx, lu[x]);
            for (int x = 0; x < L.kv[i]; ++x) L.unary[L.uoff[i] + x] = (float)(lu[x] - mx);
        }
        // table of slot s (source i, target k): psi(x_i, x_k), x_i major; the
        // host table of edge u = (a, b) is x_a major, so odd canonical
        // messages (b -> a) take it transposed; each table scaled to max 1
        std::vector<long long> poff((size_t)M + 1, 0);
        for (long long u = 0; u < M; ++u)
            poff[u + 1] = poff[u] + (long long)L.kv[d->edges[2 * u]] * L.kv[d->edges[2 * u + 1]];
        L.pair = kPairDense;
        L.pair_tab.resize((size_t)L.toff[E]);
        for (long long s = 0; s < E; ++s) {
            const int c = canon_of_slot[s];
            const long long u = c >> 1;
            const int ka = L.kv[d->edges[2 * u]], kb = L.kv[d->edges[2 * u + 1]];
            const double* P = d->pair + poff[u];
            double mx = 0.0;
            for (long long q = 0; q < (long long)ka * kb; ++q) mx = std::max(mx, P[q]);
            float* T = L.pair_tab.data() + L.toff[s];
            if (!(c & 1)) {
                for (int xa = 0; xa < ka; ++xa)
                    for (int xb = 0; xb < kb; ++xb) T[xa * kb + xb] = (float)(P[xa * kb + xb] / mx);
            } else {
                for (int xb = 0; xb < kb; ++xb)
                    for (int xa = 0; xa < ka; ++xa) T[xb * ka + xa] = (float)(P[xa * kb + xb] / mx);
            }
        }
        // the kernels take a wave per variable: no tiles
        L.tile_start.assign({0, (int)N});
        L.tile_slot.assign({0, (int)E});
        return BP_OK;
    }
    // unary: K = 2 log-odds, or log psi shifted so its max per node is 0
    if (L.layout == kLayoutLogOdds) {
        L.unary.resize((size_t)N);
        for (long long i = 0; i < N; ++i)
            L.unary[i] = (float)(d->log_unary[2 * i + 1] - d->log_unary[2 * i]);
    } else {
        L.unary.resize((size_t)(N * K));
        for (long long i = 0; i < N; ++i) {
            double mx = -INFINITY;
            for (long long x = 0; x < K; ++x) mx = std::max(mx, d->log_unary[i * K + x]);
            for (long long x = 0; x < K; ++x)
                L.unary[i * K + x] = (float)(d->log_unary[i * K + x] - mx);
        }
    }

    // Slot s holds m_{i->k}, whose update needs psi_{ik}(x_i, x_k).  For the
    // canonical message c of slot s and edge u = c >> 1 = (a, b): c even means
    // i = a, k = b (the table as given); c odd means i = b, so it is transposed.
    if (kind == BP_PAIR_ISING) {
        L.pair = kPairIsing;
        L.coupling.resize((size_t)std::max(E, 1ll));  // one entry for a graph without edges
        for (long long s = 0; s < E; ++s) L.coupling[s] = (float)d->coupling[canon_of_slot[s] >> 1];
    } else if (kind == BP_PAIR_SHARED) {
        bool sym = true;
        for (long long x = 0; x < K; ++x)
            for (long long y = 0; y < K; ++y)
                if (d->shared[x * K + y] != d->shared[y * K + x]) sym = false;
        double mx = 0.0;
        for (long long i = 0; i < K * K; ++i) mx = std::max(mx, d->shared[i]);
        L.pair_tab.resize((size_t)(K * K));
        for (long long x = 0; x < K; ++x)
            for (long long y = 0; y < K; ++y) L.pair_tab[x * K + y] = (float)(d->shared[x * K + y] / mx);
        L.pair = sym ? kPairShared : kPairSharedAsym;
        if (!sym) {
            L.orient.resize((size_t)E);
            for (long long s = 0; s < E; ++s) L.orient[s] = (canon_of_slot[s] & 1) ? 1 : 0;
        }
    } else {
        L.pair = kPairDense;
        L.pair_tab.resize((size_t)(E * K * K));
        for (long long s = 0; s < E; ++s) {
            const int c = canon_of_slot[s];
            const double* P = d->pair + (size_t)(c >> 1) * K * K;
            double mx = 0.0;
            for (long long i = 0; i < K * K; ++i) mx = std::max(mx, P[i]);
            float* T = L.pair_tab.data() + (size_t)s * K * K;
            for (long long xi = 0; xi < K; ++xi)
                for (long long xk = 0; xk < K; ++xk)
                    T[xi * K + xk] = (float)(((c & 1) ? P[xk * K + xi] : P[xi * K + xk]) / mx);
        }
    }

    // node tiles: greedy runs of target nodes within the slot and node limits;
    // a node whose in-degree alone exceeds the slot limit gets a tile of its own
    const int slot_lim = L.layout == kLayoutLogOdds ? kTileSlotsLogOdds
                                                    : std::max(1, kTileFloatsGeneric / (int)K);
    const int node_lim = L.layout == kLayoutLogOdds ? kTileNodesLogOdds
                                                    : std::min(kTileNodesMax, slot_lim);
    L.tile_start.clear();
    long long n = 0;
    while (n < N) {
        L.tile_start.push_back((int)n);
        const long long s_begin = L.node_ptr[n];
        long long m = n;
        while (m < N && (m - n) < node_lim && (L.node_ptr[m + 1] - s_begin) <= slot_lim) ++m;
        if (m == n) m = n + 1;  // oversize node
        n = m;
    }
    L.tile_start.push_back((int)N);
    L.tile_slot.resize(L.tile_start.size());
    for (size_t i = 0; i < L.tile_start.size(); ++i) L.tile_slot[i] = L.node_ptr[L.tile_start[i]];
    L.tiles4.clear();
    L.big4.clear();
    L.tile_nodes_max = 1;
    L.tile_big = 0;
    for (size_t i = 0; i + 1 < L.tile_start.size(); ++i) {
        if (L.tile_slot[i + 1] - L.tile_slot[i] > slot_lim)
            L.tile_big = 1;
        else
            L.tile_nodes_max = std::max(L.tile_nodes_max, L.tile_start[i + 1] - L.tile_start[i]);
    }
    for (size_t i = 0; i + 1 < L.tile_start.size(); ++i) {
        const int q[4] = {L.tile_start[i], L.tile_start[i + 1], L.tile_slot[i], L.tile_slot[i + 1]};
        std::vector<int>& dstv = (q[3] - q[2] > slot_lim) ? L.big4 : L.tiles4;
        dstv.insert(dstv.end(), q, q + 4);
    }
    // The regular-tile kernel also runs the iteration bookkeeping, so it must
    // launch even when every node is oversized: give it one empty tile.
    if (L.tiles4.empty()) L.tiles4.insert(L.tiles4.end(), {0, 0, 0, 0});
    return BP_OK;
}

}  // namespace

// The leading fields of DevState the host reads after a run or at a poll
// (everything before the selection histograms).
constexpr size_t kStateReadback = offsetof(DevState, hist);

// Sparse mode 2 switches to sparse re-evaluation once n_t <= E / kSparseSwitch.
#ifndef BP_SPARSE_SWITCH
#define BP_SPARSE_SWITCH 16
#endif
constexpr unsigned long long kSparseSwitch = BP_SPARSE_SWITCH;

struct bp_graph {
    HostLayout L;
    Offsets off;
    int device = 0;
    hipStream_t stream = nullptr;
    char* base = nullptr;
    bool owns_memory = false;
    // Message buffers: two pairs; pair p holds m^{t+1} under the larger [p][0]
    // and the smaller [p][1] keep threshold.  (cur_pair, cur_sel) locates m^t.
    int cur_pair = 0;
    int cur_sel = 0;
    long long t_next = 0;        // global iteration number of the next evaluation
    long long prev_active = -1;  // n_{t_next - 1}
    DevState* host_state = nullptr;  // pinned mirror
    int num_cus = 0;                 // compute units of the device
    int resident[4] = {0, 0, 0, 0};  // log-odds eval blocks resident per CU, by mode
    int lo_grid = 0;                 // tuned persistent grid of the K = 2 kernel (0: not yet)
    // sparse re-evaluation buffers: dirty u8 [N], active-node flag u8 [N],
    // target node int32 [E]; in the graph's memory (BP_FLAG_SPARSE_BUFFERS) or
    // allocated by the first sparse run (sparse_owned); the target index is
    // built once (sparse_ready)
    char* sparse_mem = nullptr;
    bool sparse_owned = false;
    bool sparse_ready = false;
    unsigned char* sp_dirty = nullptr;
    unsigned char* sp_hasact = nullptr;
    int* sp_dst = nullptr;
    // residual splash buffers: variable keys u32 [N], level marks u32 [3][N],
    // level lists i32 [3][N]; in the graph's memory (BP_FLAG_SPLASH_BUFFERS) or
    // allocated by the first BP_RS run (splash_owned); marks start at 0 and
    // carry the tag of the iteration that set them (rs_tag: the last tag used)
    char* splash_mem = nullptr;
    bool splash_owned = false;
    unsigned int rs_tag = 0;

    template <typename T>
    T* at(size_t o) const { return reinterpret_cast<T*>(base + o); }
    float* msg(int pair, int sel) const { return at<float>(off.msg[2 * pair + sel]); }
    float* cur() const { return msg(cur_pair, cur_sel); }
    DevState* st() const { return at<DevState>(off.state); }
    CounterLine* ctr() const { return at<CounterLine>(off.ctr); }
};

int create_graph_from_layout(HostLayout& layout, const bp_graph_desc* desc, bp_graph** out,
                              bool fail_upload = false);

extern "C" {

void bp_default_opts(bp_run_opts* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->max_iters = 10000;
    o->check_every = 16;
    o->dynamic_p = 1;
    o->high_p = 1.0;
    o->ratio_threshold = 0.9;
    o->warm_start = 0;
    o->profile = 0;
    o->splash_depth = 2;
}

const char* bp_last_error(void) { return g_last_error.c_str(); }

int bp_workspace_bytes(const bp_graph_desc* desc, uint64_t* bytes) {
    HostLayout L;
    int rc = build_layout(desc, L);
    if (rc != BP_OK) return rc;
    if (bytes) *bytes = plan(L).total;
    return BP_OK;
}

int bp_create_graph(const bp_graph_desc* desc, bp_graph** out) {
    if (!out) return fail(BP_EINVAL, "out is NULL");
    *out = nullptr;
    HostLayout L;
    int rc = build_layout(desc, L);
    if (rc != BP_OK) return rc;
    return create_graph_from_layout(L, desc, out);
}

}  // extern "C"

// A graph from an already built (and validated) layout; desc supplies the
// stream and the optional workspace.  The layout is moved into the graph on
// success and left with the caller on failure (the server admits it again or
// reports it).  fail_upload makes the upload step fail as a device error would
// (bp_server_inject_failures).
int create_graph_from_layout(HostLayout& layout, const bp_graph_desc* desc, bp_graph** out,
                             bool fail_upload) {
    bp_graph* g = new (std::nothrow) bp_graph();
    if (!g) return fail(BP_ENOMEM, "host allocation failed");
    g->L = std::move(layout);
    // every failure below hands the layout back before the graph is released
    auto give_back = [&](int code) {
        layout = std::move(g->L);
        bp_destroy_graph(g);
        return code;
    };
    g->off = plan(g->L);
    g->stream = (hipStream_t)desc->stream;
    hipError_t e = hipGetDevice(&g->device);
    if (e != hipSuccess) return give_back(hip_fail(e, "hipGetDevice"));
    if (desc->workspace) {
        if ((uintptr_t)desc->workspace % 256 != 0)
            return give_back(fail(BP_EINVAL, "workspace must be 256-byte aligned"));
        if (desc->workspace_bytes < g->off.total)
            return give_back(fail(BP_ENOMEM, "workspace of %llu bytes < %llu needed",
                                  (unsigned long long)desc->workspace_bytes,
                                  (unsigned long long)g->off.total));
        g->base = (char*)desc->workspace;
    } else {
        e = hipMalloc((void**)&g->base, g->off.total);
        if (e != hipSuccess) {
            g->base = nullptr;
            (void)hipGetLastError();
            return give_back(fail(e == hipErrorOutOfMemory ? BP_ENOMEM : BP_EDEVICE,
                                  "hipMalloc(%zu): %s", g->off.total, hipGetErrorString(e)));
        }
        g->owns_memory = true;
    }
    e = hipHostMalloc((void**)&g->host_state, sizeof(DevState), hipHostMallocDefault);
    if (e != hipSuccess) {
        g->host_state = nullptr;
        return give_back(hip_fail(e, "hipHostMalloc"));
    }
    if (fail_upload) return give_back(fail(BP_EDEVICE, "upload: injected failure"));
    const HostLayout& L = g->L;
    hipStream_t s = g->stream;
    auto up = [&](size_t o, const void* p, size_t n) -> hipError_t {
        if (n == 0) return hipSuccess;
        return hipMemcpyAsync(g->base + o, p, n, hipMemcpyHostToDevice, s);
    };
    hipError_t errs[17] = {
        up(g->off.kv, L.kv.data(), sizeof(int) * L.kv.size()),
        up(g->off.uoff, L.uoff.data(), sizeof(int) * L.uoff.size()),
        up(g->off.moff, L.moff.data(), sizeof(int) * L.moff.size()),
        up(g->off.toff, L.toff.data(), sizeof(int) * L.toff.size()),
        up(g->off.heavy, L.heavy.data(), sizeof(int) * L.heavy.size()),
        up(g->off.rev16, L.rev16.data(), sizeof(short) * L.rev16.size()),
        up(g->off.tile_slot, L.tile_slot.data(), sizeof(int) * L.tile_slot.size()),
        up(g->off.tiles4, L.tiles4.data(), sizeof(int) * L.tiles4.size()),
        up(g->off.big4, L.big4.data(), sizeof(int) * L.big4.size()),
        up(g->off.node_ptr, L.node_ptr.data(), sizeof(int) * L.node_ptr.size()),
        up(g->off.rev, L.rev.data(), sizeof(int) * L.rev.size()),
        up(g->off.tile, L.tile_start.data(), sizeof(int) * L.tile_start.size()),
        up(g->off.coupling, L.coupling.data(), sizeof(float) * L.coupling.size()),
        up(g->off.unary, L.unary.data(), sizeof(float) * L.unary.size()),
        up(g->off.pair, L.pair_tab.data(), sizeof(float) * L.pair_tab.size()),
        up(g->off.orient, L.orient.data(), L.orient.size())};
    for (hipError_t x : errs)
        if (x != hipSuccess) return give_back(hip_fail(x, "upload"));
    const float uni = L.layout == kLayoutLogOdds ? 0.0f : 1.0f / (float)L.K;
    e = L.layout == kLayoutRagged
            ? launch_fill_ragged(g->msg(0, 0), g->at<int>(g->off.moff), (int)L.E, s)
            : launch_fill(g->msg(0, 0), uni, L.msg_floats, s);
    if (e == hipSuccess) e = launch_init_state(g->st(), g->ctr(), s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return give_back(hip_fail(e, "initialise"));
    g->cur_pair = 0;
    g->cur_sel = 0;
    e = hipDeviceGetAttribute(&g->num_cus, hipDeviceAttributeMultiprocessorCount, g->device);
    if (e != hipSuccess) return give_back(hip_fail(e, "hipDeviceGetAttribute"));
    for (int m = 0; m < 4; ++m) g->resident[m] = logodds_blocks_per_cu(m);
    *out = g;
    return BP_OK;
}

extern "C" {

void bp_destroy_graph(bp_graph* g) {
    if (!g) return;
    {
        DeviceGuard dg(g->device);
        if (g->base) (void)hipStreamSynchronize(g->stream);
        if (g->owns_memory && g->base) (void)hipFree(g->base);
        if (g->sparse_owned && g->sparse_mem) (void)hipFree(g->sparse_mem);
        if (g->splash_owned && g->splash_mem) (void)hipFree(g->splash_mem);
        if (g->host_state) (void)hipHostFree(g->host_state);
    }
    delete g;
}

int bp_graph_info_get(const bp_graph* g, bp_graph_info* info) {
    if (!g || !info) return fail(BP_EINVAL, "NULL argument");
    info->num_vars = g->L.N;
    info->num_states = g->L.K;
    info->num_edges = g->L.M;
    info->num_messages = g->L.E;
    info->layout = g->L.layout;
    info->num_tiles = (int)g->L.tile_start.size() - 1;
    info->device_bytes = g->off.total;
    info->eval_blocks = g->lo_grid;
    info->heavy_slots = (int)(g->L.heavy.size() / 2);
    return BP_OK;
}

static unsigned int keep_threshold(double p) {
    // U = k * 2^-24 < p  <=>  k < ceil(p * 2^24)  (p * 2^24 is exact in double)
    double x = std::ceil(p * 16777216.0);
    if (x < 0.0) x = 0.0;
    if (x > 16777216.0) x = 16777216.0;
    return (unsigned int)x;
}

// The evaluation arguments of a run of `schedule` on g (everything but the
// per-launch fields t, it, in_buf, out_buf, after_final).
static EvalArgs run_args(const bp_graph* g, int schedule, double eps, double p, uint64_t seed,
                         const bp_run_opts& o, long long& rbp_k_out) {
    const HostLayout& L = g->L;
    // residual splash evaluates as frontier RBP does (candidates and keys)
    const int mode = schedule == BP_LBP ? kModeLBP
                     : (schedule == BP_RBP || schedule == BP_RS) ? kModeRBP
                                                                  : kModeRnBP;
    const unsigned int thr_lo = keep_threshold(p);
    const unsigned int thr_hi = keep_threshold(o.high_p);
    long long rbp_k = (long long)std::ceil(p * (double)L.E);
    if (rbp_k < 1) rbp_k = 1;
    // RBP: at most every message; residual splash: at most every variable (roots)
    const long long k_cap = schedule == BP_RS ? (long long)L.N : L.E;
    if (rbp_k > k_cap) rbp_k = k_cap;

    EvalArgs a{};
    a.tile_start = g->at<int>(g->off.tile);
    a.tile_slot = g->at<int>(g->off.tile_slot);
    a.tiles4 = g->at<int>(g->off.tiles4);
    a.big4 = g->at<int>(g->off.big4);
    a.num_tiles = L.layout == kLayoutLogOdds ? (int)(L.tiles4.size() / 4) : (int)L.tile_start.size() - 1;
    a.num_big = L.layout == kLayoutLogOdds ? (int)(L.big4.size() / 4) : 0;
    a.tiles_per_xcd = (a.num_tiles + 7) / 8;
    {
        // one persistent block per resident slot (the least occupancy over the
        // modes this run launches), never more than the tiles need
        const int mode_now = mode;
        int per_cu = std::min(g->resident[mode_now], g->resident[kModeEvalOnly]);
        if (per_cu < 1) per_cu = 1;
        long long cap = (long long)per_cu * std::max(g->num_cus, 1);
        cap = std::max<long long>(8, cap / 8 * 8);
        a.pipe_grid = (int)std::min<long long>(cap, std::max(8, 8 * a.tiles_per_xcd));
    }
    if (L.layout == kLayoutLogOdds && g->lo_grid > 0) a.pipe_grid = g->lo_grid;
    a.node_ptr = g->at<int>(g->off.node_ptr);
    a.rev = g->at<int>(g->off.rev);
    a.rev16 = L.rev16.empty() ? nullptr : g->at<short>(g->off.rev16);
    a.coupling = g->at<float>(g->off.coupling);
    a.unary = g->at<float>(g->off.unary);
    a.pair = g->at<float>(g->off.pair);
    a.orient = g->at<unsigned char>(g->off.orient);
    a.kv = g->at<int>(g->off.kv);
    a.uoff = g->at<int>(g->off.uoff);
    a.moff = g->at<int>(g->off.moff);
    a.toff = g->at<int>(g->off.toff);
    a.heavy = g->at<int>(g->off.heavy);
    a.num_heavy = (int)(L.heavy.size() / 2);
    if (L.layout == kLayoutRagged) {
        // a wave per heavy slot and per variable, grid-stride: at most 8
        // blocks per CU
        const long long waves = (long long)L.N + a.num_heavy;
        const long long blocks = (waves + kBlock / 64 - 1) / (kBlock / 64);
        a.pipe_grid = (int)std::max<long long>(
            1, std::min<long long>(blocks, 8ll * std::max(g->num_cus, 1)));
    }
    a.cand = g->at<float>(g->off.cand);
    a.keys = g->at<unsigned int>(g->off.keys);
    a.st = g->st();
    a.ctr = g->ctr();
    a.num_states = L.K;
    a.pair_kind = L.pair;
    a.sched = schedule == BP_RS ? kModeRS : mode;
    a.eps = (float)eps;
    // The device compares FP32 residuals with an FP32 threshold: take the largest
    // float <= eps, so that for every float r, r > eps_f exactly when r > eps.
    if ((double)a.eps > eps) a.eps = std::nextafter(a.eps, -INFINITY);
    a.key0 = (unsigned int)(seed & 0xFFFFFFFFu);
    a.key1 = (unsigned int)(seed >> 32);
    a.dynamic_p = o.dynamic_p;
    a.ratio_threshold = o.ratio_threshold;
    a.prev_active_host = g->prev_active;
    a.num_messages = (unsigned long long)L.E;
    a.num_nodes = L.N;
    a.tile_nodes_max = L.tile_nodes_max;
    a.tile_big = L.tile_big;
    a.no_mfma = L.no_mfma;
    a.mfma_bf16 = L.mfma_bf16;
    a.rbp_k = (unsigned long long)rbp_k;
    a.sel0 = g->cur_sel;
    if (mode == kModeRnBP && o.dynamic_p) {
        a.thr_a = std::max(thr_lo, thr_hi);
        a.thr_b = std::min(thr_lo, thr_hi);
        a.low_is_a = thr_lo >= thr_hi;
        a.two_outputs = thr_lo != thr_hi;
    } else {
        a.thr_a = a.thr_b = thr_lo;
        a.low_is_a = 1;
        a.two_outputs = 0;
    }
    // [E][K] rows: one whole row per message and the other outcome only where
    // the two keep decisions differ
    a.row_flags = (a.two_outputs && L.layout == kLayoutGeneric) ? 1 : 0;

    rbp_k_out = rbp_k;
    return a;
}

}  // extern "C"

// Device memory of one run besides the graph's arrays: iteration state,
// counters and the per-block tie counts of the top-k.  bp_run takes them from
// the graph's memory, bp_run_noalloc from the library's static scratch array.
struct RunScratch {
    DevState* st;
    CounterLine* ctr;
    unsigned int* ties;
    bool noalloc;  // no events, no buffer allocation
};

static int run_impl(bp_graph* g, int schedule, double eps, double p, uint64_t seed,
                    const bp_run_opts* opts, bp_run_stats* stats, const RunScratch& rs) {
    if (!g) return fail(BP_EINVAL, "graph is NULL");
    if (schedule != BP_LBP && schedule != BP_RBP && schedule != BP_RNBP && schedule != BP_RS)
        return fail(BP_EINVAL, "unknown schedule %d", schedule);
    if (!(eps >= 0.0) || !std::isfinite(eps)) return fail(BP_EINVAL, "eps must be finite and >= 0");
    if (schedule != BP_LBP && !(p > 0.0 && p <= 1.0)) return fail(BP_EINVAL, "p must be in (0, 1]");
    bp_run_opts o;
    bp_default_opts(&o);
    if (opts) o = *opts;
    if (o.max_iters < 0) return fail(BP_EINVAL, "max_iters < 0");
    if (o.check_every < 1) return fail(BP_EINVAL, "check_every < 1");
    if (schedule == BP_RNBP && o.dynamic_p && !(o.high_p > 0.0 && o.high_p <= 1.0))
        return fail(BP_EINVAL, "high_p must be in (0, 1]");
    if (!std::isfinite(o.ratio_threshold)) return fail(BP_EINVAL, "ratio_threshold not finite");
    if (o.sparse < 0 || o.sparse > 2) return fail(BP_EINVAL, "sparse must be 0, 1 or 2");
    if (o.sparse) {
        if (schedule == BP_LBP)
            return fail(BP_EINVAL, "sparse re-evaluation is for BP_RNBP and BP_RBP only");
        if (g->L.layout != kLayoutLogOdds)
            return fail(BP_EINVAL, "sparse re-evaluation needs K = 2 Ising potentials");
        if (!g->L.big4.empty())
            return fail(BP_EINVAL, "sparse re-evaluation needs every node within one tile");
        if (schedule == BP_RS) return fail(BP_EINVAL, "residual splash has no sparse mode");
    }
    const bool splash = schedule == BP_RS;
    if (splash) {
        if (g->L.layout != kLayoutLogOdds)
            return fail(BP_EINVAL, "residual splash needs K = 2 Ising potentials in the "
                                   "one-log-odds-per-message layout");
        if (o.splash_depth < 0 || o.splash_depth > kSplashMaxDepth)
            return fail(BP_EINVAL, "splash_depth must be 0, 1 or 2");
    }
    if (rs.noalloc && o.profile)
        return fail(BP_EINVAL, "profile needs HIP events, which bp_run_noalloc does not create");
    DeviceGuard dg(g->device);
    const HostLayout& L = g->L;
    hipStream_t s = g->stream;
    // sparse re-evaluation and residual splash need the target index of the
    // sparse buffers
    if ((o.sparse || splash) && !g->sparse_ready) {
        const size_t nb = ((size_t)L.N + 255) / 256 * 256;
        const size_t bytes = sparse_bytes(L);
        char* mem = g->sparse_mem;
        bool owned = g->sparse_owned;
        if (!mem && L.sparse_reserved) mem = g->at<char>(g->off.sparse);
        if (!mem) {
            if (rs.noalloc)
                return fail(BP_EINVAL, "%s without allocation needs a graph created with "
                                       "BP_FLAG_SPARSE_BUFFERS",
                            splash ? "residual splash" : "sparse re-evaluation");
            hipError_t e = hipMalloc(&mem, bytes);
            if (e != hipSuccess)
                return fail(e == hipErrorOutOfMemory ? BP_ENOMEM : BP_EDEVICE,
                            "sparse buffers (%zu bytes): %s", bytes, hipGetErrorString(e));
            owned = true;
        }
        EvalArgs b{};
        b.node_ptr = g->at<int>(g->off.node_ptr);
        b.rev = g->at<int>(g->off.rev);
        b.num_nodes = L.N;
        b.dirty = (unsigned char*)mem;
        b.dst = (int*)(mem + 2 * nb);
        hipError_t e = launch_sparse_setup(b, 1, s);
        if (e != hipSuccess) {
            // keep the graph without a target index, so that a later run retries
            if (owned && mem != g->sparse_mem) (void)hipFree(mem);
            return hip_fail(e, "target index");
        }
        g->sparse_mem = mem;
        g->sparse_owned = owned;
        g->sparse_ready = true;
        g->sp_dirty = (unsigned char*)mem;
        g->sp_hasact = (unsigned char*)(mem + nb);
        g->sp_dst = (int*)(mem + 2 * nb);
    }
    if (splash && !g->splash_mem) {
        char* mem = nullptr;
        bool owned = false;
        const size_t bytes = splash_bytes(L.N);
        if (L.splash_reserved) {
            mem = g->at<char>(g->off.splash);
        } else {
            if (rs.noalloc)
                return fail(BP_EINVAL, "residual splash without allocation needs a graph created "
                                       "with BP_FLAG_SPLASH_BUFFERS");
            hipError_t e = hipMalloc(&mem, bytes);
            if (e != hipSuccess)
                return fail(e == hipErrorOutOfMemory ? BP_ENOMEM : BP_EDEVICE,
                            "splash buffers (%zu bytes): %s", bytes, hipGetErrorString(e));
            owned = true;
        }
        const size_t part = (sizeof(unsigned int) * (size_t)L.N + 255) & ~size_t(255);
        hipError_t e = launch_fill_u32((unsigned int*)(mem + part), 0u,
                                       (long long)L.N * (kSplashMaxDepth + 1), s);
        if (e != hipSuccess) {
            if (owned) (void)hipFree(mem);
            return hip_fail(e, "splash marks");
        }
        g->splash_mem = mem;
        g->splash_owned = owned;
        g->rs_tag = 0;
    }
    if (!o.warm_start) {
        const float uni = L.layout == kLayoutLogOdds ? 0.0f : 1.0f / (float)L.K;
        if (L.layout == kLayoutRagged)
            HIP_OK(launch_fill_ragged(g->cur(), g->at<int>(g->off.moff), (int)L.E, s), "fill");
        else
            HIP_OK(launch_fill(g->cur(), uni, L.msg_floats, s), "fill");
        g->t_next = 0;
        g->prev_active = -1;
    }
    if (g->t_next + o.max_iters + 1 > 0xFFFFFFFFLL)
        return fail(BP_EINVAL, "iteration counter would pass 2^32");
    HIP_OK(launch_init_state(rs.st, rs.ctr, s), "init state");

    // residual splash evaluates with the frontier-RBP kernels (in place)
    const int mode = schedule == BP_LBP ? kModeLBP
                     : (schedule == BP_RBP || splash) ? kModeRBP
                                                      : kModeRnBP;
    long long rbp_k = 0;
    EvalArgs a = run_args(g, schedule, eps, p, seed, o, rbp_k);
    a.st = rs.st;
    a.ctr = rs.ctr;
    // frontier RBP on the K = 2 kernel: the evaluation also counts the top-k's
    // first radix digit (not for oversized nodes, the sparse phase, or k = E)
    a.hist0 = (mode == kModeRBP && !splash && L.layout == kLayoutLogOdds && a.num_big == 0 &&
               rbp_k < L.E && o.sparse != 1)
                  ? 1
                  : 0;
    a.dirty = g->sp_dirty;
    a.hasact = g->sp_hasact;
    a.dst = g->sp_dst;
    // sparse phase: messages committed in place in the buffer that holds m^t
    bool sparse_now = false;
    long long sp_it0 = 0;  // first sparse iteration of this run
    float* sp_buf = nullptr;
    if (o.sparse == 1) {
        sparse_now = true;
        sp_it0 = 0;
        sp_buf = g->cur();
        HIP_OK(launch_sparse_setup(a, 0, s), "dirty flags");
    }

    RsArgs rsa{};
    if (splash) {
        const size_t part = (sizeof(unsigned int) * (size_t)L.N + 255) & ~size_t(255);
        const size_t lv =
            (sizeof(unsigned int) * (size_t)L.N * (kSplashMaxDepth + 1) + 255) & ~size_t(255);
        rsa.st = rs.st;
        rsa.node_ptr = a.node_ptr;
        rsa.rev = a.rev;
        rsa.dst = g->sp_dst;
        rsa.unary = a.unary;
        rsa.coupling = a.coupling;
        rsa.keys = a.keys;
        rsa.m = g->cur();
        rsa.cand = a.cand;
        rsa.vkey = (unsigned int*)g->splash_mem;
        rsa.mark = (unsigned int*)(g->splash_mem + part);
        rsa.list = (int*)(g->splash_mem + part + lv);
        rsa.num_nodes = L.N;
        rsa.depth = o.splash_depth;
    }
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    if (!rs.noalloc) {
        HIP_OK(hipEventCreate(&ev0), "event");
        HIP_OK(hipEventCreate(&ev1), "event");
    }
    // profile = k > 0.  When the evaluation kernel is the only launch of an
    // iteration (LBP / RnBP without oversized nodes), a pair of events brackets
    // each chunk of back-to-back launches: chunk time / launches is the kernel's
    // average duration (gaps between dispatches included).  Otherwise every
    // k-th evaluation launch gets its own pair of events.
    std::vector<hipEvent_t> kev;
    std::vector<int> kev_used;
    const long long prof_every = o.profile > 0 ? o.profile : 0;
    bool prof_window = prof_every && mode != kModeRBP && a.num_big == 0 && !sparse_now;
    if (prof_every) {
        kev.resize(2 * (size_t)o.check_every);
        kev_used.assign((size_t)o.check_every, 0);
        for (auto& x : kev) HIP_OK(hipEventCreate(&x), "event");
    }
    double kernel_ms = 0.0;
    long long kernel_launches = 0;
    // Launch-shape tuning of the K = 2 kernel's persistent grid: the first
    // run of a graph that is long enough times kTuneLaunches launches at each
    // candidate grid (1, 2, 4 blocks per compute unit and every resident
    // block) and keeps the fastest for this run and later ones.  The grid only
    // decides which block evaluates which tile, so no result depends on it.
    constexpr int kTuneLaunches = 8;
    std::vector<int> tcand;
    std::vector<hipEvent_t> tev;
    bool tune = L.layout == kLayoutLogOdds && !rs.noalloc && g->lo_grid == 0 &&
                mode != kModeRBP && a.num_big == 0 && !sparse_now && o.sparse == 0;
    if (tune) {
        const long long most = std::max(8, 8 * a.tiles_per_xcd);
        for (int c : {1, 2, 4, 0}) {
            long long v = c ? (long long)c * std::max(g->num_cus, 1) : a.pipe_grid;
            v = std::max<long long>(8, std::min(most, v / 8 * 8));
            if (std::find(tcand.begin(), tcand.end(), (int)v) == tcand.end()) tcand.push_back((int)v);
        }
        tune = tcand.size() > 1 && o.max_iters >= (long long)tcand.size() * kTuneLaunches;
    }
    if (tune) {
        tev.assign(2 * tcand.size(), nullptr);
        for (auto& x : tev) HIP_OK(hipEventCreate(&x), "event");
    }
    const long long tune_end = tune ? (long long)tcand.size() * kTuneLaunches : 0;
    if (ev0) HIP_OK(hipEventRecord(ev0, s), "event record");

    const int kp = kpad(L.K);
    const long long t_start = g->t_next;
    const int pair0 = g->cur_pair;
    float* const start_buf = g->cur();
    unsigned int* ties = rs.ties;
    int in_chunk = 0;
    long long it = 0;
    bool final_launched = false;
    for (;; ++it) {
        const long long t = t_start + it;
        final_launched = it == o.max_iters;
        if (sparse_now) {
            // one sparse iteration: evaluate the dirty nodes, then close and commit
            a.in_buf[0] = a.in_buf[1] = sp_buf;
            a.out_buf[0] = a.out_buf[1] = sp_buf;
            a.t = (unsigned int)t;
            a.it = it;
            a.after_final = final_launched ? 1 : 0;
            a.sp_first = it == sp_it0 ? 1 : 0;
            if (mode == kModeRBP) {
                HIP_OK(launch_sparse_rbp_eval(a, s), "sparse evaluation");
                if (!final_launched) {
                    const int all = rbp_k >= L.E;
                    if (!all)
                        HIP_OK(launch_rbp_select(rs.st, a.keys, a.rev, (int)L.E,
                                                 (unsigned int)rbp_k, nullptr, 0, ties, s),
                               "top-k select");
                    const RbpSparse sp{a.dirty, a.dst, a.ctr, a.eps, (int)((t + 1) & 3), 1};
                    HIP_OK(launch_rbp_commit(rs.st, a.keys, a.rev, a.cand, sp_buf, (int)L.E, L.row,
                                             all, (int)(t & 3), ties, sp, nullptr, s),
                           "top-k commit");
                }
            } else {
                HIP_OK(launch_sparse_iteration(a, s), "sparse iteration");
            }
            ++in_chunk;
            if (in_chunk == o.check_every || final_launched) {
                HIP_OK(hipMemcpyAsync(g->host_state, rs.st, kStateReadback, hipMemcpyDeviceToHost,
                                      s),
                       "state readback");
                HIP_OK(hipStreamSynchronize(s), "synchronize");
                in_chunk = 0;
                if (g->host_state->done || final_launched) break;
            }
            continue;
        }
        if (mode == kModeRBP) {
            // frontier residual BP commits in place after the top-k selection
            a.in_buf[0] = a.in_buf[1] = start_buf;
            a.out_buf[0] = a.out_buf[1] = nullptr;
        } else {
            const int pin = (int)((pair0 + it) & 1);
            if (it == 0) {
                a.in_buf[0] = a.in_buf[1] = start_buf;
            } else {
                a.in_buf[0] = g->msg(pin, 0);
                a.in_buf[1] = g->msg(pin, 1);
            }
            a.out_buf[0] = g->msg(pin ^ 1, 0);
            a.out_buf[1] = g->msg(pin ^ 1, 1);
        }
        a.t = (unsigned int)t;
        a.it = it;
        a.after_final = 0;
        const int emode = final_launched ? kModeEvalOnly : mode;
        const bool timed = prof_every && !prof_window && (it % prof_every) == 0;
        const bool tuning = tune && it < tune_end;
        if (tuning && it % kTuneLaunches == 0) {
            a.pipe_grid = tcand[(size_t)(it / kTuneLaunches)];
            HIP_OK(hipEventRecord(tev[2 * (it / kTuneLaunches)], s), "event record");
        }
        if (prof_window && in_chunk == 0) HIP_OK(hipEventRecord(kev[0], s), "event record");
        if (timed) HIP_OK(hipEventRecord(kev[2 * in_chunk], s), "event record");
        HIP_OK(launch_eval(L.layout, kp, emode, a, s), "evaluation kernel");
        if (timed) HIP_OK(hipEventRecord(kev[2 * in_chunk + 1], s), "event record");
        if (tuning && it % kTuneLaunches == kTuneLaunches - 1)
            HIP_OK(hipEventRecord(tev[2 * (it / kTuneLaunches) + 1], s), "event record");
        if (prof_every && !prof_window) kev_used[in_chunk] = timed ? 1 : 0;
        if (splash && !final_launched) {
            if (g->rs_tag == 0xFFFFFFFFu) {
                HIP_OK(launch_fill_u32(rsa.mark, 0u, (long long)L.N * (kSplashMaxDepth + 1), s),
                       "splash marks");
                g->rs_tag = 0;
            }
            rsa.tag = ++g->rs_tag;
            HIP_OK(launch_rs_gate(rs.st, rs.ctr, (int)(t & 3), s), "splash gate");
            HIP_OK(launch_rs_select(rsa, (unsigned int)rbp_k, rbp_k >= L.N ? 1 : 0, ties, s),
                   "splash roots");
            for (int q = 0; q <= 2 * rsa.depth; ++q) {
                const int d = q <= rsa.depth ? rsa.depth - q : q - rsa.depth;
                HIP_OK(launch_rs_level(rsa, d, s), "splash level");
            }
        } else if (mode == kModeRBP && !final_launched) {
            const int all = rbp_k >= L.E;
            // the first scan of the select is also the gate (IsConverged)
            if (all)
                HIP_OK(launch_rbp_gate(rs.st, rs.ctr, (int)(t & 3), s), "top-k gate");
            else
                HIP_OK(launch_rbp_select(rs.st, a.keys, a.rev, (int)L.E, (unsigned int)rbp_k,
                                         rs.ctr + (size_t)(t & 3) * kCounterCopies, a.hist0,
                                         ties, s),
                       "top-k select");
            HIP_OK(launch_rbp_commit(rs.st, a.keys, a.rev, a.cand, start_buf, (int)L.E, L.row, all,
                                     (int)(t & 3), ties, RbpSparse{},
                                     L.layout == kLayoutRagged ? a.moff : nullptr, s),
                   "top-k commit");
        }
        ++in_chunk;
        if (in_chunk == o.check_every || final_launched) {
            if (prof_window) HIP_OK(hipEventRecord(kev[1], s), "event record");
            HIP_OK(hipMemcpyAsync(g->host_state, rs.st, kStateReadback, hipMemcpyDeviceToHost, s),
                   "state readback");
            HIP_OK(hipStreamSynchronize(s), "synchronize");
            if (prof_window) {
                float ms = 0.0f;
                HIP_OK(hipEventElapsedTime(&ms, kev[0], kev[1]), "event time");
                kernel_ms += ms;
                kernel_launches += in_chunk;
            } else if (prof_every) {
                for (int i = 0; i < in_chunk; ++i) {
                    if (!kev_used[i]) continue;
                    float ms = 0.0f;
                    HIP_OK(hipEventElapsedTime(&ms, kev[2 * i], kev[2 * i + 1]), "event time");
                    kernel_ms += ms;
                    ++kernel_launches;
                }
            }
            in_chunk = 0;
            if (tune && it + 1 >= tune_end) {
                // every candidate has run: keep the fastest
                int best = -1;
                float best_ms = 0.0f;
                for (size_t c = 0; c < tcand.size(); ++c) {
                    float ms = 0.0f;
                    HIP_OK(hipEventElapsedTime(&ms, tev[2 * c], tev[2 * c + 1]), "event time");
                    if (best < 0 || ms < best_ms) {
                        best = (int)c;
                        best_ms = ms;
                    }
                }
                g->lo_grid = tcand[(size_t)best];
                a.pipe_grid = g->lo_grid;
                tune = false;
            }
            if (g->host_state->done || final_launched) break;
            if (o.sparse == 2 && (unsigned long long)g->host_state->last_active * kSparseSwitch <=
                                     (unsigned long long)L.E) {
                // switch to sparse re-evaluation: close evaluation t (as the next
                // launch's prologue would), find the buffer that holds m^{t+1},
                // and continue in place with every node dirty
                a.t = (unsigned int)(t + 1);
                a.it = it + 1;
                a.after_final = 0;
                HIP_OK(launch_close_run(a, s), "close evaluation");
                HIP_OK(hipMemcpyAsync(g->host_state, rs.st, kStateReadback, hipMemcpyDeviceToHost,
                                      s),
                       "state readback");
                HIP_OK(hipStreamSynchronize(s), "synchronize");
                if (g->host_state->done) break;
                if (mode == kModeRBP) {
                    sp_buf = start_buf;  // frontier residual BP already commits in place
                } else {
                    g->cur_pair = (int)((pair0 + it) & 1) ^ 1;
                    g->cur_sel = (int)g->host_state->in_sel[(t + 1) & 3];
                    sp_buf = g->cur();
                }
                HIP_OK(launch_sparse_setup(a, 0, s), "dirty flags");
                sparse_now = true;
                a.hist0 = 0;
                sp_it0 = it + 1;
                prof_window = false;
            }
        }
    }
    if (sparse_now) {
        HIP_OK(launch_sparse_rmax(a, s), "max residual");
    } else {
        // close the last launched evaluation (a no-op if a later prologue already did)
        a.t = (unsigned int)(t_start + it + 1);
        a.it = it + 1;
        a.after_final = final_launched ? 1 : 0;
        HIP_OK(launch_close_run(a, s), "close run");
    }
    if (ev1) HIP_OK(hipEventRecord(ev1, s), "event record");
    HIP_OK(hipMemcpyAsync(g->host_state, rs.st, kStateReadback, hipMemcpyDeviceToHost, s),
           "state readback");
    HIP_OK(hipStreamSynchronize(s), "synchronize");
    float total_ms = 0.0f;
    if (ev0) {
        HIP_OK(hipEventElapsedTime(&total_ms, ev0, ev1), "event time");
        (void)hipEventDestroy(ev0);
        (void)hipEventDestroy(ev1);
    }
    for (auto& x : kev) (void)hipEventDestroy(x);
    for (auto& x : tev) (void)hipEventDestroy(x);

    const DevState& h = *g->host_state;
    const bool converged = h.done != 0;
    const long long final_t = converged ? h.conv_t : h.last_t;
    if (mode != kModeRBP && !sparse_now) {
        g->cur_pair = (int)((pair0 + (final_t - t_start)) & 1);
        g->cur_sel = (int)h.in_sel[final_t & 3];
        if (a.row_flags && final_t > t_start) {
            // m^final_t: whole rows of the outcome launch final_t - 1 wrote whole,
            // flagged rows of the other where the choice was the other
            const int prim = (int)h.in_sel[(final_t - 1) & 3];
            float* bufs[2] = {g->msg(g->cur_pair, 0), g->msg(g->cur_pair, 1)};
            HIP_OK(launch_resolve_rows(bufs, prim, g->cur_sel, L.E, L.K, s), "resolve rows");
            HIP_OK(hipStreamSynchronize(s), "synchronize");
            g->cur_sel = prim;
        }
    }
    g->t_next = final_t;
    g->prev_active = h.last_prev;
    if (stats) {
        std::memset(stats, 0, sizeof(*stats));
        stats->iterations = (long long)h.iterations;
        stats->converged = converged ? 1 : 0;
        stats->last_active = (long long)h.last_active;
        float rm;
        std::memcpy(&rm, &h.last_rmax, sizeof(rm));
        stats->last_max_residual = rm;
        stats->evaluated = (long long)h.evaluated;
        stats->committed = (long long)h.committed;
        stats->final_t = final_t;
        stats->device_ms = total_ms;
        stats->eval_kernel_ms = kernel_ms;
        stats->eval_kernel_launches = kernel_launches;
    }
    return converged ? BP_OK : BP_NOT_CONVERGED;
}

// Scratch bytes of a run for a graph of E messages and N variables: state,
// counters, per-block tie counts (of a top-k over messages or variables).
size_t bp::run_scratch_bytes(long long E, long long N) {
    const size_t st = (sizeof(DevState) + 255) & ~size_t(255);
    const size_t ctr = sizeof(CounterLine) * 4 * kCounterCopies;
    return st + ctr + sizeof(unsigned int) * (size_t)(std::max(E, N) / 4096 + 2);
}

int bp::run_with_scratch(bp_graph* g, int schedule, double eps, double p, uint64_t seed,
                         const bp_run_opts* opts, bp_run_stats* stats, char* scratch,
                         size_t scratch_bytes) {
    if (!g) return fail(BP_EINVAL, "graph is NULL");
    const size_t need = run_scratch_bytes(g->L.E, g->L.N);
    if (need > scratch_bytes)
        return fail(BP_EINVAL, "graph of %lld messages needs %zu bytes of run scratch, the "
                               "static scratch holds %zu",
                    (long long)g->L.E, need, scratch_bytes);
    const size_t st = (sizeof(DevState) + 255) & ~size_t(255);
    RunScratch rs{(DevState*)scratch, (CounterLine*)(scratch + st),
                  (unsigned int*)(scratch + st + sizeof(CounterLine) * 4 * kCounterCopies), true};
    return run_impl(g, schedule, eps, p, seed, opts, stats, rs);
}

int bp::graph_device(const bp_graph* g) { return g ? g->device : -1; }

int bp::report_error(int code, const char* msg) { return fail(code, "%s", msg); }

extern "C" {

int bp_run(bp_graph* g, int schedule, double eps, double p, uint64_t seed, const bp_run_opts* opts,
           bp_run_stats* stats) {
    if (!g) return fail(BP_EINVAL, "graph is NULL");
    const RunScratch rs{g->st(), g->ctr(), g->at<unsigned int>(g->off.ties), false};
    return run_impl(g, schedule, eps, p, seed, opts, stats, rs);
}

int bp_marginals_device(bp_graph* g, float* out_device) {
    if (!g || !out_device) return fail(BP_EINVAL, "NULL argument");
    DeviceGuard dg(g->device);
    const HostLayout& L = g->L;
    if (L.layout == kLayoutRagged) {
        EvalArgs a{};
        a.node_ptr = g->at<int>(g->off.node_ptr);
        a.rev = g->at<int>(g->off.rev);
        a.unary = g->at<float>(g->off.unary);
        a.kv = g->at<int>(g->off.kv);
        a.uoff = g->at<int>(g->off.uoff);
        a.moff = g->at<int>(g->off.moff);
        a.in_buf[0] = g->cur();
        a.num_nodes = L.N;
        HIP_OK(launch_marginals_ragged(a, out_device, g->stream), "marginals kernel");
        return BP_OK;
    }
    HIP_OK(launch_marginals(L.layout, kpad(L.K), g->at<int>(g->off.node_ptr), g->at<int>(g->off.rev),
                            g->at<float>(g->off.unary), g->cur(), out_device, L.N, L.K,
                            g->stream),
           "marginals kernel");
    return BP_OK;
}

int bp_marginals(bp_graph* g, float* out) {
    if (!g || !out) return fail(BP_EINVAL, "NULL argument");
    DeviceGuard dg(g->device);
    float* dev = g->at<float>(g->off.marg);
    int rc = bp_marginals_device(g, dev);
    if (rc != BP_OK) return rc;
    HIP_OK(hipMemcpyAsync(out, dev, sizeof(float) * (size_t)g->L.belief_floats,
                          hipMemcpyDeviceToHost, g->stream),
           "marginals readback");
    HIP_OK(hipStreamSynchronize(g->stream), "synchronize");
    return BP_OK;
}

int bp_get_state(bp_graph* g, float* msgs, bp_iter_state* st) {
    if (!g) return fail(BP_EINVAL, "graph is NULL");
    if (msgs) {
        DeviceGuard dg(g->device);
        const HostLayout& L = g->L;
        std::vector<float> dev((size_t)L.msg_floats);
        if (!dev.empty()) {
            HIP_OK(hipMemcpyAsync(dev.data(), g->cur(), sizeof(float) * dev.size(),
                                  hipMemcpyDeviceToHost, g->stream),
                   "state readback");
            HIP_OK(hipStreamSynchronize(g->stream), "synchronize");
        }
        for (long long c = 0; c < L.E; ++c) {
            const long long s = L.slot_of_canon[c];
            if (L.layout == kLayoutRagged) {
                for (long long q = 0; q < L.coff[c + 1] - L.coff[c]; ++q)
                    msgs[L.coff[c] + q] = dev[L.moff[s] + q];
            } else if (L.layout == kLayoutLogOdds) {
                const double lam = dev[s];
                msgs[2 * c + 1] = (float)(1.0 / (1.0 + std::exp(-lam)));
                msgs[2 * c + 0] = (float)(1.0 / (1.0 + std::exp(lam)));
            } else {
                for (int x = 0; x < L.K; ++x) msgs[c * L.K + x] = dev[s * L.K + x];
            }
        }
    }
    if (st) {
        st->t = g->t_next;
        st->prev_active = g->prev_active;
    }
    return BP_OK;
}

int bp_set_state(bp_graph* g, const float* msgs, const bp_iter_state* st) {
    if (!g) return fail(BP_EINVAL, "graph is NULL");
    const HostLayout& L = g->L;
    if (msgs) {
        std::vector<float> dev((size_t)L.msg_floats);
        for (long long c = 0; c < L.E; ++c) {
            const long long s = L.slot_of_canon[c];
            const bool rg = L.layout == kLayoutRagged;
            const long long c0 = rg ? L.coff[c] : c * L.K;
            const long long kc = rg ? L.coff[c + 1] - L.coff[c] : L.K;
            double z = 0.0;
            for (long long x = 0; x < kc; ++x) {
                const double v = msgs[c0 + x];
                if (!(v > 0.0) || !std::isfinite(v))
                    return fail(BP_EINVAL, "message %lld has a non-positive or non-finite entry", c);
                z += v;
            }
            if (rg) {
                for (long long x = 0; x < kc; ++x) dev[L.moff[s] + x] = (float)(msgs[c0 + x] / z);
            } else if (L.layout == kLayoutLogOdds) {
                dev[s] = (float)(std::log((double)msgs[2 * c + 1]) - std::log((double)msgs[2 * c]));
            } else {
                for (int x = 0; x < L.K; ++x) dev[s * L.K + x] = (float)(msgs[c * L.K + x] / z);
            }
        }
        DeviceGuard dg(g->device);
        if (!dev.empty()) {
            HIP_OK(hipMemcpyAsync(g->cur(), dev.data(), sizeof(float) * dev.size(),
                                  hipMemcpyHostToDevice, g->stream),
                   "state upload");
            HIP_OK(hipStreamSynchronize(g->stream), "synchronize");
        }
    }
    if (st) {
        if (st->t < 0 || st->t > 0xFFFFFFFFLL) return fail(BP_EINVAL, "t out of range");
        g->t_next = st->t;
        g->prev_active = st->prev_active;
    }
    return BP_OK;
}


// ---------------------------------------------------------------------------
// Serving: batched evaluation of many resident graphs (bp_server_*).
// ---------------------------------------------------------------------------
}  // extern "C"

namespace {

struct Request {
    int64_t id = 0;
    HostLayout L;  // built and validated at submission
    bp_request req{};
    uint64_t bytes = 0;
    enum State { kQueued, kResident, kRetired } state = kQueued;
    bp_graph* g = nullptr;
    uint64_t off = 0;  // arena offset
    int slot = -1;
    std::vector<float> marg;
    bp_run_stats stats{};
    int error = BP_OK;          // retired without a result: the admission's error
    std::string error_msg;
};

// First-fit allocator over the arena, 256-byte granules.
struct ArenaAlloc {
    std::map<uint64_t, uint64_t> free_;  // offset -> size
    void init(uint64_t bytes) {
        free_.clear();
        free_[0] = bytes & ~uint64_t(255);
    }
    bool take(uint64_t bytes, uint64_t* off) {
        bytes = (bytes + 255) & ~uint64_t(255);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            *off = it->first;
            const uint64_t rest = it->second - bytes, at = it->first + bytes;
            free_.erase(it);
            if (rest) free_[at] = rest;
            return true;
        }
        return false;
    }
    void give(uint64_t off, uint64_t bytes) {
        bytes = (bytes + 255) & ~uint64_t(255);
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
};

}  // namespace

struct bp_server {
    int device = 0;
    hipStream_t stream = nullptr;
    char* base = nullptr;
    uint64_t bytes = 0;
    bool owns = false;
    int max_graphs = 0;
    ArenaAlloc alloc;
    uint64_t graphs_off = 0;               // BatchGraph [max_graphs]
    uint64_t list_off = 0, list_cap = 0;   // int4 tile list (entries)
    std::vector<BatchGraph> rec;           // host mirror of the records
    std::vector<Request*> slots;           // resident request per slot
    std::vector<int> h_list;               // {graph, tile, oversized, 0}
    bool list_dirty = false;
    std::deque<Request*> queue;
    std::unordered_map<int64_t, Request*> reqs;
    long long launch = 0;
    int64_t next_id = 1;
    uint64_t done_off = 0;                 // unsigned [max_graphs]: gathered done flags
    unsigned int* h_done = nullptr;        // pinned mirror
    int inject_failures = 0;               // admissions still to fail (test hook)
    uint64_t ctl_off = 0;                  // BatchCtl: launch counter, list length
    uint32_t options = 0;                  // BP_SERVER_*
    int num_cus = 1;
    int grid = 0;                          // persistent blocks of the batched kernel
    long long resident_msgs = 0;           // messages of the resident graphs
    // recorded step (BP_SERVER_GRAPHS)
    hipGraphExec_t gexec = nullptr;
    int g_launches = 0, g_grid = 0;
    uint64_t g_list_off = ~0ull;
    // autotuner (BP_SERVER_AUTOTUNE): candidates of blocks per CU, timed on
    // live steps; a new round starts when the resident messages change 2x
    std::vector<int> cand;                 // blocks per launch
    std::vector<double> cand_ns;           // ns per resident message per launch
    int tune_next = -1;                    // candidate of the next step, -1 = not tuning
    int tuned = 0;
    long long tuned_msgs = 0;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
};

namespace {

int server_admit(bp_server* s) {
    while (!s->queue.empty()) {
        int slot = -1;
        for (int i = 0; i < s->max_graphs; ++i)
            if (!s->slots[i]) {
                slot = i;
                break;
            }
        if (slot < 0) return BP_OK;
        Request* r = s->queue.front();
        uint64_t off = 0;
        if (!s->alloc.take(r->bytes, &off)) return BP_OK;  // FIFO: wait for room
        bp_graph_desc d{};
        d.stream = (void*)s->stream;
        d.workspace = s->base + off;
        d.workspace_bytes = r->bytes;
        bp_graph* g = nullptr;
        const bool inject = s->inject_failures > 0;
        if (inject) --s->inject_failures;
        const int rc = create_graph_from_layout(r->L, &d, &g, inject);
        s->queue.pop_front();
        if (rc != BP_OK) {
            // the request leaves the queue with the error as its result; the
            // requests behind it are admitted as usual
            s->alloc.give(off, r->bytes);
            r->error = rc;
            r->error_msg = g_last_error;
            r->state = Request::kRetired;
            r->L = HostLayout();
            continue;
        }
        r->g = g;
        r->off = off;
        r->slot = slot;
        r->state = Request::kResident;
        s->slots[slot] = r;
        bp_run_opts o = r->req.opts;
        long long rbp_k = 0;
        BatchGraph& b = s->rec[slot];
        std::memset(&b, 0, sizeof(b));
        b.a = run_args(g, r->req.schedule, r->req.eps, r->req.p, r->req.seed, o, rbp_k);
        b.a.prev_active_host = -1;
        b.a.sel0 = 0;
        for (int i = 0; i < 4; ++i) b.msg[i] = g->msg(i >> 1, i & 1);
        b.first = s->launch;
        b.max_iters = o.max_iters;
        b.mode = r->req.schedule == BP_LBP ? kModeLBP : kModeRnBP;
        HIP_OK(hipMemcpyAsync(s->base + s->graphs_off + sizeof(BatchGraph) * (size_t)slot, &b,
                              sizeof(BatchGraph), hipMemcpyHostToDevice, s->stream),
               "batch record upload");
        const HostLayout& L = g->L;
        s->resident_msgs += L.E;
        for (int t = 0; t < (int)(L.tiles4.size() / 4); ++t)
            s->h_list.insert(s->h_list.end(), {slot, t, 0, 0});
        for (int t = 0; t < (int)(L.big4.size() / 4); ++t)
            s->h_list.insert(s->h_list.end(), {slot, t, 1, 0});
        s->list_dirty = true;
    }
    return BP_OK;
}

int server_upload_list(bp_server* s) {
    if (!s->list_dirty) return BP_OK;
    const uint64_t entries = s->h_list.size() / 4;
    if (entries > s->list_cap) {
        uint64_t cap = std::max<uint64_t>(entries, 2 * s->list_cap);
        uint64_t off = 0;
        if (!s->alloc.take(cap * 16, &off)) {
            cap = entries;
            if (!s->alloc.take(cap * 16, &off)) return fail(BP_ENOMEM, "arena full: tile list");
        }
        HIP_OK(hipStreamSynchronize(s->stream), "synchronize");  // the old list is no longer read
        if (s->list_cap) s->alloc.give(s->list_off, s->list_cap * 16);
        s->list_off = off;
        s->list_cap = cap;
    }
    if (entries)
        HIP_OK(hipMemcpyAsync(s->base + s->list_off, s->h_list.data(), entries * 16,
                              hipMemcpyHostToDevice, s->stream),
               "tile list upload");
    // the length lives in device memory, so a recorded step stays valid
    const int n_entries = (int)entries;
    HIP_OK(hipMemcpyAsync(s->base + s->ctl_off + offsetof(BatchCtl, entries), &n_entries,
                          sizeof(int), hipMemcpyHostToDevice, s->stream),
           "tile list length");
    HIP_OK(hipStreamSynchronize(s->stream), "synchronize");
    s->list_dirty = false;
    return BP_OK;
}

// Close the run of a finished graph exactly as bp_run closes its own, take its
// beliefs and statistics, and return its memory.
int server_retire(bp_server* s, Request* r) {
    bp_graph* g = r->g;
    BatchGraph& b = s->rec[r->slot];
    const long long last_it = std::min(s->launch - 1 - b.first, b.max_iters);
    EvalArgs a = b.a;
    a.t = (unsigned int)(last_it + 1);
    a.it = last_it + 1;
    a.after_final = last_it == b.max_iters ? 1 : 0;
    HIP_OK(launch_close_run(a, s->stream), "close run");
    HIP_OK(hipMemcpyAsync(g->host_state, g->st(), kStateReadback, hipMemcpyDeviceToHost, s->stream),
           "state readback");
    HIP_OK(hipStreamSynchronize(s->stream), "synchronize");
    const DevState& st = *g->host_state;
    const bool converged = st.done != 0;
    const long long final_t = converged ? st.conv_t : st.last_t;
    g->cur_pair = (int)(final_t & 1);
    g->cur_sel = (int)st.in_sel[final_t & 3];
    r->marg.resize((size_t)g->L.N * g->L.K);
    int rc = bp_marginals(g, r->marg.data());
    if (rc != BP_OK) return rc;
    std::memset(&r->stats, 0, sizeof(r->stats));
    r->stats.iterations = (long long)st.iterations;
    r->stats.converged = converged ? 1 : 0;
    r->stats.last_active = (long long)st.last_active;
    float rm;
    std::memcpy(&rm, &st.last_rmax, sizeof(rm));
    r->stats.last_max_residual = rm;
    r->stats.evaluated = (long long)st.evaluated;
    r->stats.committed = (long long)st.committed;
    r->stats.final_t = final_t;
    s->resident_msgs -= g->L.E;
    bp_destroy_graph(g);
    r->g = nullptr;
    s->alloc.give(r->off, r->bytes);
    s->slots[r->slot] = nullptr;
    r->slot = -1;
    r->state = Request::kRetired;
    return BP_OK;
}

}  // namespace

extern "C" {

int bp_server_create(const bp_server_desc* d, bp_server** out) {
    if (!out) return fail(BP_EINVAL, "out is NULL");
    *out = nullptr;
    if (!d) return fail(BP_EINVAL, "desc is NULL");
    if (d->max_graphs < 1 || d->max_graphs > 65536)
        return fail(BP_EINVAL, "max_graphs %d not in [1, 65536]", d->max_graphs);
    const uint64_t rec_bytes = ((sizeof(BatchGraph) * (uint64_t)d->max_graphs) + 255) & ~uint64_t(255);
    if (d->arena_bytes <= rec_bytes) return fail(BP_EINVAL, "arena_bytes too small");
    if (d->arena && (uintptr_t)d->arena % 256 != 0)
        return fail(BP_EINVAL, "arena must be 256-byte aligned");
    bp_server* s = new (std::nothrow) bp_server();
    if (!s) return fail(BP_ENOMEM, "host allocation failed");
    hipError_t e = hipGetDevice(&s->device);
    if (e != hipSuccess) {
        delete s;
        return hip_fail(e, "hipGetDevice");
    }
    if (d->options & ~(uint32_t)(BP_SERVER_GRAPHS | BP_SERVER_AUTOTUNE)) {
        delete s;
        return fail(BP_EINVAL, "unknown server options");
    }
    s->stream = (hipStream_t)d->stream;
    s->bytes = d->arena_bytes;
    s->max_graphs = d->max_graphs;
    s->options = d->options;
    if (d->arena) {
        s->base = (char*)d->arena;
    } else {
        e = hipMalloc((void**)&s->base, d->arena_bytes);
        if (e != hipSuccess) {
            delete s;
            (void)hipGetLastError();
            return fail(e == hipErrorOutOfMemory ? BP_ENOMEM : BP_EDEVICE, "hipMalloc(%llu): %s",
                        (unsigned long long)d->arena_bytes, hipGetErrorString(e));
        }
        s->owns = true;
    }
    s->alloc.init(s->bytes);
    s->alloc.take(rec_bytes, &s->graphs_off);
    if (!s->alloc.take(sizeof(unsigned int) * (uint64_t)s->max_graphs, &s->done_off) ||
        !s->alloc.take(sizeof(BatchCtl), &s->ctl_off)) {
        bp_server_destroy(s);
        return fail(BP_EINVAL, "arena_bytes too small");
    }
    e = hipDeviceGetAttribute(&s->num_cus, hipDeviceAttributeMultiprocessorCount, s->device);
    if (e != hipSuccess || s->num_cus < 1) s->num_cus = 1;
    // persistent grid: 4 blocks per compute unit unless the autotuner chooses
    s->grid = 4 * s->num_cus;
    for (int c : {1, 2, 4, 8}) s->cand.push_back(c * s->num_cus);
    s->cand_ns.assign(s->cand.size(), 0.0);
    if (s->options & BP_SERVER_AUTOTUNE) {
        if (hipEventCreate(&s->ev0) != hipSuccess || hipEventCreate(&s->ev1) != hipSuccess) {
            bp_server_destroy(s);
            return fail(BP_EDEVICE, "hipEventCreate");
        }
    }
    e = hipHostMalloc((void**)&s->h_done, sizeof(unsigned int) * (size_t)s->max_graphs,
                      hipHostMallocDefault);
    if (e != hipSuccess) {
        bp_server_destroy(s);
        return hip_fail(e, "hipHostMalloc");
    }
    // empty slots: null state pointers (the status kernel reads every slot);
    // launch counter 0, empty list
    e = hipMemsetAsync(s->base + s->graphs_off, 0, rec_bytes, s->stream);
    if (e == hipSuccess) e = hipMemsetAsync(s->base + s->ctl_off, 0, sizeof(BatchCtl), s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) {
        bp_server_destroy(s);
        return hip_fail(e, "initialise");
    }
    s->rec.resize((size_t)s->max_graphs);
    s->slots.assign((size_t)s->max_graphs, nullptr);
    *out = s;
    return BP_OK;
}

int bp_server_submit(bp_server* s, const bp_graph_desc* graph, const bp_request* req, int64_t* id) {
    if (!s || !graph || !req) return fail(BP_EINVAL, "NULL argument");
    if (graph->pair_kind != BP_PAIR_ISING || graph->num_states != 2 || graph->flags != 0)
        return fail(BP_EINVAL, "serving takes K = 2 Ising graphs in the log-odds layout");
    if (req->schedule != BP_LBP && req->schedule != BP_RNBP)
        return fail(BP_EINVAL, "serving takes BP_LBP or BP_RNBP");
    if (!(req->eps >= 0.0) || !std::isfinite(req->eps)) return fail(BP_EINVAL, "eps must be finite and >= 0");
    if (req->schedule == BP_RNBP && !(req->p > 0.0 && req->p <= 1.0)) return fail(BP_EINVAL, "p must be in (0, 1]");
    const bp_run_opts& o = req->opts;
    if (o.max_iters < 0) return fail(BP_EINVAL, "max_iters < 0");
    if (o.max_iters + 1 > 0xFFFFFFFFLL) return fail(BP_EINVAL, "max_iters too large");
    if (req->schedule == BP_RNBP && o.dynamic_p && !(o.high_p > 0.0 && o.high_p <= 1.0))
        return fail(BP_EINVAL, "high_p must be in (0, 1]");
    if (!std::isfinite(o.ratio_threshold)) return fail(BP_EINVAL, "ratio_threshold not finite");
    if (o.sparse) return fail(BP_EINVAL, "serving runs the full evaluation (opts.sparse must be 0)");
    HostLayout L;
    int rc = build_layout(graph, L);  // full validation
    if (rc != BP_OK) return rc;
    if (L.layout != kLayoutLogOdds) return fail(BP_EINVAL, "graph too large for the log-odds layout");
    const uint64_t need = plan(L).total;
    if (need + 256 > s->bytes) return fail(BP_ENOMEM, "graph needs %llu bytes, arena has %llu",
                                           (unsigned long long)need, (unsigned long long)s->bytes);
    Request* r = new (std::nothrow) Request();
    if (!r) return fail(BP_ENOMEM, "host allocation failed");
    r->L = std::move(L);
    r->req = *req;
    r->bytes = need;
    r->id = s->next_id++;
    s->queue.push_back(r);
    s->reqs[r->id] = r;
    if (id) *id = r->id;
    return BP_OK;
}

int bp_server_step(bp_server* s, int32_t launches, int32_t* finished) {
    if (finished) *finished = 0;
    if (!s) return fail(BP_EINVAL, "server is NULL");
    if (launches < 0) return fail(BP_EINVAL, "launches < 0");
    DeviceGuard dg(s->device);
    int rc = server_admit(s);
    if (rc != BP_OK) return rc;
    rc = server_upload_list(s);
    if (rc != BP_OK) return rc;
    const int blocks = (int)(s->h_list.size() / 4);
    BatchGraph* graphs = (BatchGraph*)(s->base + s->graphs_off);
    const int* list = (const int*)(s->base + s->list_off);
    BatchCtl* ctl = (BatchCtl*)(s->base + s->ctl_off);
    // autotuner: a new round when the resident work changed by 2x
    const bool tune = (s->options & BP_SERVER_AUTOTUNE) && blocks > 0 && launches > 0;
    if (tune && s->tune_next < 0 &&
        (!s->tuned || s->resident_msgs > 2 * s->tuned_msgs || 2 * s->resident_msgs < s->tuned_msgs))
        s->tune_next = 0;
    const int tuning = tune ? s->tune_next : -1;
    const int grid = tuning >= 0 ? s->cand[tuning] : s->grid;
    if (blocks > 0 && launches > 0) {
        if (tuning >= 0) HIP_OK(hipEventRecord(s->ev0, s->stream), "event record");
        if (s->options & BP_SERVER_GRAPHS) {
            if (!s->gexec || s->g_launches != launches || s->g_grid != grid ||
                s->g_list_off != s->list_off) {
                if (s->gexec) (void)hipGraphExecDestroy(s->gexec);
                s->gexec = nullptr;
                hipGraph_t gr = nullptr;
                HIP_OK(batch_graph_nodes(graphs, s->max_graphs, list, ctl, grid, launches, &gr),
                       "record batched launches");
                hipError_t e = hipGraphInstantiate(&s->gexec, gr, nullptr, nullptr, 0);
                (void)hipGraphDestroy(gr);
                if (e != hipSuccess) {
                    s->gexec = nullptr;
                    return hip_fail(e, "hipGraphInstantiate");
                }
                s->g_launches = launches;
                s->g_grid = grid;
                s->g_list_off = s->list_off;
            }
            HIP_OK(hipGraphLaunch(s->gexec, s->stream), "replay batched launches");
        } else {
            for (int k = 0; k < launches; ++k)
                HIP_OK(launch_eval_batch(graphs, s->max_graphs, list, ctl, grid, s->stream),
                       "batch evaluation");
        }
        if (tuning >= 0) HIP_OK(hipEventRecord(s->ev1, s->stream), "event record");
        // the device counter advanced once per launch; with nothing resident
        // neither moves
        s->launch += launches;
    }
    // poll every resident graph (one gathered readback of the done flags),
    // retire the finished ones
    int n = 0;
    unsigned int* d_done = (unsigned int*)(s->base + s->done_off);
    HIP_OK(launch_batch_status(graphs, s->max_graphs, d_done, s->stream), "batch status");
    HIP_OK(hipMemcpyAsync(s->h_done, d_done, sizeof(unsigned int) * (size_t)s->max_graphs,
                          hipMemcpyDeviceToHost, s->stream),
           "status readback");
    HIP_OK(hipStreamSynchronize(s->stream), "synchronize");
    if (tuning >= 0) {
        float ms = 0.0f;
        HIP_OK(hipEventElapsedTime(&ms, s->ev0, s->ev1), "event time");
        s->cand_ns[tuning] = (double)ms * 1e6 / ((double)std::max(1ll, s->resident_msgs) * launches);
        s->tune_next = tuning + 1;
        if (s->tune_next == (int)s->cand.size()) {
            int best = 0;
            for (int i = 1; i < (int)s->cand.size(); ++i)
                if (s->cand_ns[i] < s->cand_ns[best]) best = i;
            s->grid = s->cand[best];
            s->tuned = 1;
            s->tuned_msgs = s->resident_msgs;
            s->tune_next = -1;
        }
    }
    bool removed = false;
    for (Request* r : s->slots) {
        if (!r || !r->g) continue;
        const BatchGraph& b = s->rec[r->slot];
        const long long last_it = s->launch - 1 - b.first;
        if (s->h_done[r->slot] || last_it >= b.max_iters) {
            rc = server_retire(s, r);
            if (rc != BP_OK) return rc;
            ++n;
            removed = true;
        }
    }
    if (removed) {
        std::vector<int> keep;
        keep.reserve(s->h_list.size());
        for (size_t i = 0; i < s->h_list.size(); i += 4)
            if (s->slots[s->h_list[i]])
                keep.insert(keep.end(), s->h_list.begin() + i, s->h_list.begin() + i + 4);
        s->h_list.swap(keep);
        s->list_dirty = true;
    }
    if (finished) *finished = n;
    return BP_OK;
}

int bp_server_result(bp_server* s, int64_t id, float* marginals, bp_run_stats* stats) {
    if (!s) return fail(BP_EINVAL, "server is NULL");
    auto it = s->reqs.find(id);
    if (it == s->reqs.end()) return fail(BP_EINVAL, "unknown request %lld", (long long)id);
    Request* r = it->second;
    if (r->state != Request::kRetired) return BP_ESTATE;
    if (r->error != BP_OK) {
        const int code = r->error;
        fail(code, "request %lld was not admitted: %s", (long long)id, r->error_msg.c_str());
        s->reqs.erase(it);
        delete r;
        return code;
    }
    if (marginals) std::memcpy(marginals, r->marg.data(), sizeof(float) * r->marg.size());
    if (stats) *stats = r->stats;
    s->reqs.erase(it);
    delete r;
    return BP_OK;
}

int bp_server_counts(const bp_server* s, int64_t* queued, int64_t* resident, int64_t* retired) {
    if (!s) return fail(BP_EINVAL, "server is NULL");
    int64_t q = 0, a = 0, d = 0;
    for (const auto& kv : s->reqs) {
        if (kv.second->state == Request::kQueued) ++q;
        else if (kv.second->state == Request::kResident) ++a;
        else ++d;
    }
    if (queued) *queued = q;
    if (resident) *resident = a;
    if (retired) *retired = d;
    return BP_OK;
}

int bp_server_inject_failures(bp_server* s, int32_t admissions) {
    if (!s) return fail(BP_EINVAL, "server is NULL");
    if (admissions < 0) return fail(BP_EINVAL, "admissions < 0");
    s->inject_failures = admissions;
    return BP_OK;
}

void bp_server_destroy(bp_server* s) {
    if (!s) return;
    {
        DeviceGuard dg(s->device);
        (void)hipStreamSynchronize(s->stream);
        for (auto& kv : s->reqs) {
            if (kv.second->g) bp_destroy_graph(kv.second->g);
            delete kv.second;
        }
        if (s->gexec) (void)hipGraphExecDestroy(s->gexec);
        if (s->ev0) (void)hipEventDestroy(s->ev0);
        if (s->ev1) (void)hipEventDestroy(s->ev1);
        if (s->owns && s->base) (void)hipFree(s->base);
        if (s->h_done) (void)hipHostFree(s->h_done);
    }
    delete s;
}

int bp_server_config(const bp_server* s, int32_t* grid_blocks, int32_t* tuned,
                     int32_t* cand_blocks, double* cand_ns_per_msg, int32_t max_entries,
                     int32_t* entries) {
    if (!s) return fail(BP_EINVAL, "server is NULL");
    if (grid_blocks) *grid_blocks = s->grid;
    if (tuned) *tuned = s->tuned;
    const int n = std::min<int>((int)s->cand.size(), std::max(0, max_entries));
    for (int i = 0; i < n; ++i) {
        if (cand_blocks) cand_blocks[i] = s->cand[i];
        if (cand_ns_per_msg) cand_ns_per_msg[i] = s->cand_ns[i];
    }
    if (entries) *entries = n;
    return BP_OK;
}

}  // extern "C"
