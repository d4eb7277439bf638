// HIP kernels of libbp for gfx950 (CDNA4, wave64).
//
// One iteration of Alg. 1 is one launch of an evaluation kernel (plus the top-k
// selection kernels for frontier residual BP).
//
// Evaluation kernel (Eq. (2) + Eq. (4) + frontier rule + commit, fused):
// messages are stored grouped by source node (CSR by source), so slot e holds
// m_{i->k}, the message the thread of slot e recomputes, and the outgoing
// messages of a run of source nodes form one contiguous slot range.  A block
// owns such a tile of nodes:
//   phase 1  coalesced loads of the tile's own slots (old value, reverse index,
//            coupling, target id) and of the incoming messages m_{k->i} at the
//            reverse slots (the one gather per message);
//   phase 2  one thread per node (per node-state for K > 2) sums the incoming
//            logs with the log unary into A_i = log psi_i + sum_k log m_{k->i};
//   phase 3  one thread per slot computes m_{i->k} from the cavity
//            A_i - log m_{k->i} (Eq. (2) excludes exactly that message),
//            normalises it, forms the L-infinity residual against the old value,
//            applies the frontier rule and writes the next buffer at its own
//            slot (coalesced).
// Every slot of the next buffer is written exactly once per iteration, so the
// update is synchronous (Jacobi) with no atomics on message values.
//
// Randomized BP chooses p_t from n_t, which is only known once every block of
// iteration t has counted its residuals.  The kernel therefore writes the
// committed state under both keep thresholds (two output buffers); the next
// launch computes p_t from the finished counters in its prologue and reads the
// matching buffer.  No pass over the messages is needed between iterations.
#include "bp_internal.h"

namespace bp {
namespace {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).  The random filter of
// Sec. IV-A for the message i -> j, j the neighbour of rank r of i (slots of a
// source are ordered by target, so r is the slot's offset in the source's
// range), uses word r mod 4 of the output for counter (i, r div 4, t, 0): one
// call serves four messages of one source.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint4 philox4(unsigned int c0, unsigned int c1, unsigned int c2,
                                         unsigned int k0, unsigned int k1) {
    unsigned int c3 = 0u;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        // full 64-bit products: one v_mad_u64_u32 each instead of a hi/lo pair
        const unsigned long long p0 = (unsigned long long)0xD2511F53u * c0;
        const unsigned long long p1 = (unsigned long long)0xCD9E8D57u * c2;
        const unsigned int n0 = (unsigned int)(p1 >> 32) ^ c1 ^ k0;
        const unsigned int n2 = (unsigned int)(p0 >> 32) ^ c3 ^ k1;
        c0 = n0;
        c1 = (unsigned int)p1;
        c2 = n2;
        c3 = (unsigned int)p0;
    }
    return make_uint4(c0, c1, c2, c3);
}

// The 24-bit uniform of the message of rank r of source i at iteration t.
__device__ __forceinline__ unsigned int draw24(const EvalArgs& a, int i, int r) {
    const uint4 w = philox4((unsigned int)i, (unsigned int)r >> 2, a.t, a.key0, a.key1);
    const int k = r & 3;
    const unsigned int x = k == 0 ? w.x : k == 1 ? w.y : k == 2 ? w.z : w.w;
    return x >> 8;
}

// Hardware exp2 / log2 / reciprocal (v_exp_f32, v_log_f32, v_rcp_f32, about 1 ulp)
// where the argument range needs none of the library's fix-ups: exp2 may
// underflow to zero or overflow to +inf, both harmless where it is used below;
// log2 is only taken of values in [1, 2]; rcp only of values in [1, +inf].
__device__ __forceinline__ float exp2_hw(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ float log2_hw(float x) { return __builtin_amdgcn_logf(x); }
__device__ __forceinline__ float rcp_hw(float x) { return __builtin_amdgcn_rcpf(x); }

constexpr float kLog2e = 1.4426950408889634f;
constexpr float kLn2 = 0.6931471805599453f;

// 1 / (1 + e^{-x}); e^{-x} overflows to +inf for x < -88 and gives 0.
__device__ __forceinline__ float sigmoid_fast(float x) {
    return rcp_hw(1.0f + exp2_hw(-kLog2e * x));
}

// Workgroup barrier for LDS hand-offs only: waits for this wave's LDS
// operations and meets the other waves, without the release/acquire fences of
// __syncthreads(), which would also wait for every outstanding global load
// (the prefetched next tile).  No global memory written in a launch is read
// back by another wave of the same block.
__device__ __forceinline__ void lds_barrier() {
    __asm__ volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

struct RedScratch {
    float rmax[kBlock / 64];
    unsigned int act[kBlock / 64];
    unsigned int sa[kBlock / 64];
    unsigned int sb[kBlock / 64];
};

// Block-wide reduction of the per-thread residual max and counts, then one
// atomic per quantity per block into the block's counter copy (integer adds and
// an ordered max on the FP32 bit pattern of a non-negative float: both order
// independent, so the totals are deterministic).
__device__ __forceinline__ void block_accumulate(RedScratch* red, CounterLine* ctr, unsigned int t,
                                                 float rmax, unsigned int act, unsigned int sa,
                                                 unsigned int sb) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        rmax = fmaxf(rmax, __shfl_xor(rmax, o, 64));
        act += __shfl_xor(act, o, 64);
        sa += __shfl_xor(sa, o, 64);
        sb += __shfl_xor(sb, o, 64);
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red->rmax[w] = rmax;
        red->act[w] = act;
        red->sa[w] = sa;
        red->sb[w] = sb;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        float r = red->rmax[0];
        unsigned int A = red->act[0], SA = red->sa[0], SB = red->sb[0];
        for (int i = 1; i < (int)(blockDim.x >> 6); ++i) {
            r = fmaxf(r, red->rmax[i]);
            A += red->act[i];
            SA += red->sa[i];
            SB += red->sb[i];
        }
        CounterLine* c = ctr + (t & 3u) * kCounterCopies + (blockIdx.x & (kCounterCopies - 1));
        if (A) atomicAdd(&c->active, (unsigned long long)A);
        if (SA) atomicAdd(&c->sel_a, (unsigned long long)SA);
        if (SB) atomicAdd(&c->sel_b, (unsigned long long)SB);
        if (r > 0.0f) atomicMax(&c->rmax, __float_as_uint(r));
    }
}

__device__ __forceinline__ int tile_of_block(const EvalArgs& a) {
    // Workgroups are dealt to the 8 XCDs round-robin; give each XCD a contiguous
    // range of tiles so neighbouring tiles share that XCD's L2.
    const int b = blockIdx.x;
    return (b & 7) * a.tiles_per_xcd + (b >> 3);
}

__device__ __forceinline__ unsigned long long wave_sum64(unsigned long long v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ unsigned int wave_max32(unsigned int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, (unsigned int)__shfl_xor((int)v, o, 64));
    return v;
}

// Which of the two committed outcomes iteration t - 1 kept: p_{t-1} is the low
// setting when EdgeRatio = n_{t-1} / n_{t-2} exceeds the threshold (Sec. IV-A).
__device__ __forceinline__ int select_outcome(const EvalArgs& a, unsigned long long n1, long long n2) {
    if (a.sched != kModeRnBP || !a.two_outputs) return 0;
    const bool p_low = !a.dynamic_p || (n2 > 0 && ((double)n1 / (double)n2 > a.ratio_threshold));
    return (p_low == (a.low_is_a != 0)) ? 0 : 1;
}

// The counter lines the prologue needs, loaded by the 64 lanes of one wave
// (lane c reads copy c): n of iterations t - 1 and t - 2, and for the block that
// closes iteration t - 1 also its frontier sizes and max residual.
struct CtrLoad {
    unsigned long long n1, n2, sa, sb;
    unsigned int rm, done;
};

__device__ __forceinline__ void ctr_load(const EvalArgs& a, bool lead, CtrLoad& c) {
    const int lane = threadIdx.x & 63;
    const CounterLine* c1 = a.ctr + ((a.t - 1u) & 3u) * kCounterCopies + lane;
    c.done = a.st->done;
    c.n1 = c1->active;
    c.n2 = a.it >= 2 ? a.ctr[((a.t - 2u) & 3u) * kCounterCopies + lane].active : 0ull;
    c.sa = lead ? c1->sel_a : 0ull;
    c.sb = lead ? c1->sel_b : 0ull;
    c.rm = lead ? c1->rmax : 0u;
}

// Run by the 64 lanes of one wave after ctr_load: sum the counter copies of
// iteration t - 1 (and t - 2), and, when `close` is set, record iteration
// t - 1 (IsConverged, statistics, the buffer p_{t-1} selects) and clear the
// copies of t + 1.  The statistics are updated with stores and no-return
// atomics, so nothing waits.  Returns n_{t-1} and n_{t-2} (the host's value
// when t - 2 precedes the run).
__device__ void wave_close(const EvalArgs& a, bool close, const CtrLoad& c,
                           unsigned long long& n1_out, long long& n2_out) {
    const int lane = threadIdx.x & 63;
    const unsigned long long n1 = wave_sum64(c.n1);
    const unsigned long long n2 = wave_sum64(c.n2);
    const long long n2s = a.it >= 2 ? (long long)n2 : a.prev_active_host;
    n1_out = n1;
    n2_out = n2s;
    if (!close) return;
    const unsigned long long sa = wave_sum64(c.sa);
    const unsigned long long sb = wave_sum64(c.sb);
    const unsigned int rm = wave_max32(c.rm);
    CounterLine* z = a.ctr + ((a.t + 1u) & 3u) * kCounterCopies + lane;
    z->active = 0ull;
    z->sel_a = 0ull;
    z->sel_b = 0ull;
    z->rmax = 0u;
    if (lane != 0) return;
    DevState* st = a.st;
    const unsigned int tp = a.t - 1u;
    const int sel = select_outcome(a, n1, n2s);
    atomicAdd(&st->evaluated, a.num_messages);
    atomicAdd(&st->evals, 1ull);
    st->last_t = (long long)tp;
    st->last_active = n1;
    st->last_rmax = rm;
    st->last_prev = n2s;
    if (n1 == 0ull) {
        st->done = 1u;
        st->conv_t = (long long)tp;
    } else if (!a.after_final) {
        unsigned long long cm;
        if (a.sched == kModeLBP)
            cm = a.num_messages;
        else if (a.sched == kModeRBP)
            cm = a.rbp_k;
        else if (a.sched == kModeRS)
            cm = 0ull;  // the splash kernels count their commits
        else
            cm = sel ? sb : sa;
        if (cm) atomicAdd(&st->committed, cm);
        atomicAdd(&st->iterations, 1ull);
        st->in_sel[a.t & 3u] = (unsigned int)sel;
    }
}

// Start of iteration t, in two parts so that a kernel can issue other loads
// between them: prologue_issue loads the counters (wave 0), prologue_finish
// (all threads of the block) returns the buffer holding m^t, or nullptr when
// an earlier evaluation found no residual above eps (the block then exits).
// The previous launch wrote the outcome under both keep thresholds, so
// choosing p_{t-1} is choosing a buffer.  The lead block (one per graph and
// launch) also closes iteration t - 1.
__device__ __forceinline__ void prologue_issue(const EvalArgs& a, CtrLoad& c, bool lead) {
    if (a.it != 0 && threadIdx.x < 64) ctr_load(a, lead, c);
}

__device__ __forceinline__ const float* prologue_finish(const EvalArgs& a, const CtrLoad& c,
                                                        unsigned long long* s_red,
                                                        bool lead) {
    if (a.it == 0) {
        if (lead && threadIdx.x < 64) {
            CounterLine* z = a.ctr + ((a.t + 1u) & 3u) * kCounterCopies + threadIdx.x;
            z->active = 0ull;
            z->sel_a = 0ull;
            z->sel_b = 0ull;
            z->rmax = 0u;
            if (threadIdx.x == 0) a.st->in_sel[a.t & 3u] = (unsigned int)a.sel0;
        }
        return a.in_buf[0];
    }
    if (threadIdx.x < 64) {
        unsigned long long n1;
        long long n2;
        wave_close(a, lead && !c.done, c, n1, n2);
        if (threadIdx.x == 0) {
            s_red[0] = c.done ? 0ull : n1;
            s_red[1] = (unsigned long long)n2;
        }
    }
    lds_barrier();
    const unsigned long long n1 = s_red[0];
    if (n1 == 0ull) return nullptr;
    return a.in_buf[select_outcome(a, n1, (long long)s_red[1])];
}

__device__ __forceinline__ const float* iteration_prologue(const EvalArgs& a,
                                                           unsigned long long* s_red, bool lead) {
    CtrLoad c;
    prologue_issue(a, c, lead);
    return prologue_finish(a, c, s_red, lead);
}

// ---------------------------------------------------------------------------
// K = 2 Ising, one log-odds value per message: lambda = log(m(1) / m(0)).
// Aggregate L_i = u_i + sum_k lambda_{k->i} with u_i = log psi_i(1) - log psi_i(0).
// With H = (L_i - lambda_{k->i}) / 2 the outgoing message of Eq. (2) for
// psi = exp(J s_i s_k) has log-odds log cosh(J + H) - log cosh(J - H) (the sum
// over x_i in closed form; normalisation included).
// The slot e of m_{i->k} gives e as the output index, its own old value, and
// lambda_{k->i} at rev[e].
// ---------------------------------------------------------------------------
// log(1 + e^{-2|x|}), in (0, log 2]: log2 is taken of a value in (1, 2].
__device__ __forceinline__ float logcosh_tail(float x) {
    return kLn2 * log2_hw(1.0f + exp2_hw(-2.0f * kLog2e * fabsf(x)));
}

// Array access with a 32-bit byte offset from a wave-uniform base: the
// compiler emits the global_load/store form that adds a 32-bit VGPR offset to a
// 64-bit SGPR base, so per-lane accesses need no 64-bit address arithmetic.
// Every array the K = 2 kernel touches holds fewer than 2^30 four-byte elements
// (checked at graph creation).
template <class T>
__device__ __forceinline__ T ld32(const T* base, int i) {
    return *(const T*)((const char*)base + (unsigned int)i * 4u);
}
template <class T>
__device__ __forceinline__ void st32(T* base, int i, T v) {
    *(T*)((char*)base + (unsigned int)i * 4u) = v;
}
// A pointer the compiler cannot prove uniform (chosen from LDS data), made uniform.
template <class T>
__device__ __forceinline__ T* uniform_ptr(T* p) {
    const unsigned long long v = (unsigned long long)p;
    const unsigned int lo = __builtin_amdgcn_readfirstlane((unsigned int)v);
    const unsigned int hi = __builtin_amdgcn_readfirstlane((unsigned int)(v >> 32));
    return (T*)(((unsigned long long)hi << 32) | lo);
}

// Where one slot's results go: plain pointers, or buffer resources.
struct OutPtr {
    const EvalArgs& a;
    __device__ void out0(int e, float v) const { a.out_buf[0][e] = v; }
    __device__ void out1(int e, float v) const { a.out_buf[1][e] = v; }
    __device__ void cand(int e, float v) const { a.cand[e] = v; }
    __device__ void key(int e, float r) const { a.keys[e] = __float_as_uint(r); }
};
struct OutOff {
    float* o0;
    float* o1;
    float* c;
    unsigned int* k;
    __device__ void out0(int e, float v) const { st32(o0, e, v); }
    __device__ void out1(int e, float v) const { st32(o1, e, v); }
    __device__ void cand(int e, float v) const { st32(c, e, v); }
    __device__ void key(int e, float r) const { st32(k, e, __float_as_uint(r)); }
};

// Eq. (2), Eq. (4) and the frontier rule for one slot; returns the residual.
// log cosh(J + H) - log cosh(J - H) is evaluated as
// 2 sgn(J H) min(|J|, |H|) + tail(J + H) - tail(J - H): the identity
// |J + H| - |J - H| = 2 sgn(J H) min(|J|, |H|) keeps it exact in the leading term
// for any finite J and H (no cancellation of two large magnitudes, no overflow),
// and the tails are bounded by log 2.
__device__ __forceinline__ float logodds_update(float L, float lam_in, float J) {
    const float H = 0.5f * (L - lam_in);
    const float lead = copysignf(2.0f * fminf(fabsf(J), fabsf(H)), J * H);
    return lead + logcosh_tail(J + H) - logcosh_tail(J - H);
}

template <int MODE, class Out>
__device__ __forceinline__ float logodds_slot(const EvalArgs& a, const Out& out, float L,
                                              float lam_in, float J, float lam_old, int e,
                                              unsigned int u24, unsigned int& act,
                                              unsigned int& sa, unsigned int& sb) {
    const float lam_new = logodds_update(L, lam_in, J);
    const float r = fabsf(sigmoid_fast(lam_new) - sigmoid_fast(lam_old));
    const bool active = r > a.eps;
    act += active;
    if (MODE == kModeLBP) {
        out.out0(e, lam_new);
    } else if (MODE == kModeRnBP) {
        bool ka = false, kb = false;
        if (active) {
            ka = u24 < a.thr_a;
            kb = u24 < a.thr_b;
        }
        sa += ka;
        sb += kb;
        out.out0(e, ka ? lam_new : lam_old);
        if (a.two_outputs) out.out1(e, kb ? lam_new : lam_old);
    } else if (MODE == kModeRBP) {
        out.cand(e, lam_new);
        out.key(e, r);
    }
    return r;
}

constexpr int kPP = kTileSlotsLogOdds / kBlockLO;              // slots per thread per tile
constexpr int kPJ = (kTileNodesLogOdds + kBlockLO) / kBlockLO;    // node entries (TN + 1) per thread

// The per-thread share of one tile: node bounds and unaries, and the slots'
// own old values, reverse indices and couplings.
struct TileRegs {
    int n0, nn, s0, ns;
    int ptr[kPJ];
    float u[kPJ];
    float old[kPP];
    int rev[kPP];
    float J[kPP];
};

// Issue every load of a tile (indices clamped into the tile, so there is no
// per-lane branch and the loads are not ordered behind one another): the graph
// constants, then the tile's own old messages.  R16: the reverse slots are
// read as 16-bit offsets from the slot (EvalArgs.rev16).
template <class T>
__device__ __forceinline__ T ld16(const T* base, int i) {
    return *(const T*)((const char*)base + (unsigned int)i * 2u);
}
template <int MODE, bool R16 = false>
__device__ __forceinline__ void tile_load_const(TileRegs& d, const EvalArgs& a, int4 b) {
    const int tid = threadIdx.x;
    d.n0 = b.x;
    d.nn = b.y - b.x;
    d.s0 = b.z;
    d.ns = b.w - b.z;
#pragma unroll
    for (int j = 0; j < kPJ; ++j) {
        const int v = tid + j * kBlockLO;
        d.ptr[j] = ld32(a.node_ptr, d.n0 + min(v, d.nn));
        d.u[j] = ld32(a.unary, d.n0 + min(v, max(d.nn - 1, 0)));
    }
    // a tile without slots reads slot s0, which lies inside the graph's
    // device arena (the arrays are carved from one allocation in sequence)
#pragma unroll
    for (int k = 0; k < kPP; ++k) {
        const int s = d.s0 + min(tid + k * kBlockLO, max(d.ns - 1, 0));
        d.rev[k] = R16 ? s + (int)ld16(a.rev16, s) : ld32(a.rev, s);
        d.J[k] = ld32(a.coupling, s);
    }
}

__device__ __forceinline__ void tile_load_msgs(TileRegs& d, const float* m_in) {
#pragma unroll
    for (int k = 0; k < kPP; ++k)
        d.old[k] = ld32(m_in, d.s0 + min((int)threadIdx.x + k * kBlockLO, max(d.ns - 1, 0)));
}

template <int MODE, bool R16 = false>
__device__ __forceinline__ void tile_load(TileRegs& d, const EvalArgs& a, const float* m_in,
                                          int4 b) {
    tile_load_const<MODE, R16>(d, a, b);
    tile_load_msgs(d, m_in);
}

// Tile w + j * W of this block's XCD range (tiles are dealt to XCDs in
// contiguous ranges so that neighbouring tiles share an L2), or -1.
__device__ __forceinline__ int block_tile(const EvalArgs& a, int j) {
    const int w = (int)(blockIdx.x >> 3) + j * (int)(gridDim.x >> 3);
    if (w >= a.tiles_per_xcd) return -1;
    const int t = (int)(blockIdx.x & 7) * a.tiles_per_xcd + w;
    return t < a.num_tiles ? t : -1;
}

// Add 1 to LDS bin `bin` for every lane with `on`.  Residual keys share
// their leading digits, so most lanes of a wave hit one bin: the lanes whose
// bin equals the first active lane's are counted by a ballot and one atomic,
// the rest add individually.
__device__ __forceinline__ void lds_count(unsigned int* h, unsigned int bin, bool on) {
    const unsigned long long act = __ballot(on);
    if (!act) return;
    const int lead = __ffsll((long long)act) - 1;
    const unsigned int lb = (unsigned int)__shfl((int)bin, lead, 64);
    const bool same = on && bin == lb;
    const unsigned long long sm = __ballot(same);
    if ((int)(threadIdx.x & 63) == lead) atomicAdd(&h[lb], (unsigned int)__popcll(sm));
    if (on && !same) atomicAdd(&h[bin], 1u);
}

// LDS of the K = 2 tile loop.
struct LogoddsLds {
    float lam[kTileSlotsLogOdds];
    unsigned short owner[kTileSlotsLogOdds];
    unsigned int u[kTileSlotsLogOdds];  // 24-bit uniforms of the slots (RnBP)
    unsigned short ptr[kTileNodesLogOdds + 1];
    float L[kTileNodesLogOdds];
    unsigned int hist[256];             // frontier RBP: first radix digit of the keys
};

// The software-pipelined tile loop of the K = 2 kernel over a sequence of
// tiles (seq.valid(j), seq.bounds(j)): while tile j is computed, the loads of
// tile j + 1 are in flight, so the math of Eq. (2), the residual and the random
// filter overlap the memory traffic instead of following it.  `cur` holds the
// graph constants of tile 0 (issued by the caller); iteration j issues the
// loads of tile j + 1, aggregates tile j (LDS), issues the gathers of tile
// j + 1, computes and stores tile j, then stages tile j + 1 into LDS, so every
// wait falls on loads that had a whole phase to complete.
template <int MODE, class Seq, bool R16 = false>
__device__ __forceinline__ void logodds_tile_loop(const EvalArgs& a, const float* __restrict__ m_in,
                                                  const Seq& seq, TileRegs& cur, int4 bnext,
                                                  LogoddsLds& l, float& rmax, unsigned int& act,
                                                  unsigned int& sa, unsigned int& sb) {
    const OutOff out{a.out_buf[0], a.out_buf[1], a.cand, a.keys};
    const int tid = threadIdx.x;
    TileRegs nxt;
    float lin[kPP];
    tile_load_msgs(cur, m_in);
#pragma unroll
    for (int k = 0; k < kPP; ++k) lin[k] = ld32(m_in, cur.rev[k]);
    // stage tile 0
#pragma unroll
    for (int jj = 0; jj < kPJ; ++jj) {
        const int v = tid + jj * kBlockLO;
        if (v <= cur.nn) l.ptr[v] = (unsigned short)(cur.ptr[jj] - cur.s0);
        if (v < cur.nn) l.L[v] = cur.u[jj];
    }
#pragma unroll
    for (int k = 0; k < kPP; ++k) {
        const int q = tid + k * kBlockLO;
        if (q < cur.ns) l.lam[q] = lin[k];
    }
    for (int j = 0;; ++j) {
        const bool has_next = seq.valid(j + 1);
        const int4 bnext2 = seq.valid(j + 2) ? seq.bounds(j + 2) : make_int4(0, 0, 0, 0);
        if (has_next) tile_load<MODE, R16>(nxt, a, m_in, bnext);
        lds_barrier();
        // node aggregates of tile j, incoming messages in slot order; for
        // RnBP also the draws of the node's messages, four per Philox call
        for (int v = tid; v < cur.nn; v += kBlockLO) {
            const int q0 = l.ptr[v], q1 = l.ptr[v + 1];
            float L = l.L[v];
            for (int q = q0; q < q1; ++q) {
                L += l.lam[q];
                l.owner[q] = (unsigned short)v;
            }
            l.L[v] = L;
            if (MODE == kModeRnBP) {
                for (int q = q0; q < q1; q += 4) {
                    const uint4 w = philox4((unsigned int)(cur.n0 + v), (unsigned int)(q - q0) >> 2,
                                            a.t, a.key0, a.key1);
                    l.u[q] = w.x >> 8;
                    if (q + 1 < q1) l.u[q + 1] = w.y >> 8;
                    if (q + 2 < q1) l.u[q + 2] = w.z >> 8;
                    if (q + 3 < q1) l.u[q + 3] = w.w >> 8;
                }
            }
        }
        lds_barrier();
        float lin_n[kPP];
        if (has_next) {
#pragma unroll
            for (int k = 0; k < kPP; ++k) lin_n[k] = ld32(m_in, nxt.rev[k]);
        }
        // outgoing messages of tile j, written at their own slots
#pragma unroll
        for (int k = 0; k < kPP; ++k) {
            const int q = tid + k * kBlockLO;
            float r = 0.0f;
            if (q < cur.ns) {
                const int v = l.owner[q];
                const unsigned int u24 = MODE == kModeRnBP ? l.u[q] : 0u;
                r = logodds_slot<MODE>(a, out, l.L[v], lin[k], cur.J[k], cur.old[k],
                                       cur.s0 + q, u24, act, sa, sb);
                rmax = fmaxf(rmax, r);
            }
            // frontier RBP: the first radix digit of the key (top 8 bits)
            if (MODE == kModeRBP && a.hist0) lds_count(l.hist, __float_as_uint(r) >> 24, q < cur.ns);
        }
        if (!has_next) break;
        lds_barrier();  // tile j's LDS reads are done
        cur = nxt;
#pragma unroll
        for (int k = 0; k < kPP; ++k) lin[k] = lin_n[k];
#pragma unroll
        for (int jj = 0; jj < kPJ; ++jj) {
            const int v = tid + jj * kBlockLO;
            if (v <= cur.nn) l.ptr[v] = (unsigned short)(cur.ptr[jj] - cur.s0);
            if (v < cur.nn) l.L[v] = cur.u[jj];
        }
#pragma unroll
        for (int k = 0; k < kPP; ++k) {
            const int q = tid + k * kBlockLO;
            if (q < cur.ns) l.lam[q] = lin[k];
        }
        bnext = bnext2;
    }
}

// The tiles of this block's XCD range (tiles are dealt to XCDs in contiguous
// ranges so that neighbouring tiles share an L2).
struct XcdTiles {
    const EvalArgs& a;
    const int4* tiles;
    __device__ bool valid(int j) const { return block_tile(a, j) >= 0; }
    __device__ int4 bounds(int j) const { return tiles[block_tile(a, j)]; }
};

// K = 2 evaluation kernel.  A persistent grid (as many blocks as are resident)
// walks the tiles with the pipelined tile loop.
template <int MODE, bool R16>
__global__ __launch_bounds__(kBlockLO) void k_eval_logodds(EvalArgs a) {
    __shared__ LogoddsLds l;
    __shared__ RedScratch red;
    __shared__ unsigned long long s_red[2];

    const int4* __restrict__ tiles = (const int4*)a.tiles4;
    const int t0 = block_tile(a, 0), t1 = block_tile(a, 1);
    // a block without tiles loads tile 0 and computes nothing, so that the
    // first loads are unconditional
    int4 bcur = tiles[t0 >= 0 ? t0 : 0];
    int4 bnext = t1 >= 0 ? tiles[t1] : make_int4(0, 0, 0, 0);
    // the counters are loaded first and the first tile's graph constants next,
    // so that the two latencies overlap (loads complete in issue order)
    CtrLoad cl;
    prologue_issue(a, cl, blockIdx.x == 0);
    TileRegs cur;
    tile_load_const<MODE, R16>(cur, a, bcur);
    __builtin_amdgcn_sched_barrier(0);
    const float* m_sel = prologue_finish(a, cl, s_red, blockIdx.x == 0);
    if (!m_sel) return;
    const float* __restrict__ m_in = uniform_ptr(m_sel);
    float rmax = 0.0f;
    unsigned int act = 0, sa = 0, sb = 0;
    const bool hist = MODE == kModeRBP && a.hist0;
    if (hist)
        for (int i = threadIdx.x; i < 256; i += kBlockLO) l.hist[i] = 0u;  // seen after the loop's barriers
    if (t0 >= 0)
        logodds_tile_loop<MODE, XcdTiles, R16>(a, m_in, XcdTiles{a, tiles}, cur, bnext, l, rmax, act,
                                              sa, sb);
    if (hist) {
        // the block's digit counts into one of the copies of the global histogram
        lds_barrier();
        unsigned int* gh = &a.st->hist[blockIdx.x & 15][0];
        for (int i = threadIdx.x; i < 256; i += kBlockLO)
            if (l.hist[i]) atomicAdd(&gh[i], l.hist[i]);
    }
    block_accumulate(&red, a.ctr, a.t, rmax, act, sa, sb);
}

// A node whose degree exceeds a tile: one block, aggregate by a block
// reduction of the gathered incoming messages, then stream the slots.
template <int MODE>
__device__ __forceinline__ void logodds_big_node(const EvalArgs& a, const float* __restrict__ m_in,
                                                 int4 b, float* s_part, float& rmax,
                                                 unsigned int& act, unsigned int& sa,
                                                 unsigned int& sb) {
    const int tid = threadIdx.x;
    const int n0 = b.x, s0 = b.z, ns = b.w - b.z;
    float part = 0.0f;
    const int nt = (int)blockDim.x;
    for (int q = tid; q < ns; q += nt) part += m_in[a.rev[s0 + q]];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) part += __shfl_xor(part, o, 64);
    if ((tid & 63) == 0) s_part[tid >> 6] = part;
    __syncthreads();
    float L = a.unary[n0];
#pragma unroll
    for (int i = 0; i < nt / 64; ++i) L += s_part[i];
    for (int q = tid; q < ns; q += nt) {
        const int s = s0 + q;
        const unsigned int u24 = MODE == kModeRnBP ? draw24(a, n0, q) : 0u;
        const float r = logodds_slot<MODE>(a, OutPtr{a}, L, m_in[a.rev[s]], a.coupling[s], m_in[s], s,
                                           u24, act, sa, sb);
        rmax = fmaxf(rmax, r);
    }
}

// Nodes whose degree exceeds a tile, one block each.  Runs after k_eval_logodds
// in the same iteration (same prologue, no bookkeeping).
template <int MODE>
__global__ __launch_bounds__(kBlock) void k_eval_logodds_big(EvalArgs a) {
    __shared__ RedScratch red;
    __shared__ float s_part[kBlock / 64];
    __shared__ unsigned long long s_red[2];
    const int4 b = ((const int4*)a.big4)[blockIdx.x];
    const float* __restrict__ m_in = iteration_prologue(a, s_red, false);
    if (!m_in) return;
    float rmax = 0.0f;
    unsigned int act = 0, sa = 0, sb = 0;
    logodds_big_node<MODE>(a, m_in, b, s_part, rmax, act, sa, sb);
    block_accumulate(&red, a.ctr, a.t, rmax, act, sa, sb);
}

// ---------------------------------------------------------------------------
// Batched evaluation for serving: one launch evaluates one iteration of every
// graph of a batch.  The graph's arguments live in device memory and its
// iteration number is the launch index minus the launch of its first
// evaluation, so graphs admitted at different times advance independently,
// each exactly as bp_run would advance it alone (same tiles, same per-slot
// arithmetic, per-graph counters and random keys).  The launch index is a
// device counter (BatchCtl), so a sequence of launches can be recorded once in
// a HIP graph and replayed.
//
// The grid is persistent: block b takes a contiguous range of the tile list
// (entries of one graph are contiguous, regular tiles first), splits it into
// runs of one graph, and runs each graph's regular tiles through the same
// software-pipelined tile loop as bp_run's kernel, then its oversized nodes.
// ---------------------------------------------------------------------------

// Before each batched launch: the per-launch fields of every graph's
// arguments, as bp_run sets them for its iteration `it`.
__global__ void k_batch_advance(BatchGraph* graphs, int num_graphs, const BatchCtl* ctl) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= num_graphs) return;
    const long long launch = ctl->launch;
    BatchGraph& G = graphs[g];
    const long long it = launch - G.first;
    G.skip = (it < 0 || it > G.max_iters) ? 1 : 0;
    if (G.skip) return;
    EvalArgs& a = G.a;
    a.it = it;
    a.t = (unsigned int)it;
    a.after_final = 0;
    const int pin = (int)(it & 1);
    a.in_buf[0] = it == 0 ? G.msg[0] : G.msg[2 * pin];
    a.in_buf[1] = it == 0 ? G.msg[0] : G.msg[2 * pin + 1];
    a.out_buf[0] = G.msg[2 * (pin ^ 1)];
    a.out_buf[1] = G.msg[2 * (pin ^ 1) + 1];
    G.mode_now = it == G.max_iters ? kModeEvalOnly : G.mode;
}

// The regular tiles of one graph's run of list entries.
struct ListTiles {
    const int4* tiles;
    const int4* list;
    int e0, n;
    __device__ bool valid(int j) const { return j < n; }
    __device__ int4 bounds(int j) const { return tiles[list[e0 + j].y]; }
};

template <int MODE>
__device__ __forceinline__ void batch_run(const EvalArgs& a, const float* __restrict__ m_in,
                                          const int4* __restrict__ list, int e0, int nreg, int e1,
                                          LogoddsLds& l, float* s_part, float& rmax,
                                          unsigned int& act, unsigned int& sa, unsigned int& sb) {
    if (nreg > 0) {
        const ListTiles seq{(const int4*)a.tiles4, list, e0, nreg};
        TileRegs cur;
        tile_load_const<MODE>(cur, a, seq.bounds(0));
        const int4 bnext = nreg > 1 ? seq.bounds(1) : make_int4(0, 0, 0, 0);
        logodds_tile_loop<MODE>(a, m_in, seq, cur, bnext, l, rmax, act, sa, sb);
    }
    for (int e = e0 + nreg; e < e1; ++e) {
        const int4 b = ((const int4*)a.big4)[list[e].y];
        logodds_big_node<MODE>(a, m_in, b, s_part, rmax, act, sa, sb);
    }
}

__global__ __launch_bounds__(kBlockLO) void k_eval_batch(const BatchGraph* __restrict__ graphs,
                                                       const int4* __restrict__ list,
                                                       BatchCtl* ctl) {
    __shared__ LogoddsLds l;
    __shared__ float s_part[kBlock / 64];
    __shared__ RedScratch red;
    __shared__ unsigned long long s_red[2];
    // the next launch's index (k_batch_advance of this launch has read it)
    if (blockIdx.x == 0 && threadIdx.x == 0) ctl->launch += 1;
    const int n = ctl->entries;
    const int per = (n + (int)gridDim.x - 1) / (int)gridDim.x;
    int e = (int)blockIdx.x * per;
    const int e_end = min(n, e + per);
    while (e < e_end) {
        const int4 ent = list[e];  // {graph slot, tile, oversized node?, 0}
        int f = e + 1;
        while (f < e_end && list[f].x == ent.x) ++f;
        int r1 = e;
        while (r1 < f && list[r1].z == 0) ++r1;
        const BatchGraph& G = graphs[ent.x];
        if (!G.skip) {  // not admitted yet, or finished
            const EvalArgs& a = G.a;
            // the block holding the graph's first tile closes its previous iteration
            const float* m_sel = iteration_prologue(a, s_red, ent.z == 0 && ent.y == 0);
            if (m_sel) {
                const float* __restrict__ m_in = uniform_ptr(m_sel);
                float rmax = 0.0f;
                unsigned int act = 0, sa = 0, sb = 0;
                const int mode = G.mode_now;
                if (mode == kModeLBP)
                    batch_run<kModeLBP>(a, m_in, list, e, r1 - e, f, l, s_part, rmax, act, sa, sb);
                else if (mode == kModeRnBP)
                    batch_run<kModeRnBP>(a, m_in, list, e, r1 - e, f, l, s_part, rmax, act, sa, sb);
                else
                    batch_run<kModeEvalOnly>(a, m_in, list, e, r1 - e, f, l, s_part, rmax, act, sa,
                                             sb);
                block_accumulate(&red, a.ctr, a.t, rmax, act, sa, sb);
            }
        }
        lds_barrier();  // the run's LDS (and s_red) is free for the next run
        e = f;
    }
}

// ---------------------------------------------------------------------------
// Generic layout: [E][K] normalised FP32 probabilities, K <= KP.
// ---------------------------------------------------------------------------
// Lanes of one group of R = 2 or 4 consecutive lanes (R aligned) exchanging
// values with DPP quad permutations (no LDS).
__device__ __forceinline__ float dpp_xor1(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xB1, 0xF, 0xF, false));
}
__device__ __forceinline__ float dpp_xor2(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x4E, 0xF, 0xF, false));
}
__device__ __forceinline__ float dpp_xor3(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x1B, 0xF, 0xF, false));
}
template <int R>
__device__ __forceinline__ float group_max(float v) {
    v = fmaxf(v, dpp_xor1(v));
    if (R == 4) v = fmaxf(v, dpp_xor2(v));
    return v;
}
// Sum over the group in a fixed order (part 0 + part 1 [+ part 2 + part 3]),
// the same in every lane of the group.
template <int R>
__device__ __forceinline__ float group_sum(float v, int h) {
    if (R == 2) {
        const float o = dpp_xor1(v);
        return h == 0 ? v + o : o + v;
    }
    const float o1 = dpp_xor1(v), o2 = dpp_xor2(v), o3 = dpp_xor3(v);
    float p[4];
    p[0] = h == 0 ? v : h == 1 ? o1 : h == 2 ? o2 : o3;
    p[1] = h == 1 ? v : h == 0 ? o1 : h == 3 ? o2 : o3;
    p[2] = h == 2 ? v : h == 3 ? o1 : h == 0 ? o2 : o3;
    p[3] = h == 3 ? v : h == 2 ? o1 : h == 1 ? o2 : o3;
    return (p[0] + p[1]) + (p[2] + p[3]);
}
// Lane pp of each group, read by every lane of the group (DPP quad_perm
// broadcast; for R = 2 the quad holds two groups).
template <int R, int PP>
__device__ __forceinline__ float group_bcast(float v) {
    constexpr int sel = R == 4 ? PP * 0x55 : (PP | PP << 2 | (2 + PP) << 4 | (2 + PP) << 6);
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), sel, 0xF, 0xF, false));
}
template <int R>
__device__ __forceinline__ float group_bcast(float v, int pp) {
    return pp == 0 ? group_bcast<R, 0>(v)
                   : pp == 1 ? group_bcast<R, 1>(v)
                             : pp == 2 ? group_bcast<R, 2 % R>(v) : group_bcast<R, 3 % R>(v);
}

// Outcome flags of [E][K] rows (EvalArgs.row_flags).  A launch under dynamic p
// writes whole rows of one outcome (the one its prologue chose for the previous
// iteration: a prediction) and the other outcome's row only where the two keep
// decisions differ, marked by the sign bit of the whole row's first entry
// (messages are non-negative).  The next launch reads whole rows from `p` (the
// buffer of the predicted outcome); if it chose the other outcome, flagged rows
// come from `alt`.  `on` is 0 for rows written without flags.
struct FlagRows {
    const float* p;
    const float* alt;   // nullptr: the prediction held
    int on;
};

// Entry x of the row starting at `row` (x == 0 loses the flag bit).
__device__ __forceinline__ float flag_entry(const FlagRows& f, long long row, int x) {
    float v = f.p[row + x];
    if (f.on) {
        if (f.alt && (__float_as_uint(f.p[row]) >> 31)) v = f.alt[row + x];
        if (x == 0) v = fabsf(v);
    }
    return v;
}

// Where a launch writes: whole rows of outcome `prim`, the other outcome's
// rows where the decisions differ.
__device__ __forceinline__ float flag_first(float v, bool diff) {
    return diff ? __uint_as_float(__float_as_uint(v) | 0x80000000u) : v;
}

// The input rows of a launch and the outcome its own rows are written for:
// sel = the outcome its prologue chose (m_sel = in_buf[sel]); with flags the
// previous launch wrote whole rows of outcome in_sel[t - 1].
__device__ __forceinline__ FlagRows flag_inputs(const EvalArgs& a, const float* m_sel,
                                                int& p_out) {
    const int sel = (a.it >= 1 && m_sel == a.in_buf[1]) ? 1 : 0;
    p_out = a.it == 0 ? a.sel0 : sel;
    FlagRows f{m_sel, nullptr, 0};
    if (a.row_flags && a.it >= 1) {
        const int p_in = (int)a.st->in_sel[(a.t - 1u) & 3u];
        f.p = a.in_buf[p_in];
        f.alt = p_in != sel ? a.in_buf[p_in ^ 1] : nullptr;
        f.on = 1;
    }
    return f;
}

// Eq. (2) for one slot split over a group of R lanes (KP = K states, each lane
// owns KR = K / R of them): the lane computes its part of the cavity
// distribution g, and each lane forms its KR outputs c(y) = sum_x psi(x, y) g(x)
// from the shared table in LDS, taking g(x) of the other parts from their lanes
// one value at a time (a lane never holds all of g).  Messages that use the
// transposed table read psi^T, staged beside psi, so that both sum over x in
// ascending order with the same row reads.  The normalisation and the residual
// are reduced over the group.
template <int KP, int R, int MODE>
__device__ __forceinline__ void slot_update_split(const EvalArgs& a, const FlagRows& fr,
                                                  const float* s_logm, const float* s_A,
                                                  const float* s_psi, const float* s_psiT,
                                                  const unsigned short* s_owner, int s0, int n0,
                                                  int ns, float& rmax, unsigned int& act,
                                                  unsigned int& sa, unsigned int& sb, int p_out) {
    const float* __restrict__ m_in = fr.p;
    constexpr int KR = KP / R;
    constexpr int KS = KP + 1;
    const int tid = threadIdx.x;
    const int q = tid / R, h = tid % R;
    if (q >= ns) return;  // the R lanes of a slot leave together
    const int s = s0 + q;
    const int v = s_owner[q];
    float gp[KR];
    float mx = -3.402823466e38f;
#pragma unroll
    for (int i = 0; i < KR; ++i) {
        const int x = h * KR + i;
        gp[i] = s_A[v * KS + x] - s_logm[q * KS + x];
        mx = fmaxf(mx, gp[i]);
    }
    mx = group_max<R>(mx);
#pragma unroll
    for (int i = 0; i < KR; ++i) gp[i] = expf(gp[i] - mx);
    const float* tab =
        a.pair_kind == kPairSharedAsym && a.orient[s] ? s_psiT : s_psi;
    float c[KR];
#pragma unroll
    for (int j = 0; j < KR; ++j) c[j] = 0.0f;
#pragma unroll
    for (int pp = 0; pp < R; ++pp) {
#pragma unroll
        for (int i = 0; i < KR; ++i) {
            const float gx = group_bcast<R>(gp[i], pp);  // g(x), x = pp KR + i
            const float4* row = (const float4*)(tab + (pp * KR + i) * KP + h * KR);
#pragma unroll
            for (int j4 = 0; j4 < KR / 4; ++j4) {
                const float4 p4 = row[j4];
                c[4 * j4] = fmaf(p4.x, gx, c[4 * j4]);
                c[4 * j4 + 1] = fmaf(p4.y, gx, c[4 * j4 + 1]);
                c[4 * j4 + 2] = fmaf(p4.z, gx, c[4 * j4 + 2]);
                c[4 * j4 + 3] = fmaf(p4.w, gx, c[4 * j4 + 3]);
            }
        }
    }
    float z = 0.0f;
#pragma unroll
    for (int j = 0; j < KR; ++j) z += c[j];
    z = group_sum<R>(z, h);
    const float inv = 1.0f / z;
    const long long eo = (long long)s * KP + h * KR;
    float old[KR];
    float r = 0.0f;
#pragma unroll
    for (int j4 = 0; j4 < KR / 4; ++j4) {
        const float4 o4 = *(const float4*)(m_in + eo + 4 * j4);
        old[4 * j4] = o4.x;
        old[4 * j4 + 1] = o4.y;
        old[4 * j4 + 2] = o4.z;
        old[4 * j4 + 3] = o4.w;
    }
    if (fr.on) {
        // the flag is the sign of the row's first entry (lane h = 0 holds it)
        const long long row = (long long)s * KP;
        if (fr.alt && (__float_as_uint(m_in[row]) >> 31)) {
#pragma unroll
            for (int j4 = 0; j4 < KR / 4; ++j4) {
                const float4 o4 = *(const float4*)(fr.alt + eo + 4 * j4);
                old[4 * j4] = o4.x;
                old[4 * j4 + 1] = o4.y;
                old[4 * j4 + 2] = o4.z;
                old[4 * j4 + 3] = o4.w;
            }
        }
        if (h == 0) old[0] = fabsf(old[0]);
    }
#pragma unroll
    for (int j = 0; j < KR; ++j) {
        c[j] *= inv;
        r = fmaxf(r, fabsf(c[j] - old[j]));
    }
    r = group_max<R>(r);
    const bool active = r > a.eps;
    const bool lead = h == 0;  // counts once per slot
    rmax = fmaxf(rmax, r);
    act += active && lead;
    if (MODE == kModeLBP) {
#pragma unroll
        for (int j = 0; j < KR; ++j) a.out_buf[0][eo + j] = c[j];
    } else if (MODE == kModeRnBP) {
        bool ka = false, kb = false;
        if (active) {
            const int node = n0 + v;
            const unsigned int u24 = draw24(a, node, s - a.node_ptr[node]);
            ka = u24 < a.thr_a;
            kb = u24 < a.thr_b;
        }
        sa += ka && lead;
        sb += kb && lead;
        if (a.row_flags) {
            const bool kp = p_out == 0 ? ka : kb, ko = p_out == 0 ? kb : ka;
            const bool diff = ka != kb;
            float* op = a.out_buf[p_out] + eo;
#pragma unroll
            for (int j = 0; j < KR; ++j)
                op[j] = (j == 0 && h == 0) ? flag_first(kp ? c[0] : old[0], diff) : (kp ? c[j] : old[j]);
            if (diff) {
                float* os = a.out_buf[p_out ^ 1] + eo;
#pragma unroll
                for (int j = 0; j < KR; ++j) os[j] = ko ? c[j] : old[j];
            }
            return;
        }
#pragma unroll
        for (int j = 0; j < KR; ++j) a.out_buf[0][eo + j] = ka ? c[j] : old[j];
        if (a.two_outputs) {
#pragma unroll
            for (int j = 0; j < KR; ++j) a.out_buf[1][eo + j] = kb ? c[j] : old[j];
        }
    } else if (MODE == kModeRBP) {
#pragma unroll
        for (int j = 0; j < KR; ++j) a.cand[eo + j] = c[j];
        if (lead) a.keys[s] = __float_as_uint(r);
    }
}

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef short shortx4 __attribute__((ext_vector_type(4)));

// FP32 -> BF16 bit pattern, round to nearest even (finite inputs).
__device__ __forceinline__ short bf16_rne(float f) {
    const unsigned int b = __float_as_uint(f);
    return (short)((b + 0x7FFFu + ((b >> 16) & 1u)) >> 16);
}

// Eq. (2) for K = 32 with one symmetric shared table on the matrix cores.  Each
// wave takes 32 slots of the tile; the products c = g P of its slots are one
// 32 x 32 x 32 matrix product, 16 v_mfma_f32_32x32x2f32 steps with FP32 inputs
// and FP32 accumulation.  Operand layout of that instruction: lane l supplies
// A[l % 32][l / 32] and B[l / 32][l % 32] of each 32 x 2 / 2 x 32 step, and
// holds D[8 (r / 4) + 4 (l / 32) + r % 4][l % 32] in accumulator r = 0..15.
// So lane (m = l % 32, h = l / 32) computes the cavity values g(x) of slot m
// for the states x = 2 s + h, holds column m of the table for those states,
// and after the product the tile goes through LDS (rows of 33 floats) back to
// one slot per lane pair, each lane with 16 consecutive states of its slot.
// BF16: the same product with BF16 operands (v_mfma_f32_32x32x8_bf16, FP32
// accumulation): 4 steps of 8 states, lane (m, h) supplying the states
// 8 s + 4 h .. 8 s + 4 h + 3; g and the table are rounded to 8-bit mantissas.
// The lane's operand entry st of the product covers state mfma32_state(st).
template <bool BF16>
__device__ __forceinline__ int mfma32_state(int st, int h) {
    return BF16 ? 8 * (st >> 2) + 4 * h + (st & 3) : 2 * st + h;
}

// B operand of the lane: P[x][m] for its 16 states (loaded once per block).
template <bool BF16>
__device__ __forceinline__ void mfma32_table(const EvalArgs& a, float* pb) {
    const int lane = threadIdx.x & 63, m = lane & 31, h = lane >> 5;
#pragma unroll
    for (int st = 0; st < 16; ++st) pb[st] = a.pair[mfma32_state<BF16>(st, h) * 32 + m];
}

// old: the lane's 16 states of its slot's current row (issued by the caller).
// p_out (row_flags): the outcome whose rows are written whole.
template <int MODE, bool BF16 = false>
__device__ __forceinline__ void slot_update_mfma32(const EvalArgs& a, const float* pb,
                                                   const float* old, float* s_logm,
                                                   const float* s_A,
                                                   const unsigned short* s_owner, int s0,
                                                   int n0, int ns, float& rmax,
                                                   unsigned int& act, unsigned int& sa,
                                                   unsigned int& sb, int p_out = 0) {
    constexpr int K = 32, KS = 33;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int m = lane & 31, h = lane >> 5;
    const int q = 32 * w + m;  // slot of the tile
    const bool valid = q < ns;
    auto state = [&](int st) { return mfma32_state<BF16>(st, h); };
    // A operand: the cavity distribution of slot q at the lane's states
    const int v = valid ? s_owner[q] : 0;
    float gv[16];
    float mx = -3.402823466e38f;
#pragma unroll
    for (int st = 0; st < 16; ++st) {
        const int x = state(st);
        gv[st] = valid ? s_A[v * KS + x] - s_logm[q * KS + x] : 0.0f;
        mx = fmaxf(mx, gv[st]);
    }
    mx = fmaxf(mx, __shfl_xor(mx, 32, 64));
#pragma unroll
    for (int st = 0; st < 16; ++st) gv[st] = expf(gv[st] - mx);
    floatx16 d;
#pragma unroll
    for (int r = 0; r < 16; ++r) d[r] = 0.0f;
    if (BF16) {
#pragma unroll
        for (int st = 0; st < 4; ++st) {
            const shortx4 ga = {bf16_rne(gv[4 * st]), bf16_rne(gv[4 * st + 1]), bf16_rne(gv[4 * st + 2]),
                                bf16_rne(gv[4 * st + 3])};
            const shortx4 pbb = {bf16_rne(pb[4 * st]), bf16_rne(pb[4 * st + 1]), bf16_rne(pb[4 * st + 2]),
                                 bf16_rne(pb[4 * st + 3])};
            d = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(ga, pbb, d, 0, 0, 0);
        }
    } else {
#pragma unroll
        for (int st = 0; st < 16; ++st)
            d = __builtin_amdgcn_mfma_f32_32x32x2f32(gv[st], pb[st], d, 0, 0, 0);
    }
    // D[i][m] -> LDS row 32 w + i (the wave's own rows of the log buffer, which
    // its lanes have finished reading: LDS operations of a wave run in order)
    float* rows = s_logm + (32 * w) * KS;
#pragma unroll
    for (int r = 0; r < 16; ++r) rows[(8 * (r >> 2) + 4 * h + (r & 3)) * KS + m] = d[r];
    // back as slot m, states 16 h .. 16 h + 15
    float c[16];
#pragma unroll
    for (int t = 0; t < 16; ++t) c[t] = rows[m * KS + 16 * h + t];
    if (!valid) return;
    float z = 0.0f;
#pragma unroll
    for (int t = 0; t < 16; ++t) z += c[t];
    const float zo = __shfl_xor(z, 32, 64);
    z = h == 0 ? z + zo : zo + z;
    const float inv = 1.0f / z;
    const int sl = s0 + q;
    const long long eo = (long long)sl * K + 16 * h;
    float r = 0.0f;
#pragma unroll
    for (int t = 0; t < 16; ++t) {
        c[t] *= inv;
        r = fmaxf(r, fabsf(c[t] - old[t]));
    }
    r = fmaxf(r, __shfl_xor(r, 32, 64));
    const bool active = r > a.eps;
    const bool lead = h == 0;  // counts once per slot
    rmax = fmaxf(rmax, r);
    act += active && lead;
    float4* o0 = (float4*)(a.out_buf[0] + eo);
    if (MODE == kModeLBP) {
#pragma unroll
        for (int t4 = 0; t4 < 4; ++t4)
            o0[t4] = make_float4(c[4 * t4], c[4 * t4 + 1], c[4 * t4 + 2], c[4 * t4 + 3]);
    } else if (MODE == kModeRnBP) {
        bool ka = false, kb = false;
        if (active) {
            const int node = n0 + v;
            const unsigned int u24 = draw24(a, node, sl - a.node_ptr[node]);
            ka = u24 < a.thr_a;
            kb = u24 < a.thr_b;
        }
        sa += ka && lead;
        sb += kb && lead;
        if (a.row_flags) {
            // the whole row of outcome p_out, its first entry's sign bit set where
            // the outcomes differ; the other outcome's row only there
            const bool kp = p_out == 0 ? ka : kb, ko = p_out == 0 ? kb : ka;
            const bool diff = ka != kb;
            float4* op = (float4*)(a.out_buf[p_out] + eo);
#pragma unroll
            for (int t4 = 0; t4 < 4; ++t4) {
                float4 v = kp ? make_float4(c[4 * t4], c[4 * t4 + 1], c[4 * t4 + 2], c[4 * t4 + 3])
                              : make_float4(old[4 * t4], old[4 * t4 + 1], old[4 * t4 + 2],
                                            old[4 * t4 + 3]);
                if (t4 == 0 && h == 0 && diff) v.x = __uint_as_float(__float_as_uint(v.x) | 0x80000000u);
                op[t4] = v;
            }
            if (diff) {
                float4* os = (float4*)(a.out_buf[p_out ^ 1] + eo);
#pragma unroll
                for (int t4 = 0; t4 < 4; ++t4)
                    os[t4] = ko ? make_float4(c[4 * t4], c[4 * t4 + 1], c[4 * t4 + 2], c[4 * t4 + 3])
                                : make_float4(old[4 * t4], old[4 * t4 + 1], old[4 * t4 + 2],
                                              old[4 * t4 + 3]);
            }
            return;
        }
#pragma unroll
        for (int t4 = 0; t4 < 4; ++t4)
            o0[t4] = ka ? make_float4(c[4 * t4], c[4 * t4 + 1], c[4 * t4 + 2], c[4 * t4 + 3])
                        : make_float4(old[4 * t4], old[4 * t4 + 1], old[4 * t4 + 2], old[4 * t4 + 3]);
        if (a.two_outputs) {
            float4* o1 = (float4*)(a.out_buf[1] + eo);
#pragma unroll
            for (int t4 = 0; t4 < 4; ++t4)
                o1[t4] = kb ? make_float4(c[4 * t4], c[4 * t4 + 1], c[4 * t4 + 2], c[4 * t4 + 3])
                            : make_float4(old[4 * t4], old[4 * t4 + 1], old[4 * t4 + 2], old[4 * t4 + 3]);
        }
    } else if (MODE == kModeRBP) {
        float4* oc = (float4*)(a.cand + eo);
#pragma unroll
        for (int t4 = 0; t4 < 4; ++t4)
            oc[t4] = make_float4(c[4 * t4], c[4 * t4 + 1], c[4 * t4 + 2], c[4 * t4 + 3]);
        if (lead) a.keys[sl] = __float_as_uint(r);
    }
}

// A shared K x K table seen through the constant address space: with K known
// at compile time its entries are wave-uniform scalar loads (s_load into SGPRs
// that the multiply-adds read directly), not one LDS read per multiply-add.
typedef const __attribute__((address_space(4))) float* ConstF;

// c(y) += sum_x P[x][y] g(x) (T: P[y][x]) for a uniform table P.
template <int K, bool T>
__device__ __forceinline__ void matvec_uniform(ConstF P, const float* g, float* c) {
#pragma unroll
    for (int x = 0; x < K; ++x) {
        const float gx = g[x];
#pragma unroll
        for (int y = 0; y < K; ++y) c[y] = fmaf(T ? P[y * K + x] : P[x * K + y], gx, c[y]);
    }
}

// EXACT: K == KP, so K is a compile-time constant (shifts instead of
// divisions, scalar loads of a shared table).
// LDS of the [E][K] kernels: rows of K + 1 floats (a thread per slot reads its
// own row, and an odd stride puts the rows of neighbouring lanes in different
// banks).  Node rows are sized by the largest node count of a tile.
struct GenericLds {
    float* logm;             // [TS][KS] logs of the incoming messages
    float* A;                // [TN][KS] node aggregates
    float* psi;              // [K][K] shared table (paths that read it from LDS)
    float* psiT;             // [K][K] its transpose (asymmetric tables), else psi
    int* rev;                // [TS]
    int* ptr;                // [TN + 1] local slot offsets of the nodes
    unsigned short* owner;   // [TS]
};

// tables: the number of K x K tables reserved (0; 1, psi; 2, psi and psi^T);
// the launch sizes the LDS the same way
__device__ __forceinline__ GenericLds generic_lds(float* smem, int K, int TS, int TN,
                                                  int tables) {
    GenericLds l;
    const int KS = K + 1;
    l.logm = smem;
    l.A = l.logm + TS * KS;
    l.psi = l.A + ((TN * KS + 3) & ~3);  // 16-byte aligned: read as float4 rows
    l.psiT = tables == 2 ? l.psi + K * K : l.psi;
    l.rev = (int*)(l.psi + tables * K * K);
    l.ptr = l.rev + TS;
    l.owner = (unsigned short*)(l.ptr + TN + 1);
    return l;
}

// Phase 1 of a tile whose slots fit (ns <= TS): gather the incoming rows
// m_{k->i} (K consecutive threads per row; a tile holds at most
// kTileFloatsGeneric values, kPer per thread, and a thread issues all of its
// loads before using the first), take logs of K * m (the constant cancels in
// the cavity and the normalisation, and it keeps the node aggregate near zero
// for messages near uniform, where FP32 rounding of a large aggregate would
// dominate), and sum them per node with the unary: A_i(x) of Eq. (2)/(3).
// Ends with a barrier.
// Rows written with outcome flags (EvalArgs.row_flags): m_in is the buffer of
// full rows; the sign bit of a row's first entry marks a message whose other
// outcome is in m_alt.  m_alt == nullptr: the full rows hold the chosen
// outcome, and only the flag bit is cleared (a no-op on unflagged rows).
__device__ __forceinline__ void generic_phase1(const EvalArgs& a, const float* __restrict__ m_in,
                                               const GenericLds& l, int K, int n0, int nn,
                                               int s0, int ns, const float* m_alt = nullptr) {
    const int tid = threadIdx.x;
    const int KS = K + 1;
    const float fK = (float)K;
    for (int q = tid; q < ns; q += kBlock) l.rev[q] = a.rev[s0 + q];
    for (int v = tid; v <= nn; v += kBlock) l.ptr[v] = a.node_ptr[n0 + v] - s0;
    __syncthreads();
    constexpr int kPer = kTileFloatsGeneric / kBlock;
    float gat[kPer];
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        const int i = tid + j * kBlock;
        const int q = i / K, x = i - q * K;
        gat[j] = q < ns ? m_in[(long long)l.rev[q] * K + x] : 1.0f;
    }
    if (m_alt) {
        // the other outcome was chosen: flagged rows come from m_alt
        unsigned int f[kPer];
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
            const int i = tid + j * kBlock;
            const int q = i / K;
            f[j] = q < ns ? __float_as_uint(m_in[(long long)l.rev[q] * K]) >> 31 : 0u;
        }
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
            const int i = tid + j * kBlock;
            const int q = i / K, x = i - q * K;
            if (f[j]) gat[j] = m_alt[(long long)l.rev[q] * K + x];
        }
    }
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        const int i = tid + j * kBlock;
        const int q = i / K, x = i - q * K;
        if (q < ns) l.logm[q * KS + x] = logf(fK * (x == 0 ? fabsf(gat[j]) : gat[j]));
    }
    // the nodes' unaries (loads first), then the aggregates
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        const int i = tid + j * kBlock;
        const int v = i / K, x = i - v * K;
        gat[j] = v < nn ? a.unary[(long long)(n0 + v) * K + x] : 0.0f;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        const int i = tid + j * kBlock;
        const int v = i / K, x = i - v * K;
        if (v < nn) {
            const int q0 = l.ptr[v], q1 = l.ptr[v + 1];
            float acc = gat[j];
            for (int q = q0; q < q1; ++q) acc += l.logm[q * KS + x];
            l.A[v * KS + x] = acc;
            if (x == 0)
                for (int q = q0; q < q1; ++q) l.owner[q] = (unsigned short)v;
        }
    }
    __syncthreads();
}

// K = 32 with a symmetric shared table and no oversized node: Eq. (2) on the
// matrix cores (slot_update_mfma32).  A kernel of its own, so that its register
// count (and hence its occupancy) is not set by the paths it does not take.
// A block per tile; the table columns and the lane's own row are loaded at the
// start, so that they arrive while the incoming rows are gathered and
// aggregated.  (A persistent variant that pipelined several tiles per block
// ran slower: its register and LDS footprint halved the resident blocks.)
// Five waves per SIMD (96 registers, one spilled) instead of the four that the
// unconstrained allocation (115 with the accumulators) leaves: the kernel is
// bound by memory latency, so more resident waves hide more of it.
template <int MODE, bool BF16>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(5))) void k_eval_mfma32(
    EvalArgs a) {
    extern __shared__ float smem[];
    __shared__ RedScratch red;
    __shared__ unsigned long long s_red[2];
    const float* m_sel = iteration_prologue(a, s_red, blockIdx.x == 0);
    if (!m_sel) return;
    const int tile = tile_of_block(a);
    if (tile >= a.num_tiles) return;
    constexpr int K = 32;
    constexpr int TS = kTileFloatsGeneric / K;
    const GenericLds l = generic_lds(smem, K, TS, a.tile_nodes_max, 0);
    int p_out;
    const FlagRows fr = flag_inputs(a, m_sel, p_out);
    const bool flagged_in = fr.on != 0;
    const float* __restrict__ m_in = fr.p;
    const float* m_alt = fr.alt;
    const int n0 = a.tile_start[tile], n1 = a.tile_start[tile + 1];
    const int s0 = a.tile_slot[tile], s1 = a.tile_slot[tile + 1];
    const int ns = s1 - s0;
    float pb[16];
    mfma32_table<BF16>(a, pb);
    float old[16];
    {
        const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
        const int q = 32 * w + (lane & 31);
        const long long eo = (long long)(s0 + min(q, max(ns - 1, 0))) * K + 16 * (lane >> 5);
#pragma unroll
        for (int t4 = 0; t4 < 4; ++t4) {
            const float4 o4 = *(const float4*)(m_in + eo + 4 * t4);
            old[4 * t4] = o4.x;
            old[4 * t4 + 1] = o4.y;
            old[4 * t4 + 2] = o4.z;
            old[4 * t4 + 3] = o4.w;
        }
        if (flagged_in) {
            // the flag is the sign of entry 0, held by the lane with h = 0
            const unsigned int f0 = __float_as_uint(old[0]) >> 31;
            const unsigned int f = (unsigned int)__shfl((int)f0, lane & 31, 64);
            if (m_alt && f) {
#pragma unroll
                for (int t4 = 0; t4 < 4; ++t4) {
                    const float4 o4 = *(const float4*)(m_alt + eo + 4 * t4);
                    old[4 * t4] = o4.x;
                    old[4 * t4 + 1] = o4.y;
                    old[4 * t4 + 2] = o4.z;
                    old[4 * t4 + 3] = o4.w;
                }
            }
            if ((lane >> 5) == 0) old[0] = fabsf(old[0]);
        }
    }
    generic_phase1(a, m_in, l, K, n0, n1 - n0, s0, ns, m_alt);
    float rmax = 0.0f;
    unsigned int act = 0, sa = 0, sb = 0;
    slot_update_mfma32<MODE, BF16>(a, pb, old, l.logm, l.A, l.owner, s0, n0, ns, rmax, act, sa,
                                   sb, p_out);
    block_accumulate(&red, a.ctr, a.t, rmax, act, sa, sb);
}

// Waves per SIMD asked of the register allocator for k_eval_generic<KP, MODE,
// EXACT> (1 leaves it unconstrained).  The kernel waits on memory, so more
// resident waves pay for a spilled register or two: K = 8 and 32 take five
// (96 registers; 99 and 114 unconstrained), K = 64 takes three (168; 170) and
// under RnBP, whose second outcome needs more live values, or with K below the
// width, two (256; unconstrained the allocator spills into the accumulation
// registers and leaves one).  The other widths fit without a cap, and so does
// the lane-group instantiation (SPLIT: about 60 registers, LDS sets its
// occupancy).
template <int KP, int MODE, bool EXACT, bool SPLIT>
constexpr int generic_waves() {
    if (SPLIT) return 1;
    if (KP == 64) return EXACT && MODE != 1 ? 3 : 2;
    return (KP == 8 || KP == 32) && EXACT ? 5 : 1;
}

// SPLIT: the launch guarantees a shared table, K == KP with R > 1 and no tile
// holding a node over its slot limit, so only the lane-group path is compiled
// (its registers are then not those of the per-slot path).
template <int KP, int MODE, bool EXACT, bool SPLIT = false>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(generic_waves<KP, MODE, EXACT, SPLIT>())))
void k_eval_generic(EvalArgs a) {
    extern __shared__ float smem[];
    __shared__ RedScratch red;
    __shared__ unsigned long long s_red[2];
    const float* m_sel = iteration_prologue(a, s_red, blockIdx.x == 0);
    if (!m_sel) return;
    int p_out;
    const FlagRows fr = flag_inputs(a, m_sel, p_out);
    const float* __restrict__ m_in = fr.p;
    const int tile = tile_of_block(a);
    if (tile >= a.num_tiles) return;
    const int K = EXACT ? KP : a.num_states;
    const int TS = kTileFloatsGeneric / K;  // slots per tile
    const int KS = K + 1;
    const GenericLds l =
        generic_lds(smem, K, TS, a.tile_nodes_max, a.pair_kind == kPairSharedAsym ? 2 : 1);
    float* s_logm = l.logm;
    float* s_A = l.A;
    float* s_psi = l.psi;
    unsigned short* s_owner = l.owner;

    const int n0 = a.tile_start[tile], n1 = a.tile_start[tile + 1];
    const int s0 = a.tile_slot[tile], s1 = a.tile_slot[tile + 1];
    const int ns = s1 - s0, nn = n1 - n0;
    const int tid = threadIdx.x;
    const bool big = !SPLIT && ns > TS;
    const float fK = (float)K;

    // K > 16 with a shared table: each slot is split over R lanes, which read
    // the table from LDS (the lanes of a wave need different columns)
    constexpr int R = (EXACT && KP * kBlock > kTileFloatsGeneric) ? KP * kBlock / kTileFloatsGeneric : 1;
    static_assert(!SPLIT || R > 1, "the lane-group path needs K = KP > 16");
    const bool shared = SPLIT || a.pair_kind == kPairShared || a.pair_kind == kPairSharedAsym;
    if (shared && (!EXACT || R > 1))
        for (int i = tid; i < K * K; i += kBlock) s_psi[i] = a.pair[i];
    if (R > 1 && a.pair_kind == kPairSharedAsym)
        for (int i = tid; i < K * K; i += kBlock) l.psiT[i] = a.pair[(i % K) * K + i / K];
    if (!big) {
        generic_phase1(a, m_in, l, K, n0, nn, s0, ns, fr.alt);
    } else {
        // single node with degree > TS: aggregate each state with a strided sum
        for (int x = 0; x < K; ++x) {
            float part = 0.0f;
            for (int q = tid; q < ns; q += kBlock)
                part += logf(fK * flag_entry(fr, (long long)a.rev[s0 + q] * K, x));
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) part += __shfl_xor(part, o, 64);
            if ((tid & 63) == 0) red.rmax[tid >> 6] = part;
            __syncthreads();
            if (tid == 0) {
                float acc = a.unary[(long long)n0 * K + x];
                for (int i = 0; i < kBlock / 64; ++i) acc += red.rmax[i];
                s_A[x] = acc;
            }
            __syncthreads();
        }
    }
    __syncthreads();

    float rmax = 0.0f;
    unsigned int act = 0, sa = 0, sb = 0;
    if (R > 1 && shared && !big) {
        slot_update_split<KP, R, MODE>(a, fr, s_logm, s_A, s_psi, l.psiT, s_owner, s0, n0, ns, rmax, act,
                                       sa, sb, p_out);
        block_accumulate(&red, a.ctr, a.t, rmax, act, sa, sb);
        return;
    }
    for (int q = tid; q < ns; q += kBlock) {
        const int s = s0 + q;
        const int v = big ? 0 : s_owner[q];
        const int node = n0 + v;
        const long long rin = big ? (long long)a.rev[s] * K : 0;
        float g[KP];
        float mx = -3.402823466e38f;
#pragma unroll
        for (int x = 0; x < KP; ++x) {
            if (x < K) {
                const float lm = big ? logf(fK * flag_entry(fr, rin, x)) : s_logm[q * KS + x];
                g[x] = s_A[v * KS + x] - lm;
                mx = fmaxf(mx, g[x]);
            }
        }
#pragma unroll
        for (int x = 0; x < KP; ++x)
            if (x < K) g[x] = expf(g[x] - mx);
        float c[KP];
#pragma unroll
        for (int y = 0; y < KP; ++y) c[y] = 0.0f;
        if (a.pair_kind == kPairIsing) {
            // exp(J s_i s_k) scaled by exp(-|J|): one entry is 1, the other exp(-2|J|)
            const float J = a.coupling[s];
            const float ep = expf(J - fabsf(J)), em = expf(-J - fabsf(J));
            c[0] = ep * g[0] + em * g[1];
            c[1] = em * g[0] + ep * g[1];
        } else if (EXACT && a.pair_kind != kPairDense) {
            const ConstF P4 = (ConstF)(uintptr_t)a.pair;
            if (a.pair_kind == kPairSharedAsym && a.orient[s])
                matvec_uniform<KP, true>(P4, g, c);
            else
                matvec_uniform<KP, false>(P4, g, c);
        } else {
            // c(y) = sum_x psi(x, y) g(x): element (x, y) of the table at
            // P[x * sx + y * sy] (the transpose for the other direction)
            const float* P;
            int sx = K, sy = 1;
            if (a.pair_kind == kPairDense) {
                P = a.pair + (long long)s * K * K;
            } else {
                P = s_psi;
                if (a.pair_kind == kPairSharedAsym && a.orient[s]) {
                    sx = 1;
                    sy = K;
                }
            }
#pragma unroll
            for (int x = 0; x < KP; ++x) {
                if (x < K) {
                    const float gx = g[x];
#pragma unroll
                    for (int y = 0; y < KP; ++y)
                        if (y < K) c[y] = fmaf(P[x * sx + y * sy], gx, c[y]);
                }
            }
        }
        float z = 0.0f;
#pragma unroll
        for (int y = 0; y < KP; ++y)
            if (y < K) z += c[y];
        const float inv = 1.0f / z;
        const long long eo = (long long)s * K;
        float r = 0.0f;
        float old[KP];
#pragma unroll
        for (int y = 0; y < KP; ++y) {
            if (y < K) {
                c[y] *= inv;
                old[y] = flag_entry(fr, eo, y);
                r = fmaxf(r, fabsf(c[y] - old[y]));
            }
        }
        const bool active = r > a.eps;
        rmax = fmaxf(rmax, r);
        act += active;
        if (MODE == kModeLBP) {
#pragma unroll
            for (int y = 0; y < KP; ++y)
                if (y < K) a.out_buf[0][eo + y] = c[y];
        } else if (MODE == kModeRnBP) {
            bool ka = false, kb = false;
            if (active) {
                const unsigned int u24 = draw24(a, node, s - a.node_ptr[node]);
                ka = u24 < a.thr_a;
                kb = u24 < a.thr_b;
            }
            sa += ka;
            sb += kb;
            if (a.row_flags) {
                // the whole row of outcome p_out, the other where they differ
                const bool kp = p_out == 0 ? ka : kb, ko = p_out == 0 ? kb : ka;
                const bool diff = ka != kb;
                float* op = a.out_buf[p_out] + eo;
#pragma unroll
                for (int y = 0; y < KP; ++y)
                    if (y < K) op[y] = y == 0 ? flag_first(kp ? c[0] : old[0], diff) : (kp ? c[y] : old[y]);
                if (diff) {
                    float* os = a.out_buf[p_out ^ 1] + eo;
#pragma unroll
                    for (int y = 0; y < KP; ++y)
                        if (y < K) os[y] = ko ? c[y] : old[y];
                }
            } else {
#pragma unroll
                for (int y = 0; y < KP; ++y)
                    if (y < K) a.out_buf[0][eo + y] = ka ? c[y] : old[y];
                if (a.two_outputs) {
#pragma unroll
                    for (int y = 0; y < KP; ++y)
                        if (y < K) a.out_buf[1][eo + y] = kb ? c[y] : old[y];
                }
            }
        } else if (MODE == kModeRBP) {
#pragma unroll
            for (int y = 0; y < KP; ++y)
                if (y < K) a.cand[eo + y] = c[y];
            a.keys[s] = __float_as_uint(r);
        }
    }
    block_accumulate(&red, a.ctr, a.t, rmax, act, sa, sb);
}

// Closes the last evaluation of a run (one wave): the same bookkeeping the
// next evaluation's prologue would do.
__global__ void k_close_run(EvalArgs a) {
    if (a.st->done) return;
    CtrLoad c;
    ctr_load(a, true, c);
    unsigned long long n1;
    long long n2;
    wave_close(a, true, c, n1, n2);
}

__global__ void k_init_state(DevState* st, CounterLine* ctr) {
    unsigned int* w = (unsigned int*)st;
    const int nw = (int)(sizeof(DevState) / sizeof(unsigned int));
    for (int i = threadIdx.x; i < nw; i += blockDim.x) w[i] = 0u;
    unsigned int* c = (unsigned int*)ctr;
    const int nc = (int)(4 * kCounterCopies * sizeof(CounterLine) / sizeof(unsigned int));
    for (int i = threadIdx.x; i < nc; i += blockDim.x) c[i] = 0u;
    __syncthreads();
    if (threadIdx.x == 0) {
        st->conv_t = -1;
        st->last_prev = -1;
    }
}

__global__ void k_fill(float* p, float v, long long n) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        p[i] = v;
}

// ---------------------------------------------------------------------------
// Eq. (3): beliefs from the node aggregate.
// ---------------------------------------------------------------------------
__global__ void k_marginals_logodds(const int* node_ptr, const int* rev, const float* unary,
                                    const float* lam, float* out, int N) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    float L = unary[n];
    for (int s = node_ptr[n]; s < node_ptr[n + 1]; ++s) L += lam[rev[s]];
    out[2 * (long long)n + 1] = 1.0f / (1.0f + expf(-L));
    out[2 * (long long)n + 0] = 1.0f / (1.0f + expf(L));
}

// Wave-wide max and sum (every lane gets the result).
__device__ __forceinline__ float wave_max_f(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ float wave_sum_f(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Eq. (3) for the [E][K] layout: a group of W lanes per variable (W = K
// rounded up to a power of two, 64 / W variables per wave), lane x holding
// state x, so each incoming row is one coalesced read; the logs of K m are
// summed in slot order, as the evaluation kernels sum them.  The reverse slots
// of up to W incoming messages come in one load (a lane each) and eight rows
// are in flight at a time, so a variable costs a few round trips, not two per
// neighbour.  Shuffles and reductions stay inside the group, whose lanes run
// the same loop trips.
__global__ void k_marginals_generic(const int* node_ptr, const int* rev, const float* unary,
                                    const float* m, float* out, int N, int K) {
    constexpr int kRows = 8;
    const int lane = threadIdx.x & 63;
    int W = 1;
    while (W < K) W <<= 1;
    const int G = 64 / W;  // variables per wave
    const int sub = lane / W, x = lane % W, base = sub * W;
    const bool on = x < K;
    const float fK = (float)K;
    const long long waves = (long long)gridDim.x * (blockDim.x >> 6);
    const long long w0 = (long long)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    for (long long n0 = w0 * G; n0 < N; n0 += waves * G) {
        const int n = (int)(n0 + sub);
        if (n < N) {
            float acc = on ? unary[(long long)n * K + x] : -INFINITY;
            const int s0 = node_ptr[n], s1 = node_ptr[n + 1];
            for (int c = s0; c < s1; c += W) {
                const int cnt = min(W, s1 - c);
                const int r = x < cnt ? rev[c + x] : 0;
                for (int j = 0; j < cnt; j += kRows) {
                    float v[kRows];
#pragma unroll
                    for (int u = 0; u < kRows; ++u) {
                        const int ru = __shfl(r, base + (j + u) % W, 64);
                        v[u] = on && j + u < cnt ? m[(long long)ru * K + x] : 1.0f;
                    }
#pragma unroll
                    for (int u = 0; u < kRows; ++u)
                        if (on && j + u < cnt) acc += logf(fK * v[u]);
                }
            }
            float mx = acc;
            for (int o = W >> 1; o > 0; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o, 64));
            const float e = on ? expf(acc - mx) : 0.0f;
            float z = e;
            for (int o = W >> 1; o > 0; o >>= 1) z += __shfl_xor(z, o, 64);
            if (on) out[(long long)n * K + x] = e / z;
        }
    }
}

// ---------------------------------------------------------------------------
// Variables with their own numbers of states (ragged layout, Sec. II-A with
// K_i states per variable, as in the side-chain models of Sec. IV-E): the
// message i -> j holds K_j floats at moff[slot], the table of slot i -> j is
// K_i x K_j (x_i major) at toff[slot], the unary of i is K_i floats at uoff[i].
// Every slot has its own table, so Eq. (2) is a vector-matrix product whose
// table entries are each used once per iteration: 2 flops per 4-byte table
// entry, far below the ridge of the matrix cores and of the vector units, so
// the vector units take it and the kernel is bound by the table traffic.
//
// One wave per source variable (grid-stride): lane x holds the aggregate of
// states x and x + 64 (K_i <= 128); the cavity of each outgoing slot,
// g(x_i) = exp(A(x_i) - log m_{j->i}(x_i) - max), goes to LDS.  Then every
// (slot, target state) pair of the variable gets a lane, which takes the
// product with its slot's table as a chain of fused multiply-adds over the
// source states (the table entries of consecutive lanes are contiguous; a lane
// runs four pairs together, 32 loads in flight); a lane per slot forms the normalisation, the
// L-infinity residual and the frontier decision, and the pair lanes store the
// committed values.  A heavy variable (slots over the wave's LDS, or much
// product work: ragged_flat) gives each of its slots a wave of its own
// (ragged_slot), taken before the other variables, so the launch is not held
// up by one wave that runs a long chain of table loads.
// ---------------------------------------------------------------------------

// Wave-local LDS hand-off: this wave's LDS stores are complete and visible to
// its other lanes (a wave executes its LDS operations in order).
__device__ __forceinline__ void wave_lds_sync() { __asm__ volatile("s_waitcnt lgkmcnt(0)" ::: "memory"); }

// LDS per wave of the flat path: the cavity vectors of one variable's slots,
// and its slots' outputs (entries), each at most kRaggedFlat floats.

template <int MODE>
__device__ __forceinline__ void ragged_commit(const EvalArgs& a, int q, float v, float old, bool ka,
                                              bool kb) {
    if (MODE == kModeLBP) {
        a.out_buf[0][q] = v;
    } else if (MODE == kModeRnBP) {
        a.out_buf[0][q] = ka ? v : old;
        if (a.two_outputs) a.out_buf[1][q] = kb ? v : old;
    } else if (MODE == kModeRBP) {
        a.cand[q] = v;
    }
}

// One slot i -> j of a heavy variable on one wave: the aggregate of i over all
// its incoming rows (lanes over source states, rows eight at a time, summed in
// slot order as the flat path sums them), the cavity of j's row, then the
// product with the slot's table.  For K_j <= 64 the wave covers R = 64 / K_j
// table rows per step: lane r K_j + y reads entry (step R + r) K_j + y, so each
// load is one contiguous run of the table, eight steps in flight, and the R
// partial sums of each target state are added through LDS.  For larger K_j,
// lanes take target states y and y + 64 over all source states.
template <int MODE>
__device__ __forceinline__ void ragged_slot(const EvalArgs& a, const float* __restrict__ m_in, int s,
                                            int i, float* G, float* Cv, float& rmax,
                                            unsigned int& act, unsigned int& sa, unsigned int& sb) {
    const int lane = threadIdx.x & 63;
    const int Ki = a.kv[i];
    const int s0 = a.node_ptr[i], s1 = a.node_ptr[i + 1];
    const float fK = (float)Ki;
    const bool x0 = lane < Ki, x1 = lane + 64 < Ki;
    const float* U = a.unary + a.uoff[i];
    const int mo = a.moff[s], Kj = a.moff[s + 1] - mo;
    const float* __restrict__ T = a.pair + a.toff[s];
    const int rj = a.moff[a.rev[s]];
    const bool y0 = lane < Kj, y1 = lane + 64 < Kj;
    const float old0 = y0 ? m_in[mo + lane] : 0.0f;
    const float old1 = y1 ? m_in[mo + lane + 64] : 0.0f;
    float A0 = x0 ? U[lane] : 0.0f, A1 = x1 ? U[lane + 64] : 0.0f;
    for (int b = s0; b < s1; b += 64) {
        const int nb = min(64, s1 - b);
        const int my_rin = lane < nb ? a.moff[a.rev[b + lane]] : 0;
        for (int k0 = 0; k0 < nb; k0 += 8) {
            float v0[8], v1[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int rin = __shfl(my_rin, min(k0 + j, nb - 1), 64);
                v0[j] = x0 ? m_in[rin + lane] : 1.0f;
                v1[j] = x1 ? m_in[rin + lane + 64] : 1.0f;
            }
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                if (k0 + j >= nb) break;
                if (x0) A0 += logf(fK * v0[j]);
                if (x1) A1 += logf(fK * v1[j]);
            }
        }
    }
    const float c0 = x0 ? A0 - logf(fK * m_in[rj + lane]) : -INFINITY;
    const float c1 = x1 ? A1 - logf(fK * m_in[rj + lane + 64]) : -INFINITY;
    const float mx = wave_max_f(fmaxf(c0, c1));
    if (x0) G[lane] = expf(c0 - mx);
    if (x1) G[lane + 64] = expf(c1 - mx);
    wave_lds_sync();
    float o0 = 0.0f, o1 = 0.0f;
    if (Kj <= 64) {
        const int R = 64 / Kj;
        const int r = lane / Kj;
        const int RK = R * Kj;
        const int steps = (Ki + R - 1) / R;
        float acc = 0.0f;
        int st = 0;
        for (; st + 8 <= steps; st += 8) {
            float tv[8], gv[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int x = (st + u) * R + r;
                const bool ok = lane < RK && x < Ki;
                tv[u] = ok ? T[(st + u) * RK + lane] : 0.0f;
                gv[u] = ok ? G[x] : 0.0f;
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) acc = fmaf(tv[u], gv[u], acc);
        }
        if (st < steps) {
            // the remaining steps (fewer than eight), predicated, loads together
            float tv[8], gv[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int x = (st + u) * R + r;
                const bool ok = st + u < steps && lane < RK && x < Ki;
                tv[u] = ok ? T[(st + u) * RK + lane] : 0.0f;
                gv[u] = ok ? G[x] : 0.0f;
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) acc = fmaf(tv[u], gv[u], acc);
        }
        Cv[lane] = acc;
        wave_lds_sync();
        if (y0)
            for (int q = 0; q < R; ++q) o0 += Cv[q * Kj + lane];
    } else {
        int x = 0;
        for (; x + 8 <= Ki; x += 8) {
            float t0[8], t1[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                t0[u] = T[(x + u) * Kj + lane];
                t1[u] = y1 ? T[(x + u) * Kj + lane + 64] : 0.0f;
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const float gx = G[x + u];
                o0 = fmaf(t0[u], gx, o0);
                o1 = fmaf(t1[u], gx, o1);
            }
        }
        if (x < Ki) {
            float t0[8], t1[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const bool ok = x + u < Ki;
                t0[u] = ok ? T[(x + u) * Kj + lane] : 0.0f;
                t1[u] = ok && y1 ? T[(x + u) * Kj + lane + 64] : 0.0f;
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                if (x + u >= Ki) break;
                const float gx = G[x + u];
                o0 = fmaf(t0[u], gx, o0);
                o1 = fmaf(t1[u], gx, o1);
            }
        }
    }
    const float z = wave_sum_f(o0 + o1);
    o0 /= z;
    o1 /= z;
    const float res = wave_max_f(fmaxf(y0 ? fabsf(o0 - old0) : 0.0f, y1 ? fabsf(o1 - old1) : 0.0f));
    const bool active = res > a.eps;
    bool ka = false, kb = false;
    if (MODE == kModeRnBP && active) {
        const unsigned int u24 = draw24(a, i, s - s0);
        ka = u24 < a.thr_a;
        kb = u24 < a.thr_b;
    }
    if (y0) ragged_commit<MODE>(a, mo + lane, o0, old0, ka, kb);
    if (y1) ragged_commit<MODE>(a, mo + lane + 64, o1, old1, ka, kb);
    if (lane == 0) {
        if (MODE == kModeRBP) a.keys[s] = __float_as_uint(res);
        act += active;
        sa += ka;
        sb += kb;
        rmax = fmaxf(rmax, res);
    }
    wave_lds_sync();  // G and Cv are free for the wave's next slot
}

// Four waves per SIMD: 124 to 127 registers, none spilled (three waves and up
// to 141 registers unconstrained).
template <int MODE>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4))) void k_eval_ragged(
    EvalArgs a) {
    __shared__ RedScratch red;
    __shared__ unsigned long long s_red[2];
    __shared__ float s_g[kBlock / 64][kRaggedFlat];    // cavity vectors, slot-major
    __shared__ float s_c[kBlock / 64][kRaggedFlat];    // outputs of the variable's slots
    __shared__ int s_off[kBlock / 64][kRaggedMaxDeg + 1];
    __shared__ int s_rin[kBlock / 64][kRaggedMaxDeg];    // row of the message into the variable
    __shared__ int s_toff[kBlock / 64][kRaggedMaxDeg];   // table of the slot
    __shared__ float s_inv[kBlock / 64][kRaggedMaxDeg];
    __shared__ unsigned int s_keep[kBlock / 64][kRaggedMaxDeg];
    const float* __restrict__ m_in = iteration_prologue(a, s_red, blockIdx.x == 0);
    if (!m_in) return;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    float* G = s_g[w];
    float* Cv = s_c[w];
    int* off = s_off[w];
    const int waves = (int)(gridDim.x * (blockDim.x >> 6));
    float rmax = 0.0f;
    unsigned int act = 0, sa = 0, sb = 0;
    const int gw = (int)(blockIdx.x * (blockDim.x >> 6) + w);
    for (int h = gw; h < a.num_heavy; h += waves)
        ragged_slot<MODE>(a, m_in, a.heavy[2 * h], a.heavy[2 * h + 1], G, Cv, rmax, act, sa, sb);
    for (int i = gw; i < a.num_nodes; i += waves) {
        const int Ki = a.kv[i];
        const int s0 = a.node_ptr[i], s1 = a.node_ptr[i + 1];
        const int deg = s1 - s0;
        const float* U = a.unary + a.uoff[i];
        const float fK = (float)Ki;  // log(K_i m) keeps the aggregate near zero
        const bool x0 = lane < Ki, x1 = lane + 64 < Ki;
        float A0 = x0 ? U[lane] : 0.0f, A1 = x1 ? U[lane + 64] : 0.0f;
        const int mo0 = a.moff[s0];
        const int P = a.moff[s1] - mo0;  // outputs of all slots of the variable
        if (!ragged_flat(deg, Ki, P)) continue;  // a heavy variable: its slots are done
        {
            // Flat path.  A lane per slot fetches the slot's offsets (all in
            // flight at once); the incoming rows are loaded eight slots at a
            // time and their logs kept in LDS for the cavities; then the
            // outputs of all slots at once (a lane per (slot, target state)
            // pair), the per-slot sums, residuals and frontier decisions (a
            // lane per slot), and the stores.
            for (int k = lane; k < deg; k += 64) {
                s_rin[w][k] = a.moff[a.rev[s0 + k]];
                s_toff[w][k] = a.toff[s0 + k];
                off[k] = a.moff[s0 + k] - mo0;
            }
            if (lane == 0) off[deg] = P;
            wave_lds_sync();
            for (int k0 = 0; k0 < deg; k0 += 8) {
                float v0[8], v1[8];
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const int k = min(k0 + j, deg - 1);
                    const int rin = s_rin[w][k];
                    v0[j] = x0 ? m_in[rin + lane] : 1.0f;
                    v1[j] = x1 ? m_in[rin + lane + 64] : 1.0f;
                }
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    if (k0 + j >= deg) break;
                    const float l0 = logf(fK * v0[j]), l1 = logf(fK * v1[j]);
                    if (x0) {
                        A0 += l0;
                        G[(k0 + j) * Ki + lane] = l0;
                    }
                    if (x1) {
                        A1 += l1;
                        G[(k0 + j) * Ki + lane + 64] = l1;
                    }
                }
            }
            wave_lds_sync();
            for (int k = 0; k < deg; ++k) {
                const float c0 = x0 ? A0 - G[k * Ki + lane] : -INFINITY;
                const float c1 = x1 ? A1 - G[k * Ki + lane + 64] : -INFINITY;
                const float mx = wave_max_f(fmaxf(c0, c1));
                if (x0) G[k * Ki + lane] = expf(c0 - mx);
                if (x1) G[k * Ki + lane + 64] = expf(c1 - mx);
            }
            wave_lds_sync();
            // up to four pairs per lane at once (p, p + 64, p + 128, p + 192):
            // their table loads are independent, so 4 x 8 are in flight
            for (int pb = 0; pb < P; pb += 256) {
                const float* T[4];
                const float* g[4];
                int Kj[4];
                bool on[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int p = pb + lane + 64 * j;
                    on[j] = p < P;
                    const int pp = on[j] ? p : P - 1;
                    int k = 0;
                    while (off[k + 1] <= pp) ++k;
                    Kj[j] = off[k + 1] - off[k];
                    T[j] = a.pair + s_toff[w][k] + (pp - off[k]);
                    g[j] = G + k * Ki;
                }
                float acc[4] = {0.0f, 0.0f, 0.0f, 0.0f};
                // eight source states per step, the last step predicated (a
                // variable with few states takes one step, not one per state)
                for (int x = 0; x < Ki; x += 8) {
                    float tv[4][8];
#pragma unroll
                    for (int j = 0; j < 4; ++j)
#pragma unroll
                        for (int u = 0; u < 8; ++u) tv[j][u] = x + u < Ki ? T[j][(x + u) * Kj[j]] : 0.0f;
#pragma unroll
                    for (int j = 0; j < 4; ++j)
#pragma unroll
                        for (int u = 0; u < 8; ++u)
                            if (x + u < Ki) acc[j] = fmaf(tv[j][u], g[j][x + u], acc[j]);
                }
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    if (on[j]) Cv[pb + lane + 64 * j] = acc[j];
            }
            wave_lds_sync();
            for (int k = lane; k < deg; k += 64) {
                float z = 0.0f;
                for (int q = off[k]; q < off[k + 1]; ++q) z += Cv[q];
                s_inv[w][k] = 1.0f / z;
            }
            wave_lds_sync();
            // normalised outputs back into Cv, |change| into G (cavities are done)
            for (int p = lane; p < P; p += 64) {
                int k = 0;
                while (off[k + 1] <= p) ++k;
                const float v = Cv[p] * s_inv[w][k];
                Cv[p] = v;
                G[p] = fabsf(v - m_in[mo0 + p]);
            }
            wave_lds_sync();
            for (int k = lane; k < deg; k += 64) {
                float r = 0.0f;
                for (int q = off[k]; q < off[k + 1]; ++q) r = fmaxf(r, G[q]);
                const bool active = r > a.eps;
                bool ka = false, kb = false;
                if (MODE == kModeRnBP && active) {
                    const unsigned int u24 = draw24(a, i, k);
                    ka = u24 < a.thr_a;
                    kb = u24 < a.thr_b;
                }
                if (MODE == kModeRBP) a.keys[s0 + k] = __float_as_uint(r);
                s_keep[w][k] = (ka ? 1u : 0u) | (kb ? 2u : 0u);
                act += active;
                sa += ka;
                sb += kb;
                rmax = fmaxf(rmax, r);
            }
            wave_lds_sync();
            for (int p = lane; p < P; p += 64) {
                int k = 0;
                while (off[k + 1] <= p) ++k;
                const unsigned int kp = s_keep[w][k];
                const float old = MODE == kModeRnBP ? m_in[mo0 + p] : 0.0f;
                ragged_commit<MODE>(a, mo0 + p, Cv[p], old, kp & 1u, kp & 2u);
            }
            wave_lds_sync();  // the wave's LDS is free for its next variable
        }
    }
    block_accumulate(&red, a.ctr, a.t, rmax, act, sa, sb);
}

// Eq. (3) for the ragged layout: one wave per variable.
__global__ __launch_bounds__(kBlock) void k_marginals_ragged(EvalArgs a, float* out) {
    const float* __restrict__ m = a.in_buf[0];
    const int lane = threadIdx.x & 63;
    const int waves = (int)(gridDim.x * (blockDim.x >> 6));
    for (int i = (int)(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)); i < a.num_nodes;
         i += waves) {
        const int Ki = a.kv[i];
        const float* U = a.unary + a.uoff[i];
        const float fK = (float)Ki;
        const bool x0 = lane < Ki, x1 = lane + 64 < Ki;
        float A0 = x0 ? U[lane] : -INFINITY, A1 = x1 ? U[lane + 64] : -INFINITY;
        for (int s = a.node_ptr[i]; s < a.node_ptr[i + 1]; ++s) {
            const int rin = a.moff[a.rev[s]];
            if (x0) A0 += logf(fK * m[rin + lane]);
            if (x1) A1 += logf(fK * m[rin + lane + 64]);
        }
        const float mx = wave_max_f(fmaxf(A0, A1));
        const float e0 = x0 ? expf(A0 - mx) : 0.0f, e1 = x1 ? expf(A1 - mx) : 0.0f;
        const float z = wave_sum_f(e0 + e1);
        if (x0) out[a.uoff[i] + lane] = e0 / z;
        if (x1) out[a.uoff[i] + lane + 64] = e1 / z;
    }
}

// The uniform start state: 1 / K_j in every entry of message i -> j.
__global__ void k_fill_ragged(float* m, const int* moff, int E) {
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < E; e += gridDim.x * blockDim.x) {
        const int q0 = moff[e], q1 = moff[e + 1];
        const float v = 1.0f / (float)(q1 - q0);
        for (int q = q0; q < q1; ++q) m[q] = v;
    }
}

// ---------------------------------------------------------------------------
// Sparse re-evaluation (K = 2 log-odds layout, RnBP), messages committed in
// place.  The candidate of Eq. (2) for i -> j depends only on the messages into
// i (and on i's own old value for the residual), so after a commit only the
// messages out of nodes that received a committed message ("dirty" nodes) can
// change.  Every other stored candidate and residual is, bit for bit, what a
// full evaluation would compute again: the same arithmetic on the same inputs,
// and a committed message whose source is clean has candidate = message and
// residual 0.
//
// n_t is carried as a running count: the evaluation adds, per re-evaluated
// slot, (new residual > eps) - (old residual > eps), and the commit subtracts
// the committed slots; both add into counter set t & 3 of the iteration whose
// count they change, and the commit of iteration t reads
// n_t = n_{t-1} + (sum of set t & 3).  R_t is only reported for the last
// evaluation of a run, so it is taken once, over the stored residuals, after
// the run.  A node flag records whether any of the node's slots is active, so
// the commit visits only such nodes.
// ---------------------------------------------------------------------------
constexpr int kSparseChunk = 4;  // slots per group of loads (= words of one Philox call)
constexpr int kSparseGridMax = 1024;  // blocks of the residual-max pass

__device__ __forceinline__ int sparse_grid_stride() { return (int)(gridDim.x * blockDim.x); }

// Block sum of a signed and an unsigned per-thread count, added into counter
// copy (blockIdx & 63) of set `set`: the signed one into its active count
// (wrapping modulo 2^64), the unsigned one into sel_a (evaluated slots) or,
// with `committed`, into sel_b.
__device__ __forceinline__ void sparse_accumulate(CounterLine* ctr, unsigned int set, int d,
                                                  unsigned int ev, int* s_d, unsigned int* s_ev,
                                                  bool committed) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        d += __shfl_xor(d, o, 64);
        ev += __shfl_xor(ev, o, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        s_d[threadIdx.x >> 6] = d;
        s_ev[threadIdx.x >> 6] = ev;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        long long D = 0;
        unsigned long long EV = 0;
        for (int w = 0; w < kBlock / 64; ++w) {
            D += s_d[w];
            EV += s_ev[w];
        }
        CounterLine* c = ctr + (set & 3u) * kCounterCopies + (blockIdx.x & (kCounterCopies - 1));
        if (D) atomicAdd(&c->active, (unsigned long long)D);
        if (EV) atomicAdd(committed ? &c->sel_b : &c->sel_a, EV);
    }
}

// Operands of up to four consecutive slots c .. c+3 of a node ending at s1
// (indices clamped into the node, so the loads are unconditional).
struct SparseChunk {
    float lin[kSparseChunk], J[kSparseChunk], old[kSparseChunk];
    unsigned int key[kSparseChunk];
};

__device__ __forceinline__ void sparse_load_lin(const EvalArgs& a, const float* m, int c, int s1,
                                                float* lin) {
#pragma unroll
    for (int k = 0; k < kSparseChunk; ++k) lin[k] = m[a.rev[min(c + k, s1 - 1)]];
}

__device__ __forceinline__ void sparse_load_chunk(const EvalArgs& a, const float* m, int c, int s1,
                                                  SparseChunk& d) {
#pragma unroll
    for (int k = 0; k < kSparseChunk; ++k) {
        const int e = min(c + k, s1 - 1);
        d.lin[k] = m[a.rev[e]];
        d.J[k] = a.coupling[e];
        d.old[k] = m[e];
        d.key[k] = a.keys[e];
    }
}

__device__ __forceinline__ void sparse_eval_chunk(const EvalArgs& a, float L, int c, int s1,
                                                  const SparseChunk& d, unsigned int& act,
                                                  unsigned int& old_act) {
    unsigned int unused = 0;
#pragma unroll
    for (int k = 0; k < kSparseChunk; ++k) {
        if (c + k >= s1) break;
        old_act += (!a.sp_first && __uint_as_float(d.key[k]) > a.eps) ? 1u : 0u;
        logodds_slot<kModeRBP>(a, OutPtr{a}, L, d.lin[k], d.J[k], d.old[k], c + k, 0u, act, unused,
                               unused);
    }
}

// Iteration t, evaluation: the slots of every dirty node are evaluated again
// (the incoming messages are summed in slot order, as the tiled kernel sums
// them; operands are loaded four slots at a time, and a node of at most four
// slots is evaluated from one set of loads).  sp_first: the first sparse
// iteration of a run, whose stored residuals are not yet valid (counted as 0).
__global__ __launch_bounds__(kBlock) void k_sparse_eval(EvalArgs a) {
    __shared__ int s_d[kBlock / 64];
    __shared__ unsigned int s_ev[kBlock / 64];
    if (a.st->done) return;
    const float* __restrict__ m = a.in_buf[0];
    int delta = 0;
    unsigned int ev = 0;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < a.num_nodes; i += sparse_grid_stride()) {
        if (!a.dirty[i]) continue;
        a.dirty[i] = 0;
        const int s0 = a.node_ptr[i], s1 = a.node_ptr[i + 1];
        const float u = a.unary[i];
        unsigned int act = 0, old_act = 0;
        if (s1 > s0) {
            SparseChunk d;
            sparse_load_chunk(a, m, s0, s1, d);
            float L = u;
#pragma unroll
            for (int k = 0; k < kSparseChunk; ++k)
                if (s0 + k < s1) L += d.lin[k];
            for (int c = s0 + kSparseChunk; c < s1; c += kSparseChunk) {
                float lin[kSparseChunk];
                sparse_load_lin(a, m, c, s1, lin);
#pragma unroll
                for (int k = 0; k < kSparseChunk; ++k)
                    if (c + k < s1) L += lin[k];
            }
            sparse_eval_chunk(a, L, s0, s1, d, act, old_act);
            for (int c = s0 + kSparseChunk; c < s1; c += kSparseChunk) {
                sparse_load_chunk(a, m, c, s1, d);
                sparse_eval_chunk(a, L, c, s1, d, act, old_act);
            }
        }
        a.hasact[i] = act ? 1 : 0;
        delta += (int)act - (int)old_act;
        ev += (unsigned int)(s1 - s0);
    }
    sparse_accumulate(a.ctr, a.t, delta, ev, s_d, s_ev, false);
}

// Iteration t, commit.  Every block forms n_t and n_{t-1} and takes p_t from
// EdgeRatio = n_t / n_{t-1} (Sec. IV-A); block 0 also closes evaluation t
// (IsConverged, statistics including the commits of iteration t - 1, n_t kept
// for the next iteration) and clears counter set t + 2.  Then the active slots of flagged nodes are drawn (the
// same Philox words as the tiled kernel, one call per four slots) and the kept
// ones committed in place; their targets are marked dirty.  After the last
// allowed commit (after_final) the evaluation is closed and nothing committed.
// Each thread takes one node; its flag, slot range and first four residuals
// are loaded before the counters are summed, so the two latencies overlap.
__global__ __launch_bounds__(kBlock) void k_sparse_commit(EvalArgs a) {
    __shared__ unsigned long long s_n[3];
    __shared__ int s_d[kBlock / 64];
    __shared__ unsigned int s_ev[kBlock / 64];
    const int i = blockIdx.x * kBlock + threadIdx.x;
    const bool mine = i < a.num_nodes && a.hasact[i];
    int s0 = 0, s1 = 0;
    unsigned int key[kSparseChunk] = {0u, 0u, 0u, 0u};
    if (mine) {
        s0 = a.node_ptr[i];
        s1 = a.node_ptr[i + 1];
#pragma unroll
        for (int k = 0; k < kSparseChunk; ++k) key[k] = a.keys[min(s0 + k, s1 - 1)];
    }
    // wave 0 reads the done flag once for the block (block 0 may set it during
    // this launch, so the other waves must not read it themselves)
    if (threadIdx.x < 64) {
        const int lane = threadIdx.x;
        const unsigned int done = a.st->done;
        const CounterLine* c0 = a.ctr + (a.t & 3u) * kCounterCopies + lane;
        const long long d = (long long)wave_sum64(c0->active);
        const long long base = a.sp_first ? 0ll : (long long)a.st->sp_n[(a.t - 1u) & 3u];
        const unsigned long long n1 = (unsigned long long)(base + d);
        long long n2;
        if (!a.sp_first)
            n2 = (long long)a.st->sp_n[(a.t - 1u) & 3u];
        else if (a.it >= 1)  // switched from the full evaluation: its count of t - 1
            n2 = (long long)wave_sum64(a.ctr[((a.t - 1u) & 3u) * kCounterCopies + lane].active);
        else
            n2 = a.prev_active_host;
        if (blockIdx.x == 0 && !done) {
            const unsigned long long ev = wave_sum64(c0->sel_a);
            // messages committed by iteration t - 1 (none on the first sparse iteration)
            const unsigned long long cm_prev = a.sp_first ? 0ull : wave_sum64(c0->sel_b);
            CounterLine* z = a.ctr + ((a.t + 2u) & 3u) * kCounterCopies + lane;
            z->active = 0ull;
            z->sel_a = 0ull;
            z->sel_b = 0ull;
            z->rmax = 0u;
            if (lane == 0) {
                DevState* st = a.st;
                atomicAdd(&st->evaluated, ev);
                atomicAdd(&st->evals, 1ull);
                if (cm_prev) atomicAdd(&st->committed, cm_prev);
                st->sp_n[a.t & 3u] = n1;
                st->last_t = (long long)a.t;
                st->last_active = n1;
                st->last_rmax = 0u;  // taken after the run
                st->last_prev = n2;
                if (n1 == 0ull) {
                    st->done = 1u;
                    st->conv_t = (long long)a.t;
                } else if (!a.after_final) {
                    atomicAdd(&st->iterations, 1ull);
                }
            }
        }
        if (lane == 0) {
            s_n[0] = n1;
            s_n[1] = (unsigned long long)n2;
            s_n[2] = done;
        }
    }
    __syncthreads();
    const unsigned long long n1 = s_n[0];
    if (s_n[2] || n1 == 0ull || a.after_final) return;
    const unsigned int thr = select_outcome(a, n1, (long long)s_n[1]) ? a.thr_b : a.thr_a;
    float* __restrict__ m = a.out_buf[0];
    unsigned int cm = 0;
    if (mine) {
        unsigned int left = 0;
        for (int c = s0; c < s1; c += kSparseChunk) {
            if (c != s0) {
#pragma unroll
                for (int k = 0; k < kSparseChunk; ++k) key[k] = a.keys[min(c + k, s1 - 1)];
            }
            bool any = false;
#pragma unroll
            for (int k = 0; k < kSparseChunk; ++k)
                any |= c + k < s1 && __uint_as_float(key[k]) > a.eps;
            if (!any) continue;
            const uint4 w = philox4((unsigned int)i, (unsigned int)(c - s0) >> 2, a.t, a.key0, a.key1);
            const unsigned int u[kSparseChunk] = {w.x >> 8, w.y >> 8, w.z >> 8, w.w >> 8};
            bool take[kSparseChunk];
            float cv[kSparseChunk];
            int dv[kSparseChunk];
#pragma unroll
            for (int k = 0; k < kSparseChunk; ++k) {
                const bool act = c + k < s1 && __uint_as_float(key[k]) > a.eps;
                take[k] = act && u[k] < thr;
                left += act && !take[k];
                if (take[k]) {
                    cv[k] = a.cand[c + k];
                    dv[k] = a.dst[c + k];
                }
            }
#pragma unroll
            for (int k = 0; k < kSparseChunk; ++k) {
                if (!take[k]) continue;
                m[c + k] = cv[k];
                a.keys[c + k] = 0u;
                a.dirty[dv[k]] = 1;
                ++cm;
            }
        }
        if (!left) a.hasact[i] = 0;
    }
    // the committed slots leave the count of iteration t + 1; their number is
    // added to the statistics when iteration t + 1 is closed
    sparse_accumulate(a.ctr, a.t + 1u, -(int)cm, cm, s_d, s_ev, true);
}

// Per-graph setup: the target of each slot (slot rev[e] carries the reverse
// message, whose target is the source of e), then every node dirty.
__global__ __launch_bounds__(kBlock) void k_sparse_setup(EvalArgs a, int build_dst) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= a.num_nodes) return;
    if (build_dst) {
        for (int e = a.node_ptr[i]; e < a.node_ptr[i + 1]; ++e) a.dst[a.rev[e]] = i;
    }
    a.dirty[i] = 1;
}

// After a sparse run: R_t of its last evaluation, the largest stored residual
// (no commit followed that evaluation, so the stored residuals are its own).
// One atomic per block.
__global__ __launch_bounds__(kBlock) void k_sparse_rmax(EvalArgs a) {
    __shared__ unsigned int s_r[kBlock / 64];
    unsigned int r = 0;
    for (long long e = (long long)blockIdx.x * kBlock + threadIdx.x; e < (long long)a.num_messages;
         e += (long long)gridDim.x * kBlock)
        r = max(r, a.keys[e]);
    r = wave_max32(r);
    if ((threadIdx.x & 63) == 0) s_r[threadIdx.x >> 6] = r;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kBlock / 64; ++w) r = max(r, s_r[w]);
        if (r) atomicMax(&a.st->last_rmax, r);
    }
}

// ---------------------------------------------------------------------------
// Greedy top-k for frontier residual BP: most-significant-digit radix select
// over the FP32 bit patterns of the residuals (monotone for values >= 0),
// 4 passes of 8 bits, then a commit that takes every key above the threshold
// and the lowest-slot keys equal to it (slots are ordered by (target, source)).
// ---------------------------------------------------------------------------
constexpr int kSelBlock = 256;
constexpr int kCommitChunk = 4096;

// IsConverged for the top-k step: nothing is selected or committed when the
// evaluation of iteration t found no residual above eps.
__global__ void k_rbp_gate(DevState* st, const CounterLine* ctr, int slot) {
    const unsigned long long n = wave_sum64(ctr[slot * kCounterCopies + threadIdx.x].active);
    if (threadIdx.x == 0) st->rbp_skip = (st->done || n == 0ull) ? 1u : 0u;
}

// Keys per thread of a histogram pass and positions per thread of the tie
// count and the commit: loaded as four 16-byte vectors, so that a thread's
// loads are all in flight at once.
constexpr int kSelPer = 16;
constexpr int kHistCopies = 16;  // copies of the global digit histogram
static_assert(kCommitChunk == kSelBlock * kSelPer, "one commit chunk per block");

// The keys (or slot indices) base[q0 .. q0+15], clamped to n (entries past n
// are left unchanged).  base is 16-byte aligned (arena offsets are multiples
// of 256 bytes).
template <class T>
__device__ __forceinline__ void sel_load16(const T* base, long long q0, long long n, T* v) {
    if (q0 + kSelPer <= n) {
        const uint4* p = (const uint4*)(base + q0);
#pragma unroll
        for (int j = 0; j < kSelPer / 4; ++j) {
            const uint4 w = p[j];
            v[4 * j + 0] = (T)w.x;
            v[4 * j + 1] = (T)w.y;
            v[4 * j + 2] = (T)w.z;
            v[4 * j + 3] = (T)w.w;
        }
    } else {
#pragma unroll
        for (int j = 0; j < kSelPer; ++j)
            if (q0 + j < n) v[j] = base[q0 + j];
    }
}

// Digit histogram of pass `pass` (8 bits from the top) of the keys matching
// the prefix fixed so far, over the chunks of kCommitChunk keys this block
// takes (grid-stride), added into one of kHistCopies copies of the global
// histogram (by block index) so that blocks do not queue on one address.
__device__ __forceinline__ void rbp_hist_block(const DevState* st, const unsigned int* keys, int E,
                                               int pass, unsigned int* ghist, unsigned int* h) {
    h[threadIdx.x] = 0u;
    __syncthreads();
    const unsigned int prefix = pass ? st->sel_prefix : 0u;
    const unsigned int mask = pass ? st->sel_mask : 0u;
    const int shift = 24 - 8 * pass;
    const int chunks = (E + kCommitChunk - 1) / kCommitChunk;
    for (int c = blockIdx.x; c < chunks; c += gridDim.x) {
        const long long q0 = (long long)c * kCommitChunk + (long long)threadIdx.x * kSelPer;
        unsigned int v[kSelPer];
        sel_load16(keys, q0, (long long)E, v);
#pragma unroll
        for (int j = 0; j < kSelPer; ++j)
            lds_count(h, (v[j] >> shift) & 255u, q0 + j < E && (v[j] & mask) == prefix);
    }
    __syncthreads();
    if (h[threadIdx.x])
        atomicAdd(&ghist[(blockIdx.x & (kHistCopies - 1)) * 256 + threadIdx.x], h[threadIdx.x]);
}

// Pick the digit of pass `pass` (one block): the largest b whose suffix count
// S(b) (keys with digit >= b) reaches the number still to take, digit 0 if
// none; clear the histogram copies for the next pass.
__device__ __forceinline__ void rbp_scan_block(DevState* st, int pass, unsigned int k,
                                               unsigned int* ghist, unsigned int* h) {
    const int b = threadIdx.x;
    unsigned int hb = 0;
#pragma unroll
    for (int c = 0; c < kHistCopies; ++c) {
        hb += ghist[c * 256 + b];
        ghist[c * 256 + b] = 0u;
    }
    h[b] = hb;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
        const unsigned int add = b + o < 256 ? h[b + o] : 0u;
        __syncthreads();
        h[b] += add;
        __syncthreads();
    }
    const unsigned int krem = pass ? st->sel_krem : k;
    const unsigned int S = h[b];
    const unsigned int S1 = b < 255 ? h[b + 1] : 0u;
    const bool pick = b == 0 ? S1 < krem : (S >= krem && S1 < krem);
    if (pick) {
        const unsigned int prefix = pass ? st->sel_prefix : 0u;
        const unsigned int mask = pass ? st->sel_mask : 0u;
        const int shift = 24 - 8 * pass;
        const unsigned int left = krem - S1;
        st->sel_prefix = prefix | ((unsigned int)b << shift);
        st->sel_mask = mask | (0xFFu << shift);
        st->sel_krem = left;
        if (pass == 3) {
            st->sel_ties = hb;
            st->sel_rank_ties = (hb != left) ? 1u : 0u;
        }
    }
}

// One histogram pass (a block per chunk of kCommitChunk keys).
__global__ __launch_bounds__(kSelBlock) void k_rbp_hist(DevState* st, const unsigned int* keys,
                                                        int E, int pass) {
    __shared__ unsigned int h[256];
    if (st->rbp_skip) return;
    rbp_hist_block(st, keys, E, pass, &st->hist[0][0], h);
}

// The digit pick of pass `pass`.  With gate_ctr (first pass only) it is also
// IsConverged for the top-k: nothing is selected or committed when the
// evaluation found no residual above eps (the copies that evaluation filled
// are then left for the next run's reset).
__global__ __launch_bounds__(kSelBlock) void k_rbp_scan(DevState* st, int pass, unsigned int k,
                                                        const CounterLine* gate_ctr) {
    __shared__ unsigned int h[256];
    __shared__ unsigned int s_skip;
    if (gate_ctr) {
        if (threadIdx.x < 64) {
            const unsigned long long n = wave_sum64(gate_ctr[threadIdx.x].active);
            if (threadIdx.x == 0) {
                s_skip = (st->done || n == 0ull) ? 1u : 0u;
                st->rbp_skip = s_skip;
            }
        }
    } else if (threadIdx.x == 0) {
        s_skip = st->rbp_skip;
    }
    __syncthreads();
    if (s_skip) return;
    rbp_scan_block(st, pass, k, &st->hist[0][0], h);
}

// Ties at the threshold key are taken in (target, source) order.  Slots are
// ordered by (source, target), so position p visits the message in slot rev[p],
// whose (target, source) is the (source, target) of slot p: walking positions
// in order walks tied messages in (target, source) order.  Without rev the
// positions are the keys' indices (residual splash ranks tied variables by id).
// Each block counts the ties among its kCommitChunk positions.
__global__ __launch_bounds__(kSelBlock) void k_rbp_tiecount(DevState* st, const unsigned int* keys,
                                                            const int* rev, int E,
                                                            unsigned int* block_ties) {
    __shared__ unsigned int part[kSelBlock / 64];
    if (st->rbp_skip || !st->sel_rank_ties) return;
    const unsigned int T = st->sel_prefix;
    const long long q0 = (long long)blockIdx.x * kCommitChunk + (long long)threadIdx.x * kSelPer;
    unsigned int c = 0;
    if (rev) {
        int e[kSelPer];
        sel_load16(rev, q0, (long long)E, e);
#pragma unroll
        for (int j = 0; j < kSelPer; ++j)
            if (q0 + j < E) c += keys[e[j]] == T;
    } else {
        // positions are the keys' own indices (variables of residual splash)
        unsigned int kv[kSelPer];
        sel_load16(keys, q0, (long long)E, kv);
#pragma unroll
        for (int j = 0; j < kSelPer; ++j)
            if (q0 + j < E) c += kv[j] == T;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned int sum = 0;
        for (int i = 0; i < kSelBlock / 64; ++i) sum += part[i];
        block_ties[blockIdx.x] = sum;
    }
}

// Exclusive prefix sums of the nb block tie counts, in place (one block: each
// thread takes a contiguous run, the run totals are scanned in LDS).
__global__ __launch_bounds__(kSelBlock) void k_rbp_tiescan(DevState* st, unsigned int* block_ties,
                                                           int nb) {
    __shared__ unsigned int part[kSelBlock];
    if (st->rbp_skip || !st->sel_rank_ties) return;
    const int per = (nb + kSelBlock - 1) / kSelBlock;
    const int r0 = threadIdx.x * per, r1 = min(nb, r0 + per);
    unsigned int run = 0;
    for (int i = r0; i < r1; ++i) run += block_ties[i];
    part[threadIdx.x] = run;
    __syncthreads();
    for (int o = 1; o < kSelBlock; o <<= 1) {
        const unsigned int add = threadIdx.x >= (unsigned)o ? part[threadIdx.x - o] : 0u;
        __syncthreads();
        part[threadIdx.x] += add;
        __syncthreads();
    }
    unsigned int acc = part[threadIdx.x] - run;
    for (int i = r0; i < r1; ++i) {
        const unsigned int v = block_ties[i];
        block_ties[i] = acc;
        acc += v;
    }
}

// Commit the frontier: every key above the threshold, and among keys equal to
// it the first sel_krem in position order (ranked ties) or all of them.  A
// thread takes kSelPer consecutive positions; the ties before it come from an
// exclusive scan over the block's threads plus the block's offset.
__global__ __launch_bounds__(kSelBlock) void k_rbp_commit(DevState* st, unsigned int* keys,
                                                          const int* rev, const float* cand,
                                                          float* m, int E, int row, int all,
                                                          const unsigned int* block_ties,
                                                          RbpSparse sp, const int* moff) {
    __shared__ unsigned int part[kSelBlock / 64];
    __shared__ unsigned int s_cm[kSelBlock / 64];
    if (st->rbp_skip) return;
    const unsigned int T = st->sel_prefix;
    const bool rank = !all && st->sel_rank_ties;
    const unsigned int krem = st->sel_krem;
    const long long q0 = (long long)blockIdx.x * kCommitChunk + (long long)threadIdx.x * kSelPer;
    int e[kSelPer];
    if (rank) {
        sel_load16(rev, q0, (long long)E, e);
    } else {
#pragma unroll
        for (int j = 0; j < kSelPer; ++j) e[j] = (int)(q0 + j);
    }
    unsigned int take = 0, tie = 0;  // bit j: position q0 + j
    unsigned int kv[kSelPer];
    if (all) {
#pragma unroll
        for (int j = 0; j < kSelPer; ++j)
            if (q0 + j < E) take |= 1u << j;
        if (sp.on) sel_load16(keys, q0, (long long)E, kv);
    } else {
        if (rank) {
#pragma unroll
            for (int j = 0; j < kSelPer; ++j) kv[j] = q0 + j < E ? keys[e[j]] : 0u;
        } else {
            sel_load16(keys, q0, (long long)E, kv);  // positions are slots: contiguous
        }
#pragma unroll
        for (int j = 0; j < kSelPer; ++j) {
            if (q0 + j >= E) continue;
            if (kv[j] > T) take |= 1u << j;
            if (kv[j] == T) tie |= 1u << j;
        }
        if (!rank) take |= tie;
    }
    if (rank) {
        // ties before this thread: inclusive scan within the wave, then the
        // totals of the lower waves
        const unsigned int c = (unsigned int)__popc(tie);
        const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
        unsigned int x = c;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const unsigned int y = (unsigned int)__shfl_up((int)x, o, 64);
            if (lane >= o) x += y;
        }
        if (lane == 63) part[w] = x;
        __syncthreads();
        unsigned int before = block_ties[blockIdx.x] + x - c;
        for (int i = 0; i < w; ++i) before += part[i];
#pragma unroll
        for (int j = 0; j < kSelPer; ++j) {
            if (!(tie >> j & 1u)) continue;
            if (before < krem) take |= 1u << j;
            ++before;
        }
    }
    unsigned int cm = 0;  // committed messages whose residual was above eps
    if (take && row == 1) {
        float cv[kSelPer];
#pragma unroll
        for (int j = 0; j < kSelPer; ++j)
            if (take >> j & 1u) cv[j] = cand[e[j]];
#pragma unroll
        for (int j = 0; j < kSelPer; ++j)
            if (take >> j & 1u) m[e[j]] = cv[j];
        if (sp.on) {
            // sparse re-evaluation: the committed message's residual is 0 until
            // its source is evaluated again; its target is evaluated again
            int dv[kSelPer];
#pragma unroll
            for (int j = 0; j < kSelPer; ++j)
                if (take >> j & 1u) dv[j] = sp.dst[e[j]];
#pragma unroll
            for (int j = 0; j < kSelPer; ++j) {
                if (!(take >> j & 1u)) continue;
                cm += __uint_as_float(kv[j]) > sp.eps ? 1u : 0u;
                keys[e[j]] = 0u;
                sp.dirty[dv[j]] = 1;
            }
        }
    } else if (take && moff) {
        // ragged rows: slot e's K_j values at moff[e]
#pragma unroll
        for (int j = 0; j < kSelPer; ++j)
            if (take >> j & 1u)
                for (int q = moff[e[j]]; q < moff[e[j] + 1]; ++q) m[q] = cand[q];
    } else if (take) {
#pragma unroll
        for (int j = 0; j < kSelPer; ++j)
            if (take >> j & 1u)
                for (int x = 0; x < row; ++x)
                    m[(long long)e[j] * row + x] = cand[(long long)e[j] * row + x];
    }
    if (sp.on) {
        // the committed active messages leave the running count of the next iteration
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) cm += __shfl_xor(cm, o, 64);
        if ((threadIdx.x & 63) == 0) s_cm[threadIdx.x >> 6] = cm;
        __syncthreads();
        if (threadIdx.x == 0) {
            unsigned int c = 0;
            for (int w = 0; w < kSelBlock / 64; ++w) c += s_cm[w];
            CounterLine* z = sp.ctr + (unsigned)sp.set * kCounterCopies +
                             (blockIdx.x & (kCounterCopies - 1));
            if (c) atomicAdd(&z->active, (unsigned long long)(-(long long)c));
        }
    }
}

// Frontier residual BP with sparse re-evaluation: close evaluation t after
// k_sparse_eval (one wave).  n_t = n_{t-1} + the running-count changes of
// counter set t & 3; statistics as the full path records them (k messages
// committed per committing iteration); the top-k kernels run only when n_t > 0
// and t is not the evaluation after the last allowed commit.  Clears counter
// set t + 2.
__global__ void k_sparse_rbp_close(EvalArgs a) {
    const int lane = threadIdx.x;
    DevState* st = a.st;
    const unsigned int done = st->done;
    const CounterLine* c0 = a.ctr + (a.t & 3u) * kCounterCopies + lane;
    const long long d = (long long)wave_sum64(c0->active);
    const long long base = a.sp_first ? 0ll : (long long)st->sp_n[(a.t - 1u) & 3u];
    const unsigned long long n1 = (unsigned long long)(base + d);
    long long n2;
    if (!a.sp_first)
        n2 = (long long)st->sp_n[(a.t - 1u) & 3u];
    else if (a.it >= 1)  // switched from the full evaluation: its count of t - 1
        n2 = (long long)wave_sum64(a.ctr[((a.t - 1u) & 3u) * kCounterCopies + lane].active);
    else
        n2 = a.prev_active_host;
    const unsigned long long ev = wave_sum64(c0->sel_a);
    if (done) {
        if (lane == 0) st->rbp_skip = 1u;
        return;
    }
    CounterLine* z = a.ctr + ((a.t + 2u) & 3u) * kCounterCopies + lane;
    z->active = 0ull;
    z->sel_a = 0ull;
    z->sel_b = 0ull;
    z->rmax = 0u;
    if (lane != 0) return;
    atomicAdd(&st->evaluated, ev);
    atomicAdd(&st->evals, 1ull);
    st->sp_n[a.t & 3u] = n1;
    st->last_t = (long long)a.t;
    st->last_active = n1;
    st->last_rmax = 0u;  // taken after the run
    st->last_prev = n2;
    if (n1 == 0ull) {
        st->done = 1u;
        st->conv_t = (long long)a.t;
        st->rbp_skip = 1u;
    } else if (a.after_final) {
        st->rbp_skip = 1u;
    } else {
        atomicAdd(&st->iterations, 1ull);
        atomicAdd(&st->committed, a.rbp_k);
        st->rbp_skip = 0u;
    }
}

// ---------------------------------------------------------------------------
// Residual splash (Sec. II-B, Sec. III-A) in frontier form, K = 2 log-odds
// layout, messages committed in place.  After the evaluation of iteration t
// (the candidate and residual key of every message, as for frontier RBP):
//   1. the residual of variable v is the largest residual of the messages into
//      v (for each slot s of v, slot rev[s] holds the message into v);
//   2. the k variables of largest residual are the roots: the radix select of
//      frontier RBP over the variable keys, tied variables taken by id;
//   3. level d holds every variable at distance exactly d from some root: a
//      thread per root marks its neighbours (d = 1) and their neighbours that
//      are neither the root nor adjacent to it (d = 2) with the iteration's tag;
//   4. the marked variables of each level are compacted into a list (wave
//      ballot and lane prefix counts, a block prefix sum in LDS, one atomic per
//      block);
//   5. the levels are updated in the order h, ..., 0, ..., h with two launches
//      each: the candidates of every message out of the level's variables,
//      computed from the messages as they stand, then their commit.
// The list order depends on the order in which blocks append; no result does
// (every message of a level is computed from the state the level starts from).
// ---------------------------------------------------------------------------
constexpr int kRsGrid = 512;  // blocks of the grid-stride splash kernels

// IsConverged for the splash: nothing is selected or updated when the
// evaluation of iteration t found no residual above eps; the level lists of
// iteration t start empty.
__global__ void k_rs_gate(DevState* st, const CounterLine* ctr, int slot) {
    const unsigned long long n = wave_sum64(ctr[slot * kCounterCopies + threadIdx.x].active);
    if (threadIdx.x == 0) st->rbp_skip = (st->done || n == 0ull) ? 1u : 0u;
    if (threadIdx.x <= kSplashMaxDepth) st->rs_count[threadIdx.x] = 0u;
}

// Block-wide exclusive prefix of the per-thread item counts c (lane prefix by
// shuffles, wave totals in LDS) and one atomic per block on *count; returns the
// list position of the thread's first item.  Called by every thread of the
// block; s_w holds kBlock / 64 + 1 words.
__device__ __forceinline__ unsigned int block_append(unsigned int c, unsigned int* count,
                                                     unsigned int* s_w) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    unsigned int x = c;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const unsigned int y = (unsigned int)__shfl_up((int)x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) s_w[w] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned int tot = 0;
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) {
            const unsigned int v = s_w[i];
            s_w[i] = tot;
            tot += v;
        }
        s_w[kBlock / 64] = tot ? atomicAdd(count, tot) : 0u;
    }
    __syncthreads();
    const unsigned int pos = s_w[kBlock / 64] + s_w[w] + x - c;
    __syncthreads();  // s_w is reused by the next call
    return pos;
}


// 1. Variable residual keys (FP32 bit patterns of non-negative residuals order
// as unsigned integers).
__global__ __launch_bounds__(kBlock) void k_rs_vkeys(RsArgs r) {
    if (r.st->rbp_skip) return;
    for (int v = blockIdx.x * kBlock + threadIdx.x; v < r.num_nodes; v += gridDim.x * kBlock) {
        const int s0 = r.node_ptr[v], s1 = r.node_ptr[v + 1];
        unsigned int k = 0u;
        for (int s = s0; s < s1; ++s) k = max(k, r.keys[r.rev[s]]);
        r.vkey[v] = k;
    }
}

// 2. The roots: every variable whose key is above the selected threshold, and
// among the variables equal to it the first sel_krem by id (all of them when
// `all`); each is marked in level 0 and appended to list 0.  Same chunking as
// the tie count (kSelPer consecutive variables per thread).
__global__ __launch_bounds__(kSelBlock) void k_rs_roots(RsArgs r, int all,
                                                        const unsigned int* block_ties) {
    __shared__ unsigned int part[kSelBlock / 64];
    __shared__ unsigned int s_w[kBlock / 64 + 1];
    static_assert(kSelBlock == kBlock, "block_append assumes kBlock threads");
    const DevState* st = r.st;
    if (st->rbp_skip) return;
    const int N = r.num_nodes;
    const unsigned int T = st->sel_prefix;
    const bool rank = !all && st->sel_rank_ties;
    const unsigned int krem = st->sel_krem;
    const long long q0 = (long long)blockIdx.x * kCommitChunk + (long long)threadIdx.x * kSelPer;
    unsigned int take = 0, tie = 0;
    if (all) {
#pragma unroll
        for (int j = 0; j < kSelPer; ++j)
            if (q0 + j < N) take |= 1u << j;
    } else {
        unsigned int kv[kSelPer];
        sel_load16(r.vkey, q0, (long long)N, kv);
#pragma unroll
        for (int j = 0; j < kSelPer; ++j) {
            if (q0 + j >= N) continue;
            if (kv[j] > T) take |= 1u << j;
            if (kv[j] == T) tie |= 1u << j;
        }
        if (!rank) take |= tie;
    }
    if (rank) {
        const unsigned int c = (unsigned int)__popc(tie);
        const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
        unsigned int x = c;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const unsigned int y = (unsigned int)__shfl_up((int)x, o, 64);
            if (lane >= o) x += y;
        }
        if (lane == 63) part[w] = x;
        __syncthreads();
        unsigned int before = block_ties[blockIdx.x] + x - c;
        for (int i = 0; i < w; ++i) before += part[i];
#pragma unroll
        for (int j = 0; j < kSelPer; ++j) {
            if (!(tie >> j & 1u)) continue;
            if (before < krem) take |= 1u << j;
            ++before;
        }
    }
    unsigned int pos = block_append((unsigned int)__popc(take), &r.st->rs_count[0], s_w);
#pragma unroll
    for (int j = 0; j < kSelPer; ++j) {
        if (!(take >> j & 1u)) continue;
        const int v = (int)(q0 + j);
        r.mark[v] = r.tag;
        r.list[pos++] = v;
    }
}

// Whether w is among the targets dst[s0 .. s1) (ascending: the slots of a
// source are ordered by target).
__device__ __forceinline__ bool rs_adjacent(const int* dst, int s0, int s1, int w) {
    int lo = s0, hi = s1;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (dst[mid] < w)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo < s1 && dst[lo] == w;
}

// 3. Levels 1 and 2 of every root's splash: a variable at distance exactly 1 is
// a neighbour of the root; one at distance exactly 2 is a neighbour of a
// neighbour that is neither the root nor one of its neighbours.  Marks are
// plain stores of the iteration's tag (several roots may store the same word).
__global__ __launch_bounds__(kBlock) void k_rs_bfs(RsArgs r) {
    if (r.st->rbp_skip) return;
    const unsigned int nr = r.st->rs_count[0];
    const size_t N = (size_t)r.num_nodes;
    unsigned int* m1 = r.mark + N;
    unsigned int* m2 = r.mark + 2 * N;
    for (unsigned int i = blockIdx.x * kBlock + threadIdx.x; i < nr; i += gridDim.x * kBlock) {
        const int root = r.list[i];
        const int s0 = r.node_ptr[root], s1 = r.node_ptr[root + 1];
        for (int s = s0; s < s1; ++s) {
            const int u = r.dst[s];
            m1[u] = r.tag;
            if (r.depth < 2) continue;
            const int u0 = r.node_ptr[u], u1 = r.node_ptr[u + 1];
            for (int q = u0; q < u1; ++q) {
                const int w = r.dst[q];
                if (w == root || rs_adjacent(r.dst, s0, s1, w)) continue;
                m2[w] = r.tag;
            }
        }
    }
}

// 4. The lists of levels 1 .. h.  Each block takes a contiguous range of the
// variables: it counts its marked variables of a level (block sum), reserves
// their places with one atomic, then writes them in order, a chunk of 256 at a
// time (wave ballot, the lane's rank among the flagged lanes of its wave
// (mbcnt), the wave offsets from a prefix sum in LDS).  A small grid keeps the
// atomics on the level counters few (one per block and level).
constexpr int kRsListGrid = 128;
__global__ __launch_bounds__(kBlock) void k_rs_lists(RsArgs r) {
    __shared__ unsigned int s_w[kBlock / 64];
    __shared__ unsigned int s_base;
    if (r.st->rbp_skip) return;
    const int N = r.num_nodes;
    const int tid = (int)threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int per = ((N + (int)gridDim.x - 1) / (int)gridDim.x + kBlock - 1) / kBlock * kBlock;
    const int v0 = (int)blockIdx.x * per, v1 = min(N, v0 + per);
    for (int d = 1; d <= r.depth; ++d) {
        const unsigned int* mk = r.mark + (size_t)d * N;
        int* L = r.list + (size_t)d * N;
        unsigned int c = 0;
        for (int v = v0 + tid; v < v1; v += kBlock) c += mk[v] == r.tag ? 1u : 0u;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) c += (unsigned int)__shfl_xor((int)c, o, 64);
        if (lane == 0) s_w[w] = c;
        __syncthreads();
        if (tid == 0) {
            unsigned int tot = 0;
            for (int i = 0; i < kBlock / 64; ++i) tot += s_w[i];
            s_base = tot ? atomicAdd(&r.st->rs_count[d], tot) : 0u;
        }
        __syncthreads();
        unsigned int off = s_base;
        for (int vb = v0; vb < v1; vb += kBlock) {
            const int v = vb + tid;
            const bool f = v < v1 && mk[v] == r.tag;
            const unsigned long long b = __ballot(f);
            const unsigned int before = __builtin_amdgcn_mbcnt_hi(
                (unsigned int)(b >> 32), __builtin_amdgcn_mbcnt_lo((unsigned int)b, 0u));
            __syncthreads();  // s_w of the previous chunk has been read
            if (lane == 0) s_w[w] = (unsigned int)__popcll(b);
            __syncthreads();
            unsigned int wpre = 0, tot = 0;
            for (int i = 0; i < kBlock / 64; ++i) {
                const unsigned int x = s_w[i];
                if (i < w) wpre += x;
                tot += x;
            }
            if (f) L[off + wpre + before] = v;
            off += tot;
        }
        __syncthreads();  // s_w and s_base are reused by the next level
    }
}

// 5a. Eq. (2) for every message out of the variables of level d, from the
// messages as they stand (the incoming log-odds summed in slot order with the
// unary, as the tiled kernel sums them).
__global__ __launch_bounds__(kBlock) void k_rs_level_eval(RsArgs r, int d) {
    if (r.st->rbp_skip) return;
    const unsigned int n = r.st->rs_count[d];
    const int* L = r.list + (size_t)d * r.num_nodes;
    for (unsigned int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
        const int v = L[i];
        const int s0 = r.node_ptr[v], s1 = r.node_ptr[v + 1];
        float agg = r.unary[v];
        for (int s = s0; s < s1; ++s) agg += r.m[r.rev[s]];
        for (int s = s0; s < s1; ++s) r.cand[s] = logodds_update(agg, r.m[r.rev[s]], r.coupling[s]);
    }
}

// 5b. Commit level d's candidates; the committed messages are added to the
// run's commit and evaluation counts (one atomic per block).
__global__ __launch_bounds__(kBlock) void k_rs_level_commit(RsArgs r, int d) {
    __shared__ unsigned int s_c[kBlock / 64];
    if (r.st->rbp_skip) return;
    const unsigned int n = r.st->rs_count[d];
    const int* L = r.list + (size_t)d * r.num_nodes;
    unsigned int c = 0;
    for (unsigned int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
        const int v = L[i];
        const int s0 = r.node_ptr[v], s1 = r.node_ptr[v + 1];
        for (int s = s0; s < s1; ++s) r.m[s] = r.cand[s];
        c += (unsigned int)(s1 - s0);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
    if ((threadIdx.x & 63) == 0) s_c[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long C = 0;
        for (int w = 0; w < kBlock / 64; ++w) C += s_c[w];
        if (C) {
            atomicAdd(&r.st->committed, C);
            atomicAdd(&r.st->evaluated, C);
        }
    }
}

__global__ void k_fill_u32(unsigned int* p, unsigned int v, long long n) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        p[i] = v;
}

}  // namespace

// ---------------------------------------------------------------------------
// Launch wrappers
// ---------------------------------------------------------------------------
hipError_t launch_init_state(DevState* st, CounterLine* ctr, hipStream_t s) {
    k_init_state<<<1, 256, 0, s>>>(st, ctr);
    return hipGetLastError();
}

hipError_t launch_fill(float* p, float v, long long n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    long long blocks = (n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    k_fill<<<(int)blocks, 256, 0, s>>>(p, v, n);
    return hipGetLastError();
}

template <int KP, bool EXACT, bool SPLIT = false>
static hipError_t launch_generic_kp(int mode, const EvalArgs& a, int grid, size_t shm,
                                    hipStream_t s) {
    switch (mode) {
    case kModeLBP: k_eval_generic<KP, kModeLBP, EXACT, SPLIT><<<grid, kBlock, shm, s>>>(a); break;
    case kModeRnBP: k_eval_generic<KP, kModeRnBP, EXACT, SPLIT><<<grid, kBlock, shm, s>>>(a); break;
    case kModeRBP: k_eval_generic<KP, kModeRBP, EXACT, SPLIT><<<grid, kBlock, shm, s>>>(a); break;
    default: k_eval_generic<KP, kModeEvalOnly, EXACT, SPLIT><<<grid, kBlock, shm, s>>>(a); break;
    }
    return hipGetLastError();
}

template <int KP>
static hipError_t launch_generic_k(int mode, const EvalArgs& a, int grid, size_t shm,
                                   hipStream_t s) {
    if (a.num_states != KP) return launch_generic_kp<KP, false>(mode, a, grid, shm, s);
    if constexpr (KP * kBlock > kTileFloatsGeneric) {
        // every tile on the lane-group path
        if ((a.pair_kind == kPairShared || a.pair_kind == kPairSharedAsym) && !a.tile_big)
            return launch_generic_kp<KP, true, true>(mode, a, grid, shm, s);
    }
    return launch_generic_kp<KP, true>(mode, a, grid, shm, s);
}

hipError_t launch_eval(int layout, int kp, int mode, const EvalArgs& a, hipStream_t s) {
    const int grid = 8 * a.tiles_per_xcd;
    if (grid <= 0) return hipSuccess;
    if (layout == kLayoutLogOdds) {
        const int g = a.pipe_grid;
        if (a.rev16) {
            switch (mode) {
            case kModeLBP: k_eval_logodds<kModeLBP, true><<<g, kBlockLO, 0, s>>>(a); break;
            case kModeRnBP: k_eval_logodds<kModeRnBP, true><<<g, kBlockLO, 0, s>>>(a); break;
            case kModeRBP: k_eval_logodds<kModeRBP, true><<<g, kBlockLO, 0, s>>>(a); break;
            default: k_eval_logodds<kModeEvalOnly, true><<<g, kBlockLO, 0, s>>>(a); break;
            }
        } else {
            switch (mode) {
            case kModeLBP: k_eval_logodds<kModeLBP, false><<<g, kBlockLO, 0, s>>>(a); break;
            case kModeRnBP: k_eval_logodds<kModeRnBP, false><<<g, kBlockLO, 0, s>>>(a); break;
            case kModeRBP: k_eval_logodds<kModeRBP, false><<<g, kBlockLO, 0, s>>>(a); break;
            default: k_eval_logodds<kModeEvalOnly, false><<<g, kBlockLO, 0, s>>>(a); break;
            }
        }
        if (a.num_big > 0) {
            switch (mode) {
            case kModeLBP: k_eval_logodds_big<kModeLBP><<<a.num_big, kBlock, 0, s>>>(a); break;
            case kModeRnBP: k_eval_logodds_big<kModeRnBP><<<a.num_big, kBlock, 0, s>>>(a); break;
            case kModeRBP: k_eval_logodds_big<kModeRBP><<<a.num_big, kBlock, 0, s>>>(a); break;
            default: k_eval_logodds_big<kModeEvalOnly><<<a.num_big, kBlock, 0, s>>>(a); break;
            }
        }
        return hipGetLastError();
    }
    if (layout == kLayoutRagged) {
        const int g = a.pipe_grid;
        switch (mode) {
        case kModeLBP: k_eval_ragged<kModeLBP><<<g, kBlock, 0, s>>>(a); break;
        case kModeRnBP: k_eval_ragged<kModeRnBP><<<g, kBlock, 0, s>>>(a); break;
        case kModeRBP: k_eval_ragged<kModeRBP><<<g, kBlock, 0, s>>>(a); break;
        default: k_eval_ragged<kModeEvalOnly><<<g, kBlock, 0, s>>>(a); break;
        }
        return hipGetLastError();
    }
    const int K = a.num_states;
    const int TS = kTileFloatsGeneric / K;
    const int TN = a.tile_nodes_max;
    if (K == 32 && a.pair_kind == kPairShared && !a.tile_big && !a.no_mfma) {
        // no shared table in LDS
        const size_t shm = sizeof(float) * (size_t)(TS * (K + 1) + ((TN * (K + 1) + 3) & ~3)) +
                           sizeof(int) * (size_t)(TS + TN + 1) + sizeof(unsigned short) * (size_t)TS;
        if (a.mfma_bf16) {
            switch (mode) {
            case kModeLBP: k_eval_mfma32<kModeLBP, true><<<grid, kBlock, shm, s>>>(a); break;
            case kModeRnBP: k_eval_mfma32<kModeRnBP, true><<<grid, kBlock, shm, s>>>(a); break;
            case kModeRBP: k_eval_mfma32<kModeRBP, true><<<grid, kBlock, shm, s>>>(a); break;
            default: k_eval_mfma32<kModeEvalOnly, true><<<grid, kBlock, shm, s>>>(a); break;
            }
        } else {
            switch (mode) {
            case kModeLBP: k_eval_mfma32<kModeLBP, false><<<grid, kBlock, shm, s>>>(a); break;
            case kModeRnBP: k_eval_mfma32<kModeRnBP, false><<<grid, kBlock, shm, s>>>(a); break;
            case kModeRBP: k_eval_mfma32<kModeRBP, false><<<grid, kBlock, shm, s>>>(a); break;
            default: k_eval_mfma32<kModeEvalOnly, false><<<grid, kBlock, shm, s>>>(a); break;
            }
        }
        return hipGetLastError();
    }
    const int tables = a.pair_kind == kPairSharedAsym ? 2 : 1;
    const size_t shm =
        sizeof(float) * (size_t)(TS * (K + 1) + ((TN * (K + 1) + 3) & ~3) + tables * K * K) +
        sizeof(int) * (size_t)(TS + TN + 1) + sizeof(unsigned short) * (size_t)TS;
    switch (kp) {
    case 2: return launch_generic_k<2>(mode, a, grid, shm, s);
    case 4: return launch_generic_k<4>(mode, a, grid, shm, s);
    case 8: return launch_generic_k<8>(mode, a, grid, shm, s);
    case 16: return launch_generic_k<16>(mode, a, grid, shm, s);
    case 32: return launch_generic_k<32>(mode, a, grid, shm, s);
    case 64: return launch_generic_k<64>(mode, a, grid, shm, s);
    default: return hipErrorInvalidValue;
    }
}

int logodds_blocks_per_cu(int mode) {
    int n = 0;
    hipError_t e;
    switch (mode) {
    case kModeLBP:
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, (const void*)k_eval_logodds<kModeLBP, true>, kBlockLO, 0);
        break;
    case kModeRnBP:
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, (const void*)k_eval_logodds<kModeRnBP, true>, kBlockLO, 0);
        break;
    case kModeRBP:
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, (const void*)k_eval_logodds<kModeRBP, true>, kBlockLO, 0);
        break;
    default:
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, (const void*)k_eval_logodds<kModeEvalOnly, true>, kBlockLO, 0);
        break;
    }
    return e == hipSuccess ? n : 0;
}

// The done flag of every graph of a batch, gathered for one readback.
__global__ void k_batch_status(const BatchGraph* graphs, int num_graphs, unsigned int* done) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= num_graphs) return;
    const DevState* st = graphs[g].a.st;
    done[g] = st ? st->done : 0u;
}

hipError_t launch_batch_status(const BatchGraph* graphs, int num_graphs, unsigned int* done,
                               hipStream_t s) {
    k_batch_status<<<(num_graphs + 255) / 256, 256, 0, s>>>(graphs, num_graphs, done);
    return hipGetLastError();
}

hipError_t launch_eval_batch(BatchGraph* graphs, int num_graphs, const int* list, BatchCtl* ctl,
                             int grid, hipStream_t s) {
    k_batch_advance<<<(num_graphs + 255) / 256, 256, 0, s>>>(graphs, num_graphs, ctl);
    k_eval_batch<<<grid, kBlockLO, 0, s>>>(graphs, (const int4*)list, ctl);
    return hipGetLastError();
}

hipError_t batch_graph_nodes(BatchGraph* graphs, int num_graphs, const int* list, BatchCtl* ctl,
                             int grid, int launches, hipGraph_t* out) {
    hipGraph_t gr = nullptr;
    hipError_t e = hipGraphCreate(&gr, 0);
    if (e != hipSuccess) return e;
    void* adv_args[3] = {(void*)&graphs, (void*)&num_graphs, (void*)&ctl};
    const int4* lst = (const int4*)list;
    void* ev_args[3] = {(void*)&graphs, (void*)&lst, (void*)&ctl};
    hipKernelNodeParams pa{};
    pa.func = (void*)k_batch_advance;
    pa.gridDim = dim3((unsigned)((num_graphs + 255) / 256));
    pa.blockDim = dim3(256);
    pa.kernelParams = adv_args;
    hipKernelNodeParams pe{};
    pe.func = (void*)k_eval_batch;
    pe.gridDim = dim3((unsigned)grid);
    pe.blockDim = dim3(kBlock);
    pe.kernelParams = ev_args;
    hipGraphNode_t prev = nullptr;
    for (int k = 0; k < launches && e == hipSuccess; ++k) {
        hipGraphNode_t na = nullptr, ne = nullptr;
        e = hipGraphAddKernelNode(&na, gr, prev ? &prev : nullptr, prev ? 1 : 0, &pa);
        if (e == hipSuccess) e = hipGraphAddKernelNode(&ne, gr, &na, 1, &pe);
        prev = ne;
    }
    if (e != hipSuccess) {
        (void)hipGraphDestroy(gr);
        return e;
    }
    *out = gr;
    return hipSuccess;
}

hipError_t launch_close_run(const EvalArgs& a, hipStream_t s) {
    k_close_run<<<1, 64, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_marginals(int layout, int kp, const int* node_ptr, const int* rev,
                            const float* unary, const float* m, float* out, int N, int K,
                            hipStream_t s) {
    (void)kp;
    if (N <= 0) return hipSuccess;
    const int grid = (N + 255) / 256;
    if (layout == kLayoutLogOdds)
        k_marginals_logodds<<<grid, 256, 0, s>>>(node_ptr, rev, unary, m, out, N);
    else {
        int W = 1;
        while (W < K) W <<= 1;
        const long long per_block = 4ll * (64 / W);  // four waves of 64 / W variables
        k_marginals_generic<<<(int)std::min<long long>((N + per_block - 1) / per_block, 65536), 256,
                              0, s>>>(node_ptr, rev, unary, m, out, N, K);
    }
    return hipGetLastError();
}

hipError_t launch_marginals_ragged(const EvalArgs& a, float* out, hipStream_t s) {
    if (a.num_nodes <= 0) return hipSuccess;
    const int waves = kBlock / 64;
    long long g = ((long long)a.num_nodes + waves - 1) / waves;
    if (g > 8192) g = 8192;
    k_marginals_ragged<<<(int)g, kBlock, 0, s>>>(a, out);
    return hipGetLastError();
}

hipError_t launch_fill_ragged(float* m, const int* moff, int E, hipStream_t s) {
    if (E <= 0) return hipSuccess;
    long long g = ((long long)E + 255) / 256;
    if (g > 8192) g = 8192;
    k_fill_ragged<<<(int)g, 256, 0, s>>>(m, moff, E);
    return hipGetLastError();
}

hipError_t launch_sparse_iteration(const EvalArgs& a, hipStream_t s) {
    // at least one block, so that a graph without slots still closes its
    // evaluation (n_t = 0)
    const int grid = a.num_nodes > 0 ? (a.num_nodes + kBlock - 1) / kBlock : 1;
    k_sparse_eval<<<grid, kBlock, 0, s>>>(a);
    k_sparse_commit<<<grid, kBlock, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_sparse_rbp_eval(const EvalArgs& a, hipStream_t s) {
    const int grid = a.num_nodes > 0 ? (a.num_nodes + kBlock - 1) / kBlock : 1;
    k_sparse_eval<<<grid, kBlock, 0, s>>>(a);
    k_sparse_rbp_close<<<1, 64, 0, s>>>(a);
    return hipGetLastError();
}

// After a run with outcome flags: rows of `prim` whose first entry carries the
// flag take the other outcome's row (when the last choice was the other
// outcome) or just lose the flag.
__global__ void k_resolve_rows(float* prim, const float* other, int take_other, long long E,
                               int K) {
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < E;
         e += (long long)gridDim.x * blockDim.x) {
        float* r = prim + e * K;
        const float v0 = r[0];
        if (!(__float_as_uint(v0) >> 31)) continue;
        if (take_other) {
            for (int x = 0; x < K; ++x) r[x] = other[e * K + x];
        } else {
            r[0] = fabsf(v0);
        }
    }
}

hipError_t launch_resolve_rows(float* const* pair_bufs, int prim, int sel, long long E, int K,
                               hipStream_t s) {
    if (E <= 0) return hipSuccess;
    long long g = (E + 255) / 256;
    if (g > 4096) g = 4096;
    k_resolve_rows<<<(int)g, 256, 0, s>>>(pair_bufs[prim], pair_bufs[prim ^ 1], sel != prim ? 1 : 0,
                                          E, K);
    return hipGetLastError();
}

hipError_t launch_sparse_rmax(const EvalArgs& a, hipStream_t s) {
    long long g = ((long long)a.num_messages + kBlock - 1) / kBlock;
    const int grid = g < 1 ? 1 : g > kSparseGridMax ? kSparseGridMax : (int)g;
    k_sparse_rmax<<<grid, kBlock, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_sparse_setup(const EvalArgs& a, int build_dst, hipStream_t s) {
    const int grid = (a.num_nodes + kBlock - 1) / kBlock;
    if (grid <= 0) return hipSuccess;
    k_sparse_setup<<<grid, kBlock, 0, s>>>(a, build_dst);
    return hipGetLastError();
}

hipError_t launch_rbp_gate(DevState* st, const CounterLine* ctr, int slot_idx, hipStream_t s) {
    k_rbp_gate<<<1, 64, 0, s>>>(st, ctr, slot_idx);
    return hipGetLastError();
}

hipError_t launch_rbp_select(DevState* st, const unsigned int* keys, const int* rev, int E,
                             unsigned int k, const CounterLine* gate_ctr, int hist0_done,
                             unsigned int* block_ties, hipStream_t s) {
    const int nb = (E + kCommitChunk - 1) / kCommitChunk;
    const int grid = nb > 0 ? nb : 1;
    for (int pass = 0; pass < 4; ++pass) {
        if (pass > 0 || !hist0_done) k_rbp_hist<<<grid, kSelBlock, 0, s>>>(st, keys, E, pass);
        k_rbp_scan<<<1, kSelBlock, 0, s>>>(st, pass, k, pass == 0 ? gate_ctr : nullptr);
    }
    k_rbp_tiecount<<<grid, kSelBlock, 0, s>>>(st, keys, rev, E, block_ties);
    k_rbp_tiescan<<<1, kSelBlock, 0, s>>>(st, block_ties, nb);
    return hipGetLastError();
}

hipError_t launch_rbp_commit(DevState* st, unsigned int* keys, const int* rev,
                             const float* cand, float* m, int E, int row, int all, int slot_idx,
                             const unsigned int* block_ties, const RbpSparse& sp,
                             const int* moff, hipStream_t s) {
    (void)slot_idx;
    const int nb = (E + kCommitChunk - 1) / kCommitChunk;
    if (nb <= 0) return hipSuccess;
    k_rbp_commit<<<nb, kSelBlock, 0, s>>>(st, keys, rev, cand, m, E, row, all, block_ties, sp,
                                         moff);
    return hipGetLastError();
}

size_t splash_bytes(int num_nodes) {
    const size_t n = (size_t)(num_nodes > 0 ? num_nodes : 0);
    const size_t part = (sizeof(unsigned int) * n + 255) & ~size_t(255);
    const size_t lv = (sizeof(unsigned int) * n * (kSplashMaxDepth + 1) + 255) & ~size_t(255);
    return part + 2 * lv;
}

static int rs_grid(long long items) {
    const long long g = (items + kBlock - 1) / kBlock;
    return g < 1 ? 1 : g > kRsGrid ? kRsGrid : (int)g;
}

hipError_t launch_rs_gate(DevState* st, const CounterLine* ctr, int slot_idx, hipStream_t s) {
    k_rs_gate<<<1, 64, 0, s>>>(st, ctr, slot_idx);
    return hipGetLastError();
}

hipError_t launch_rs_select(const RsArgs& r, unsigned int k, int all, unsigned int* block_ties,
                            hipStream_t s) {
    const int N = r.num_nodes;
    if (N <= 0) return hipSuccess;
    k_rs_vkeys<<<rs_grid(N), kBlock, 0, s>>>(r);
    if (!all) {
        hipError_t e = launch_rbp_select(r.st, r.vkey, nullptr, N, k, nullptr, 0, block_ties, s);
        if (e != hipSuccess) return e;
    }
    k_rs_roots<<<(N + kCommitChunk - 1) / kCommitChunk, kSelBlock, 0, s>>>(r, all, block_ties);
    if (r.depth >= 1) {
        k_rs_bfs<<<rs_grid(N), kBlock, 0, s>>>(r);
        k_rs_lists<<<kRsListGrid, kBlock, 0, s>>>(r);
    }
    return hipGetLastError();
}

hipError_t launch_rs_level(const RsArgs& r, int d, hipStream_t s) {
    if (r.num_nodes <= 0) return hipSuccess;
    k_rs_level_eval<<<rs_grid(r.num_nodes), kBlock, 0, s>>>(r, d);
    k_rs_level_commit<<<rs_grid(r.num_nodes), kBlock, 0, s>>>(r, d);
    return hipGetLastError();
}

hipError_t launch_fill_u32(unsigned int* p, unsigned int v, long long n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    long long blocks = (n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    k_fill_u32<<<(int)blocks, 256, 0, s>>>(p, v, n);
    return hipGetLastError();
}

}  // namespace bp

// ---------------------------------------------------------------------------
// bp_run_noalloc: bp_run with its per-run scratch (iteration state, counters,
// top-k tie counts) in a file-scope device array instead of the graph's
// memory.  Each GPU holds its own copy of the array; its device address is
// looked up once per device, with that device current, and only that address
// is handed to kernels (the array's name is a host-side stand-in).
// ---------------------------------------------------------------------------
#include <mutex>

namespace {
constexpr size_t kNoAllocScratchBytes = size_t(1) << 20;  // graphs up to ~10^9 messages
constexpr int kNoAllocMaxDevices = 64;
std::mutex g_noalloc_mu;
char* g_noalloc_ptr[kNoAllocMaxDevices];
}  // namespace

static __device__ __align__(256) char scratch[kNoAllocScratchBytes];

extern "C" int bp_run_noalloc(bp_graph* g, int schedule, double eps, double p, uint64_t seed,
                              const bp_run_opts* opts, bp_run_stats* stats) {
    if (!g) return bp::report_error(BP_EINVAL, "graph is NULL");
    const int dev = bp::graph_device(g);
    if (dev < 0 || dev >= kNoAllocMaxDevices)
        return bp::report_error(BP_EDEVICE, "device index out of the static scratch table");
    char* ptr = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_noalloc_mu);
        ptr = g_noalloc_ptr[dev];
        if (!ptr) {
            int prev = -1;
            if (hipGetDevice(&prev) != hipSuccess)
                return bp::report_error(BP_EDEVICE, "hipGetDevice failed");
            if (prev != dev && hipSetDevice(dev) != hipSuccess)
                return bp::report_error(BP_EDEVICE, "hipSetDevice failed");
            void* addr = nullptr;
            const hipError_t e = hipGetSymbolAddress(&addr, HIP_SYMBOL(scratch));
            if (prev != dev) (void)hipSetDevice(prev);
            if (e != hipSuccess || !addr)
                return bp::report_error(BP_EDEVICE, "hipGetSymbolAddress(scratch) failed");
            ptr = (char*)addr;
            g_noalloc_ptr[dev] = ptr;
        }
    }
    return bp::run_with_scratch(g, schedule, eps, p, seed, opts, stats, ptr,
                                kNoAllocScratchBytes);
}
