// HIP kernels of libbp for gfx950 (CDNA4, wave64).
//
// One iteration of Alg. 1 is one launch of an evaluation kernel followed by one
// launch of k_finish (plus the top-k selection kernels for frontier residual BP).
//
// Evaluation kernel (Eq. (2) + Eq. (4) + frontier rule + commit, fused):
// messages are stored grouped by target node (CSR by destination), so the
// incoming messages of a run of target nodes form one contiguous slot range.
// A 256-thread block owns such a tile of nodes:
//   phase 1  coalesced load of the tile's incoming messages into LDS (as logs);
//   phase 2  one thread per node (per node-state for K > 2) sums them with the
//            log unary into the node aggregate A_i = log psi_i + sum_k log m_{k->i};
//   phase 3  one thread per slot: the slot holds m_{k->i}, so the thread computes
//            the outgoing message m_{i->k} from the cavity A_i - log m_{k->i}
//            (Eq. (2) excludes exactly that message), normalises it, reads the
//            old m_{i->k} at the reverse slot, forms the L-infinity residual, applies
//            the frontier rule and writes the committed value to the next buffer.
// Every slot of the next buffer is written exactly once per iteration (each
// message is the outgoing message of exactly one node), so the update is
// synchronous (Jacobi) with no atomics on message values.
#include "bp_internal.h"

namespace bp {
namespace {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), output word 0 only.
// ---------------------------------------------------------------------------
__device__ __forceinline__ unsigned int philox_word0(unsigned int c0, unsigned int c1,
                                                     unsigned int c2, unsigned int k0,
                                                     unsigned int k1) {
    unsigned int c3 = 0u;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const unsigned int hi0 = __umulhi(0xD2511F53u, c0), lo0 = 0xD2511F53u * c0;
        const unsigned int hi1 = __umulhi(0xCD9E8D57u, c2), lo1 = 0xCD9E8D57u * c2;
        const unsigned int n0 = hi1 ^ c1 ^ k0;
        const unsigned int n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    return c0;
}

__device__ __forceinline__ float sigmoid_fast(float x) {
    return __frcp_rn(1.0f + __expf(-x));
}

// log cosh(x) + log 2, i.e. |x| + log(1 + exp(-2|x|)); the constant cancels in
// the differences it is used in.
__device__ __forceinline__ float logcosh_shift(float x) {
    const float a = fabsf(x);
    return a + __logf(1.0f + __expf(-2.0f * a));
}

struct RedScratch {
    float rmax[kBlock / 64];
    unsigned int act[kBlock / 64];
    unsigned int sa[kBlock / 64];
    unsigned int sb[kBlock / 64];
};

// Block-wide reduction of the per-thread residual max and counts, then one
// atomic per quantity per block (integer adds and an ordered max on the
// FP32 bit pattern of a non-negative float: both order independent).
__device__ __forceinline__ void block_accumulate(RedScratch* red, DevState* st, int slot,
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
#pragma unroll
        for (int i = 1; i < kBlock / 64; ++i) {
            r = fmaxf(r, red->rmax[i]);
            A += red->act[i];
            SA += red->sa[i];
            SB += red->sb[i];
        }
        if (A) atomicAdd(&st->active[slot], (unsigned long long)A);
        if (SA) atomicAdd(&st->sel_a[slot], (unsigned long long)SA);
        if (SB) atomicAdd(&st->sel_b[slot], (unsigned long long)SB);
        if (r > 0.0f) atomicMax(&st->rmax[slot], __float_as_uint(r));
    }
}

// Append the slots of this wave whose `need` is set to the revert list:
// ballot + popcount prefix inside the wave, one atomic per wave.
__device__ __forceinline__ void wave_append(bool need, int value, int* list,
                                            unsigned int* len) {
    const unsigned long long mask = __ballot(need);
    if (mask == 0ull) return;
    const int lane = threadIdx.x & 63;
    unsigned int base = 0;
    if (lane == 0) base = atomicAdd(len, (unsigned int)__popcll(mask));
    base = __shfl(base, 0, 64);
    if (need) {
        const unsigned int pre = (unsigned int)__popcll(mask & ((1ull << lane) - 1ull));
        list[base + pre] = value;
    }
}

__device__ __forceinline__ int tile_of_block(const EvalArgs& a) {
    // Workgroups are dealt to the 8 XCDs round-robin; give each XCD a contiguous
    // range of tiles so neighbouring tiles share that XCD's L2.
    const int b = blockIdx.x;
    return (b & 7) * a.tiles_per_xcd + (b >> 3);
}

// ---------------------------------------------------------------------------
// K = 2 Ising, one log-odds value per message: lambda = log(m(1) / m(0)).
// Aggregate L_i = u_i + sum_k lambda_{k->i} with u_i = log psi_i(1) - log psi_i(0).
// With H = (L_i - lambda_{k->i}) / 2 the outgoing message of Eq. (2) for
// psi = exp(J s_i s_k) has log-odds log cosh(J + H) - log cosh(J - H).
// ---------------------------------------------------------------------------
constexpr int kPerThreadLO = kTileSlotsLogOdds / kBlock;

template <int MODE>
__global__ __launch_bounds__(kBlock) void k_eval_logodds(EvalArgs a) {
    __shared__ float s_lam[kTileSlotsLogOdds];
    __shared__ unsigned short s_owner[kTileSlotsLogOdds];
    __shared__ float s_L[kTileNodesMax];
    __shared__ RedScratch red;
    __shared__ float s_part[kBlock / 64];

    DevState* st = a.st;
    if (st->done) return;
    const int tile = tile_of_block(a);
    if (tile >= a.num_tiles) return;
    const int n0 = a.tile_start[tile], n1 = a.tile_start[tile + 1];
    const int s0 = a.in_ptr[n0], s1 = a.in_ptr[n1];
    const int ns = s1 - s0, nn = n1 - n0;
    const int tid = threadIdx.x;

    float rmax = 0.0f;
    unsigned int act = 0, sa = 0, sb = 0;

    if (ns <= kTileSlotsLogOdds) {
        float lam[kPerThreadLO];
#pragma unroll
        for (int k = 0; k < kPerThreadLO; ++k) {
            const int q = tid + k * kBlock;
            lam[k] = 0.0f;
            if (q < ns) {
                lam[k] = a.m_in[s0 + q];
                s_lam[q] = lam[k];
            }
        }
        __syncthreads();
        for (int v = tid; v < nn; v += kBlock) {
            const int n = n0 + v;
            const int q0 = a.in_ptr[n] - s0, q1 = a.in_ptr[n + 1] - s0;
            float L = a.unary[n];
            for (int q = q0; q < q1; ++q) {
                L += s_lam[q];
                s_owner[q] = (unsigned short)v;
            }
            s_L[v] = L;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kPerThreadLO; ++k) {
            const int q = tid + k * kBlock;
            bool need = false;
            int e = 0;
            if (q < ns) {
                const int s = s0 + q;
                const int v = s_owner[q];
                const float H = 0.5f * (s_L[v] - lam[k]);
                const float J = a.coupling[s];
                const float lam_new = logcosh_shift(J + H) - logcosh_shift(J - H);
                e = a.rev[s];
                const float lam_old = a.m_in[e];
                const float r = fabsf(sigmoid_fast(lam_new) - sigmoid_fast(lam_old));
                const bool active = r > a.eps;
                rmax = fmaxf(rmax, r);
                act += active;
                if (MODE == kModeLBP) {
                    a.m_out[e] = lam_new;
                } else if (MODE == kModeRnBP) {
                    bool ka = false, kb = false;
                    if (active) {
                        const unsigned int u24 =
                            philox_word0((unsigned int)(n0 + v), (unsigned int)a.src[s], a.t,
                                         a.key0, a.key1) >> 8;
                        ka = u24 < a.thr_a;
                        kb = u24 < a.thr_b;
                    }
                    sa += ka;
                    sb += kb;
                    need = ka && !kb;
                    a.m_out[e] = ka ? lam_new : lam_old;
                } else if (MODE == kModeRBP) {
                    a.cand[e] = lam_new;
                    a.keys[e] = __float_as_uint(r);
                }
            }
            if (MODE == kModeRnBP) wave_append(need, e, a.revert_list, &st->revert_len[a.slot_idx]);
        }
    } else {
        // A single node whose in-degree exceeds the tile: aggregate by a block
        // reduction, then stream the slots.
        float part = 0.0f;
        for (int q = tid; q < ns; q += kBlock) part += a.m_in[s0 + q];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) part += __shfl_xor(part, o, 64);
        if ((tid & 63) == 0) s_part[tid >> 6] = part;
        __syncthreads();
        float L = a.unary[n0];
#pragma unroll
        for (int i = 0; i < kBlock / 64; ++i) L += s_part[i];
        for (int base = 0; base < ns; base += kBlock) {
            const int q = base + tid;
            bool need = false;
            int e = 0;
            if (q < ns) {
                const int s = s0 + q;
                const float lam_q = a.m_in[s];
                const float H = 0.5f * (L - lam_q);
                const float J = a.coupling[s];
                const float lam_new = logcosh_shift(J + H) - logcosh_shift(J - H);
                e = a.rev[s];
                const float lam_old = a.m_in[e];
                const float r = fabsf(sigmoid_fast(lam_new) - sigmoid_fast(lam_old));
                const bool active = r > a.eps;
                rmax = fmaxf(rmax, r);
                act += active;
                if (MODE == kModeLBP) {
                    a.m_out[e] = lam_new;
                } else if (MODE == kModeRnBP) {
                    bool ka = false, kb = false;
                    if (active) {
                        const unsigned int u24 =
                            philox_word0((unsigned int)n0, (unsigned int)a.src[s], a.t, a.key0,
                                         a.key1) >> 8;
                        ka = u24 < a.thr_a;
                        kb = u24 < a.thr_b;
                    }
                    sa += ka;
                    sb += kb;
                    need = ka && !kb;
                    a.m_out[e] = ka ? lam_new : lam_old;
                } else if (MODE == kModeRBP) {
                    a.cand[e] = lam_new;
                    a.keys[e] = __float_as_uint(r);
                }
            }
            if (MODE == kModeRnBP) wave_append(need, e, a.revert_list, &st->revert_len[a.slot_idx]);
        }
    }
    block_accumulate(&red, st, a.slot_idx, rmax, act, sa, sb);
}

// ---------------------------------------------------------------------------
// Generic layout: [E][K] normalised FP32 probabilities, K <= KP.
// ---------------------------------------------------------------------------
template <int KP, int MODE>
__global__ __launch_bounds__(kBlock) void k_eval_generic(EvalArgs a) {
    extern __shared__ float smem[];
    __shared__ RedScratch red;
    DevState* st = a.st;
    if (st->done) return;
    const int tile = tile_of_block(a);
    if (tile >= a.num_tiles) return;
    const int K = a.num_states;
    const int TS = kTileFloatsGeneric / K;  // slots (and nodes) per tile
    float* s_logm = smem;                   // [TS][K]
    float* s_A = s_logm + TS * K;           // [TS][K]
    float* s_psi = s_A + TS * K;            // [K][K] shared table
    unsigned short* s_owner = (unsigned short*)(s_psi + K * K);

    const int n0 = a.tile_start[tile], n1 = a.tile_start[tile + 1];
    const int s0 = a.in_ptr[n0], s1 = a.in_ptr[n1];
    const int ns = s1 - s0, nn = n1 - n0;
    const int tid = threadIdx.x;
    const bool big = ns > TS;

    if (a.pair_kind == kPairShared || a.pair_kind == kPairSharedAsym)
        for (int i = tid; i < K * K; i += kBlock) s_psi[i] = a.pair[i];
    if (!big) {
        const long long base = (long long)s0 * K;
        for (int i = tid; i < ns * K; i += kBlock) s_logm[i] = __logf(a.m_in[base + i]);
        __syncthreads();
        for (int i = tid; i < nn * K; i += kBlock) {
            const int v = i / K, x = i - v * K;
            const int n = n0 + v;
            const int q0 = a.in_ptr[n] - s0, q1 = a.in_ptr[n + 1] - s0;
            float acc = a.unary[(long long)n * K + x];
            for (int q = q0; q < q1; ++q) acc += s_logm[q * K + x];
            s_A[i] = acc;
            if (x == 0)
                for (int q = q0; q < q1; ++q) s_owner[q] = (unsigned short)v;
        }
    } else {
        // single node with in-degree > TS: aggregate each state with a strided sum
        for (int x = 0; x < K; ++x) {
            float part = 0.0f;
            for (int q = tid; q < ns; q += kBlock) part += __logf(a.m_in[(long long)(s0 + q) * K + x]);
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
    for (int base = 0; base < ns; base += kBlock) {
        const int q = base + tid;
        bool need = false;
        int e = 0;
        if (q < ns) {
            const int s = s0 + q;
            const int v = big ? 0 : s_owner[q];
            const int node = n0 + v;
            float g[KP];
            float mx = -3.402823466e38f;
#pragma unroll
            for (int x = 0; x < KP; ++x) {
                if (x < K) {
                    const float lm = big ? __logf(a.m_in[(long long)s * K + x]) : s_logm[q * K + x];
                    g[x] = s_A[v * K + x] - lm;
                    mx = fmaxf(mx, g[x]);
                }
            }
#pragma unroll
            for (int x = 0; x < KP; ++x)
                if (x < K) g[x] = __expf(g[x] - mx);
            float c[KP];
#pragma unroll
            for (int y = 0; y < KP; ++y) c[y] = 0.0f;
            if (a.pair_kind == kPairIsing) {
                const float J = a.coupling[s];
                const float ep = __expf(J), em = __expf(-J);
                c[0] = ep * g[0] + em * g[1];
                c[1] = em * g[0] + ep * g[1];
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
            e = a.rev[s];
            const long long eo = (long long)e * K;
            float r = 0.0f;
            float old[KP];
#pragma unroll
            for (int y = 0; y < KP; ++y) {
                if (y < K) {
                    c[y] *= inv;
                    old[y] = a.m_in[eo + y];
                    r = fmaxf(r, fabsf(c[y] - old[y]));
                }
            }
            const bool active = r > a.eps;
            rmax = fmaxf(rmax, r);
            act += active;
            if (MODE == kModeLBP) {
#pragma unroll
                for (int y = 0; y < KP; ++y)
                    if (y < K) a.m_out[eo + y] = c[y];
            } else if (MODE == kModeRnBP) {
                bool ka = false, kb = false;
                if (active) {
                    const unsigned int u24 = philox_word0((unsigned int)node, (unsigned int)a.src[s],
                                                          a.t, a.key0, a.key1) >> 8;
                    ka = u24 < a.thr_a;
                    kb = u24 < a.thr_b;
                }
                sa += ka;
                sb += kb;
                need = ka && !kb;
#pragma unroll
                for (int y = 0; y < KP; ++y)
                    if (y < K) a.m_out[eo + y] = ka ? c[y] : old[y];
            } else if (MODE == kModeRBP) {
#pragma unroll
                for (int y = 0; y < KP; ++y)
                    if (y < K) a.cand[eo + y] = c[y];
                a.keys[e] = __float_as_uint(r);
            }
        }
        if (MODE == kModeRnBP) wave_append(need, e, a.revert_list, &st->revert_len[a.slot_idx]);
    }
    block_accumulate(&red, st, a.slot_idx, rmax, act, sa, sb);
}

// ---------------------------------------------------------------------------
// End of iteration t: IsConverged, p_t from EdgeRatio, the revert of messages
// kept only under the larger threshold when p_t takes the smaller one, and the
// scalar bookkeeping.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_finish(FinishArgs a) {
    DevState* st = a.st;
    if (st->done) return;
    const unsigned long long n_t = st->active[a.slot_idx];
    const bool converged = n_t == 0ull;
    bool p_low = false;
    if (a.mode == kModeRnBP) {
        if (a.dynamic_p) {
            const long long np = a.has_prev_in_run ? (long long)st->active[a.prev_slot_idx]
                                                   : a.prev_active_host;
            p_low = np > 0 && ((double)n_t / (double)np > a.ratio_threshold);
        } else {
            p_low = true;
        }
    }
    const bool use_a = !a.thresholds_differ || (p_low == (a.low_is_a != 0));
    if (a.mode == kModeRnBP && !converged && !a.final_eval && !use_a) {
        const unsigned int len = st->revert_len[a.slot_idx];
        const int row = a.row;
        for (unsigned int i = blockIdx.x * blockDim.x + threadIdx.x; i < len;
             i += gridDim.x * blockDim.x) {
            const long long e = a.revert_list[i];
            for (int x = 0; x < row; ++x) a.m_out[e * row + x] = a.m_in[e * row + x];
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        unsigned long long committed = 0;
        if (!converged && !a.final_eval) {
            if (a.mode == kModeLBP)
                committed = a.num_messages;
            else if (a.mode == kModeRBP)
                committed = a.rbp_k;
            else
                committed = use_a ? st->sel_a[a.slot_idx] : st->sel_b[a.slot_idx];
            st->committed += committed;
            st->iterations += 1;
        }
        st->last_t = a.t;
        st->last_active = n_t;
        st->last_rmax = st->rmax[a.slot_idx];
        st->evaluated += a.num_messages;
        const long long np_seen = a.has_prev_in_run ? (long long)st->active[a.prev_slot_idx]
                                                    : a.prev_active_host;
        st->last_prev = np_seen;
        if (a.trace) {
            const long long i = a.trace_base + (long long)st->evals;
            if (i >= 0 && i < a.trace_cap) {
                long long* row = a.trace + 4 * i;
                row[0] = (long long)n_t;
                row[1] = (long long)committed;
                row[2] = (long long)(p_low ? 1 : 0);
                row[3] = (long long)st->rmax[a.slot_idx];
            }
        }
        st->evals += 1ull;
        if (converged) {
            st->done = 1u;
            st->conv_t = a.t;
        }
        const int z = (a.slot_idx + 2) & 3;
        st->active[z] = 0ull;
        st->sel_a[z] = 0ull;
        st->sel_b[z] = 0ull;
        st->rmax[z] = 0u;
        st->revert_len[z] = 0u;
    }
}

__global__ void k_init_state(DevState* st) {
    unsigned int* w = (unsigned int*)st;
    const int nw = (int)(sizeof(DevState) / sizeof(unsigned int));
    for (int i = threadIdx.x; i < nw; i += blockDim.x) w[i] = 0u;
    __syncthreads();
    if (threadIdx.x == 0) st->conv_t = -1;
}

__global__ void k_fill(float* p, float v, long long n) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        p[i] = v;
}

// ---------------------------------------------------------------------------
// Eq. (3): beliefs from the node aggregate.
// ---------------------------------------------------------------------------
__global__ void k_marginals_logodds(const int* in_ptr, const float* unary, const float* lam,
                                    float* out, int N) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    float L = unary[n];
    for (int s = in_ptr[n]; s < in_ptr[n + 1]; ++s) L += lam[s];
    out[2 * (long long)n + 1] = 1.0f / (1.0f + expf(-L));
    out[2 * (long long)n + 0] = 1.0f / (1.0f + expf(L));
}

__global__ void k_marginals_generic(const int* in_ptr, const float* unary, const float* m,
                                    float* out, int N, int K) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    float A[kMaxK];
    float mx = -3.402823466e38f;
    for (int x = 0; x < K; ++x) {
        float acc = unary[(long long)n * K + x];
        for (int s = in_ptr[n]; s < in_ptr[n + 1]; ++s) acc += logf(m[(long long)s * K + x]);
        A[x] = acc;
        mx = fmaxf(mx, acc);
    }
    float z = 0.0f;
    for (int x = 0; x < K; ++x) {
        A[x] = expf(A[x] - mx);
        z += A[x];
    }
    for (int x = 0; x < K; ++x) out[(long long)n * K + x] = A[x] / z;
}

// ---------------------------------------------------------------------------
// Greedy top-k for frontier residual BP: most-significant-digit radix select
// over the FP32 bit patterns of the residuals (monotone for values >= 0),
// 4 passes of 8 bits, then a commit that takes every key above the threshold
// and the lowest-slot keys equal to it (slots are ordered by (target, source)).
// ---------------------------------------------------------------------------
constexpr int kSelBlock = 256;
constexpr int kCommitChunk = 4096;

__global__ __launch_bounds__(kSelBlock) void k_rbp_hist(DevState* st, const unsigned int* keys,
                                                        int E, int pass, int slot) {
    __shared__ unsigned int h[256];
    if (st->done || st->active[slot] == 0ull) return;
    for (int i = threadIdx.x; i < 256; i += kSelBlock) h[i] = 0u;
    __syncthreads();
    const unsigned int prefix = pass ? st->sel_prefix : 0u;
    const unsigned int mask = pass ? st->sel_mask : 0u;
    const int shift = 24 - 8 * pass;
    for (int e = blockIdx.x * kSelBlock + threadIdx.x; e < E; e += gridDim.x * kSelBlock) {
        const unsigned int k = keys[e];
        if ((k & mask) == prefix) atomicAdd(&h[(k >> shift) & 255u], 1u);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < 256; i += kSelBlock)
        if (h[i]) atomicAdd(&st->hist[pass][i], h[i]);
}

__global__ __launch_bounds__(kSelBlock) void k_rbp_scan(DevState* st, int pass, unsigned int k,
                                                        int slot) {
    __shared__ unsigned int h[256];
    if (st->done || st->active[slot] == 0ull) return;
    const int i = threadIdx.x;
    h[i] = st->hist[pass][i];
    st->hist[pass][i] = 0u;
    __syncthreads();
    if (i == 0) {
        unsigned int krem = pass ? st->sel_krem : k;
        unsigned int prefix = pass ? st->sel_prefix : 0u;
        unsigned int mask = pass ? st->sel_mask : 0u;
        const int shift = 24 - 8 * pass;
        unsigned int above = 0u;
        int b = 255;
        for (; b > 0; --b) {
            if (above + h[b] >= krem) break;
            above += h[b];
        }
        krem -= above;
        prefix |= (unsigned int)b << shift;
        mask |= 0xFFu << shift;
        st->sel_prefix = prefix;
        st->sel_mask = mask;
        st->sel_krem = krem;
        if (pass == 3) {
            st->sel_ties = h[b];
            st->sel_rank_ties = (h[b] != krem) ? 1u : 0u;
        }
    }
}

__global__ __launch_bounds__(kSelBlock) void k_rbp_tiecount(DevState* st, const unsigned int* keys,
                                                            int E, int slot,
                                                            unsigned int* block_ties) {
    __shared__ unsigned int part[kSelBlock / 64];
    if (st->done || st->active[slot] == 0ull || !st->sel_rank_ties) return;
    const unsigned int T = st->sel_prefix;
    const int beg = blockIdx.x * kCommitChunk;
    const int end = min(E, beg + kCommitChunk);
    unsigned int c = 0;
    for (int e = beg + threadIdx.x; e < end; e += kSelBlock) c += keys[e] == T;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned int s = 0;
        for (int i = 0; i < kSelBlock / 64; ++i) s += part[i];
        block_ties[blockIdx.x] = s;
    }
}

__global__ __launch_bounds__(kSelBlock) void k_rbp_tiescan(DevState* st, int slot,
                                                           unsigned int* block_ties, int nb) {
    if (st->done || st->active[slot] == 0ull || !st->sel_rank_ties) return;
    if (threadIdx.x == 0) {
        unsigned int run = 0;
        for (int b = 0; b < nb; ++b) {
            const unsigned int v = block_ties[b];
            block_ties[b] = run;
            run += v;
        }
    }
}

__global__ __launch_bounds__(kSelBlock) void k_rbp_commit(DevState* st, const unsigned int* keys,
                                                          const float* cand, float* m, int E,
                                                          int row, int all, int slot,
                                                          const unsigned int* block_ties) {
    __shared__ unsigned int wsum[kSelBlock / 64];
    if (st->done || st->active[slot] == 0ull) return;
    const int beg = blockIdx.x * kCommitChunk;
    const int end = min(E, beg + kCommitChunk);
    const unsigned int T = st->sel_prefix;
    const bool rank = !all && st->sel_rank_ties;
    const unsigned int krem = st->sel_krem;
    unsigned int offset = rank ? block_ties[blockIdx.x] : 0u;
    for (int base = beg; base < end; base += kSelBlock) {
        const int e = base + threadIdx.x;
        bool take = false, tie = false;
        if (e < end) {
            if (all) {
                take = true;
            } else {
                const unsigned int k = keys[e];
                take = k > T;
                tie = k == T;
                if (tie && !rank) take = true;
            }
        }
        if (rank) {
            const unsigned long long mk = __ballot(tie);
            const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
            if (lane == 0) wsum[w] = (unsigned int)__popcll(mk);
            __syncthreads();
            unsigned int before = offset;
            for (int i = 0; i < w; ++i) before += wsum[i];
            before += (unsigned int)__popcll(mk & ((1ull << lane) - 1ull));
            if (tie && before < krem) take = true;
            unsigned int tot = 0;
            for (int i = 0; i < kSelBlock / 64; ++i) tot += wsum[i];
            __syncthreads();
            offset += tot;
        }
        if (take)
            for (int x = 0; x < row; ++x) m[(long long)e * row + x] = cand[(long long)e * row + x];
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// Launch wrappers
// ---------------------------------------------------------------------------
hipError_t launch_init_state(DevState* st, hipStream_t s) {
    k_init_state<<<1, 256, 0, s>>>(st);
    return hipGetLastError();
}

hipError_t launch_fill(float* p, float v, long long n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    long long blocks = (n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    k_fill<<<(int)blocks, 256, 0, s>>>(p, v, n);
    return hipGetLastError();
}

template <int KP>
static hipError_t launch_generic_kp(int mode, const EvalArgs& a, int grid, size_t shm,
                                    hipStream_t s) {
    switch (mode) {
    case kModeLBP: k_eval_generic<KP, kModeLBP><<<grid, kBlock, shm, s>>>(a); break;
    case kModeRnBP: k_eval_generic<KP, kModeRnBP><<<grid, kBlock, shm, s>>>(a); break;
    case kModeRBP: k_eval_generic<KP, kModeRBP><<<grid, kBlock, shm, s>>>(a); break;
    default: k_eval_generic<KP, kModeEvalOnly><<<grid, kBlock, shm, s>>>(a); break;
    }
    return hipGetLastError();
}

hipError_t launch_eval(int layout, int kp, int mode, const EvalArgs& a, hipStream_t s) {
    const int grid = 8 * a.tiles_per_xcd;
    if (grid <= 0) return hipSuccess;
    if (layout == kLayoutLogOdds) {
        switch (mode) {
        case kModeLBP: k_eval_logodds<kModeLBP><<<grid, kBlock, 0, s>>>(a); break;
        case kModeRnBP: k_eval_logodds<kModeRnBP><<<grid, kBlock, 0, s>>>(a); break;
        case kModeRBP: k_eval_logodds<kModeRBP><<<grid, kBlock, 0, s>>>(a); break;
        default: k_eval_logodds<kModeEvalOnly><<<grid, kBlock, 0, s>>>(a); break;
        }
        return hipGetLastError();
    }
    const int K = a.num_states;
    const int TS = kTileFloatsGeneric / K;
    const size_t shm = sizeof(float) * (size_t)(2 * TS * K + K * K) +
                       sizeof(unsigned short) * (size_t)TS;
    switch (kp) {
    case 2: return launch_generic_kp<2>(mode, a, grid, shm, s);
    case 4: return launch_generic_kp<4>(mode, a, grid, shm, s);
    case 8: return launch_generic_kp<8>(mode, a, grid, shm, s);
    case 16: return launch_generic_kp<16>(mode, a, grid, shm, s);
    case 32: return launch_generic_kp<32>(mode, a, grid, shm, s);
    case 64: return launch_generic_kp<64>(mode, a, grid, shm, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_finish(const FinishArgs& a, hipStream_t s) {
    k_finish<<<256, kBlock, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_marginals(int layout, int kp, const int* in_ptr, const float* unary,
                            const float* m, float* out, int N, int K, hipStream_t s) {
    (void)kp;
    if (N <= 0) return hipSuccess;
    const int grid = (N + 255) / 256;
    if (layout == kLayoutLogOdds)
        k_marginals_logodds<<<grid, 256, 0, s>>>(in_ptr, unary, m, out, N);
    else
        k_marginals_generic<<<grid, 256, 0, s>>>(in_ptr, unary, m, out, N, K);
    return hipGetLastError();
}

hipError_t launch_rbp_select(DevState* st, const unsigned int* keys, int E, unsigned int k,
                             int slot_idx, unsigned int* block_ties, hipStream_t s) {
    int grid = (E + kSelBlock * 16 - 1) / (kSelBlock * 16);
    if (grid < 1) grid = 1;
    if (grid > 4096) grid = 4096;
    for (int pass = 0; pass < 4; ++pass) {
        k_rbp_hist<<<grid, kSelBlock, 0, s>>>(st, keys, E, pass, slot_idx);
        k_rbp_scan<<<1, kSelBlock, 0, s>>>(st, pass, k, slot_idx);
    }
    const int nb = (E + kCommitChunk - 1) / kCommitChunk;
    k_rbp_tiecount<<<nb > 0 ? nb : 1, kSelBlock, 0, s>>>(st, keys, E, slot_idx, block_ties);
    k_rbp_tiescan<<<1, kSelBlock, 0, s>>>(st, slot_idx, block_ties, nb);
    return hipGetLastError();
}

hipError_t launch_rbp_commit(DevState* st, const unsigned int* keys, const float* cand, float* m,
                             int E, int row, int all, int slot_idx,
                             const unsigned int* block_ties, hipStream_t s) {
    const int nb = (E + kCommitChunk - 1) / kCommitChunk;
    if (nb <= 0) return hipSuccess;
    k_rbp_commit<<<nb, kSelBlock, 0, s>>>(st, keys, cand, m, E, row, all, slot_idx, block_ties);
    return hipGetLastError();
}

}  // namespace bp
