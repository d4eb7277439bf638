// Internal declarations shared by the host side (bp_api.cpp) and the kernels
// (bp_kernels.hip) of libbp.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/bp.h"

namespace bp {

// Tile limits of the evaluation kernel.  A tile is a run of consecutive source
// nodes whose outgoing messages (a contiguous slot range) are processed by one
// block; the slot limit depends on the message layout.
#ifndef BP_BLOCK
#define BP_BLOCK 256
#endif
constexpr int kBlock = BP_BLOCK;
#ifndef BP_BLOCK_LOGODDS
#define BP_BLOCK_LOGODDS 256
#endif
constexpr int kBlockLO = BP_BLOCK_LOGODDS;  // threads of the K = 2 tile kernels
static_assert(kBlockLO % 64 == 0 && kBlockLO <= kBlock, "K = 2 tile kernel block size");
#ifndef BP_TILE_SLOTS_LOGODDS
#define BP_TILE_SLOTS_LOGODDS 512
#endif
constexpr int kTileSlotsLogOdds = BP_TILE_SLOTS_LOGODDS;  // K = 2 log-odds layout
constexpr int kTileNodesLogOdds = kTileSlotsLogOdds / 2;  // nodes per log-odds tile
#ifndef BP_TILE_FLOATS_GENERIC
#define BP_TILE_FLOATS_GENERIC 4096
#endif
constexpr int kTileFloatsGeneric = BP_TILE_FLOATS_GENERIC;  // [E][K] layout: tile slots = this / K
constexpr int kTileNodesMax = 2048;      // nodes per tile (owner index fits in u16)
constexpr int kMaxK = 64;
constexpr int kMaxKRagged = 128;  // largest K_i of a graph with per-variable state counts
// Ragged layout: a variable's slots are evaluated by one wave together (its
// aggregate shared, the outputs of all its slots at once) when its cavity
// vectors (deg K_i floats) and its outputs (P = sum of K_j over its slots)
// each fit kRaggedFlat floats of the wave's LDS and its product work P K_i is
// at most kRaggedHeavyWork; every other variable ("heavy") gives each of its
// slots a wave of its own, so that no wave carries a long chain of table
// loads.  Host (heavy slot list) and kernel decide with the same function.
#ifndef BP_RAGGED_FLAT
#define BP_RAGGED_FLAT 1024
#endif
constexpr int kRaggedFlat = BP_RAGGED_FLAT;
constexpr int kRaggedMaxDeg = 64;
#ifndef BP_RAGGED_HEAVY_WORK
#define BP_RAGGED_HEAVY_WORK 16384
#endif
constexpr int kRaggedHeavyWork = BP_RAGGED_HEAVY_WORK;
__host__ __device__ inline bool ragged_flat(int deg, int ki, int p) {
    return deg <= kRaggedMaxDeg && deg * ki <= kRaggedFlat && p <= kRaggedFlat &&
           p * ki <= kRaggedHeavyWork;
}

// 0: one log-odds value per message (K = 2 Ising); 1: K floats per message;
// 2: K_j floats per message i -> j (per-variable state counts)
enum Layout : int { kLayoutLogOdds = 0, kLayoutGeneric = 1, kLayoutRagged = 2 };
enum PairDev : int { kPairIsing = 0, kPairShared = 1, kPairSharedAsym = 2, kPairDense = 3 };
enum Mode : int { kModeLBP = 0, kModeRnBP = 1, kModeRBP = 2, kModeEvalOnly = 3 };
// EvalArgs::sched of residual splash runs: the evaluation kernels run their
// frontier-RBP instantiation (candidates and residual keys), and the splash
// kernels count the commits themselves.
constexpr int kModeRS = 4;
constexpr int kSplashMaxDepth = 2;

// Per-iteration counters.  Blocks add into one of kCounterCopies copies (by
// block index), each copy on its own 128-byte line, so that the atomics of a
// launch do not queue on a single address; readers sum the copies.
// Iteration u uses copy set u & 3: iteration t accumulates into t & 3 while
// its prologue reads the finished sets of t - 1 and t - 2 and clears (t + 1) & 3.
constexpr int kCounterCopies = 64;
struct alignas(128) CounterLine {
    unsigned long long active;  // residual > eps
    unsigned long long sel_a;   // frontier size under the larger keep threshold
    unsigned long long sel_b;   // frontier size under the smaller keep threshold
    unsigned int rmax;          // max residual as FP32 bits (residuals are >= 0)
    unsigned int pad[25];
};
static_assert(sizeof(CounterLine) == 128, "one counter copy per cache line");

// Per-run scalar state on the device.
struct DevState {
    unsigned int in_sel[4];         // which of the two buffers held m^t (by t & 3)
    unsigned int done;              // set once an evaluation finds n_t == 0
    unsigned int last_rmax;
    unsigned int rbp_skip;          // frontier residual BP: nothing to commit this iteration
    unsigned int pad0;
    long long conv_t;               // t of that evaluation, -1 if none
    long long last_t;               // t of the last closed evaluation
    unsigned long long last_active; // n_t of the last closed evaluation
    long long last_prev;            // n_{t-1} seen by the last closed evaluation (-1 if none)
    unsigned long long evaluated;   // Eq. (2) evaluations in this run
    unsigned long long committed;   // committed messages in this run
    unsigned long long iterations;  // commits in this run
    unsigned long long evals;       // evaluations closed in this run
    // greedy top-k selection (frontier residual BP)
    unsigned int hist[16][256];     // copies of the digit histogram of a radix pass
    unsigned int sel_prefix;        // key bits fixed so far
    unsigned int sel_mask;
    unsigned int sel_krem;          // how many more keys to take among the prefix
    unsigned int sel_ties;          // keys equal to the final threshold
    unsigned int sel_rank_ties;     // 1 if ties must be ranked by slot
    unsigned int pad2[3];
    // sparse re-evaluation: n_t by t & 3
    unsigned long long sp_n[4];
    // residual splash: length of the variable list of each level
    unsigned int rs_count[kSplashMaxDepth + 1];
    unsigned int pad3;
};

struct EvalArgs {
    const int* tile_start;      // [T+1] first node of each tile ([E][K] layout)
    const int* tile_slot;       // [T+1] first slot of each tile ([E][K] layout)
    const int* tiles4;          // log-odds layout: [T][4] {n0, n1, s0, s1} of the regular tiles
    const int* big4;            // log-odds layout: [num_big][4] single-node tiles over the limit
    int num_tiles;
    int tiles_per_xcd;          // ceil(T / 8): block -> tile remap for XCD locality
    int num_big;
    int pipe_grid;              // blocks of the persistent log-odds kernel (multiple of 8)
    const int* node_ptr;        // [N+1] slot range of each source node
    const int* rev;             // [E] slot of the reverse message
    const short* rev16;         // K = 2 log-odds layout: rev[e] - e as 16 bits, or nullptr
    const float* coupling;      // [E] Ising J per slot
    const float* unary;         // log-odds [N] (K = 2 log-odds layout) or log psi [N][K]
    const float* pair;          // shared [K][K] or dense [E][K][K]
    const unsigned char* orient;// [E] 1 if the shared table must be transposed for the slot
    // per-variable state counts (ragged layout)
    const int* kv;              // [N] K_i
    const int* uoff;            // [N+1] first unary (and belief) entry of each variable
    const int* moff;            // [E+1] first message entry of each slot (K_j entries)
    const int* toff;            // [E+1] first table entry of each slot (K_i x K_j, x_i major)
    const int* heavy;           // [num_heavy][2] {slot, source} of the slots of heavy variables
    int num_heavy;
    const float* in_buf[2];     // m^t: candidates chosen by p_{t-1} (both equal on a run's first launch)
    float* out_buf[2];          // m^{t+1} under the larger [0] and smaller [1] keep threshold
    float* cand;                // RBP candidates, same layout as m
    unsigned int* keys;         // RBP residual keys [E]
    DevState* st;
    CounterLine* ctr;           // [4][kCounterCopies]
    int num_states;             // K
    int pair_kind;              // PairDev
    unsigned int t;             // global iteration number (RNG counter word 2)
    long long it;               // launch index within this run
    int sched;                  // Mode of the run (LBP / RnBP / RBP)
    int after_final;            // k_close_run after an evaluation-only launch
    float eps;
    unsigned int thr_a;         // larger keep threshold on the 24-bit uniform
    unsigned int thr_b;         // smaller keep threshold
    unsigned int key0, key1;    // Philox key
    int two_outputs;            // RnBP with differing thresholds: write out_buf[1] too
    int row_flags;              // K = 32 matrix-core kernel with two_outputs: one full row
                                // per message (the outcome the last iteration chose), the
                                // other outcome only where they differ, flagged by the
                                // sign bit of the full row's first entry
    int dynamic_p;
    int low_is_a;               // 1 if p (low) has the larger threshold
    int sel0;                   // buffer index of the start state (recorded, first launch)
    double ratio_threshold;
    long long prev_active_host; // n_{t-1} from the iteration state (second launch)
    unsigned long long num_messages;
    int num_nodes;
    int tile_nodes_max;         // [E][K] layout: most nodes in one regular tile
    int tile_big;               // [E][K] layout: 1 if some node's slots exceed a tile
    int no_mfma;                // K = 32 shared table on the vector units (not the matrix cores)
    int mfma_bf16;              // K = 32 shared table: BF16 operands on the matrix cores
    int hist0;                  // frontier RBP, K = 2 kernel: also count the first radix
                                // digit of every residual key into st->hist
    unsigned long long rbp_k;   // RBP frontier size
    // sparse re-evaluation (K = 2 log-odds layout, RnBP)
    unsigned char* dirty;       // [N] 1 if a message into the node was committed
    unsigned char* hasact;      // [N] 1 if a slot of the node has residual > eps
    int* dst;                   // [E] target node of each slot
    int sp_first;               // first sparse iteration of a run (stored residuals invalid)
};

// One graph of a serving batch (device memory).  `a` holds the graph's
// arguments as bp_run would set them; before every batched launch a small
// kernel sets the per-launch fields (t, it, in_buf, out_buf, the mode of the
// final evaluation) from the launch index.
struct BatchGraph {
    EvalArgs a;
    float* msg[4];          // message buffer b of pair p at msg[2 p + b]
    long long first;        // global launch index of the graph's first evaluation
    long long max_iters;    // commits allowed; launch max_iters evaluates only
    int mode;               // kModeLBP or kModeRnBP
    int mode_now;           // this launch: mode, or kModeEvalOnly for the final evaluation
    int skip;               // this launch: 1 if the graph is not evaluated
    int pad;
};

// Control block of a server's batched launches (device memory): the index of
// the next launch (read by k_batch_advance, advanced by the evaluation kernel,
// so that recorded launch sequences can be replayed) and the tile-list length.
struct BatchCtl {
    long long launch;
    int entries;
    int pad[13];
};

// Launch wrappers (bp_kernels.hip).  All return the hipError_t of the launch.
// One batched iteration: k_batch_advance, then the persistent evaluation
// kernel on `grid` blocks.
hipError_t launch_eval_batch(BatchGraph* graphs, int num_graphs, const int* list, BatchCtl* ctl,
                             int grid, hipStream_t s);
// The same `launches` iterations as a HIP graph of kernel nodes only.
hipError_t batch_graph_nodes(BatchGraph* graphs, int num_graphs, const int* list, BatchCtl* ctl,
                             int grid, int launches, hipGraph_t* out);
hipError_t launch_batch_status(const BatchGraph* graphs, int num_graphs, unsigned int* done,
                               hipStream_t s);
hipError_t launch_init_state(DevState* st, CounterLine* ctr, hipStream_t s);
hipError_t launch_fill(float* p, float v, long long n, hipStream_t s);
hipError_t launch_eval(int layout, int kp, int mode, const EvalArgs& a, hipStream_t s);
hipError_t launch_close_run(const EvalArgs& a, hipStream_t s);
int logodds_blocks_per_cu(int mode);
hipError_t launch_marginals(int layout, int kp, const int* node_ptr, const int* rev,
                            const float* unary, const float* m, float* out, int N, int K,
                            hipStream_t s);
// ragged layout: Eq. (3) into out [sum K_i] (a.in_buf[0] holds the messages),
// and the uniform start state 1 / K_j of every message into m
hipError_t launch_marginals_ragged(const EvalArgs& a, float* out, hipStream_t s);
hipError_t launch_fill_ragged(float* m, const int* moff, int E, hipStream_t s);
// sparse re-evaluation: one iteration (evaluate the dirty nodes, then close and
// commit), and the per-graph setup (target index, every node dirty)
hipError_t launch_sparse_iteration(const EvalArgs& a, hipStream_t s);
hipError_t launch_sparse_setup(const EvalArgs& a, int build_dst, hipStream_t s);
hipError_t launch_sparse_rmax(const EvalArgs& a, hipStream_t s);  // R_t after a sparse run
// After a run with row_flags: the state m^t (rows of buffer `prim` of pair
// msg, flagged rows taken from the other buffer when `sel` differs) made
// whole in buffer `prim`.
hipError_t launch_resolve_rows(float* const* pair_bufs, int prim, int sel, long long E, int K,
                               hipStream_t s);
// frontier residual BP selection
hipError_t launch_rbp_gate(DevState* st, const CounterLine* ctr, int slot_idx, hipStream_t s);
// gate_ctr: the counter set of the evaluation (the first scan sets rbp_skip
// from it), or null when rbp_skip is already set; hist0_done: the evaluation
// kernel already counted the first digit.
hipError_t launch_rbp_select(DevState* st, const unsigned int* keys, const int* rev, int E,
                             unsigned int k, const CounterLine* gate_ctr, int hist0_done,
                             unsigned int* block_ties, hipStream_t s);
// Extra work of the top-k commit under sparse re-evaluation (on = 0: none):
// committed slots get residual key 0 and their targets are marked dirty, and
// the committed slots with residual > eps leave the running count of set `set`.
struct RbpSparse {
    unsigned char* dirty;
    const int* dst;
    CounterLine* ctr;
    float eps;
    int set;
    int on;
};
// moff (ragged layout, else nullptr): slot e's row is cand[moff[e] .. moff[e+1]).
hipError_t launch_rbp_commit(DevState* st, unsigned int* keys, const int* rev,
                             const float* cand, float* m, int E, int row, int all, int slot_idx,
                             const unsigned int* block_ties, const RbpSparse& sp,
                             const int* moff, hipStream_t s);
// frontier residual BP under sparse re-evaluation: evaluate the dirty nodes,
// then close the evaluation (one wave) and gate the top-k kernels
hipError_t launch_sparse_rbp_eval(const EvalArgs& a, hipStream_t s);

// Residual splash (K = 2 log-odds layout, messages committed in place).
struct RsArgs {
    DevState* st;
    const int* node_ptr;        // [N+1]
    const int* rev;             // [E]
    const int* dst;             // [E] target variable of each slot
    const float* unary;         // [N] log-odds unaries
    const float* coupling;      // [E]
    const unsigned int* keys;   // [E] residual keys of the evaluation of iteration t
    float* m;                   // [E] messages, updated in place
    float* cand;                // [E] candidates of the level being updated
    unsigned int* vkey;         // [N] variable residual keys
    unsigned int* mark;         // [depth + 1][N]: tag if the variable is in level d
    int* list;                  // [depth + 1][N]: the variables of each level
    int num_nodes;
    int depth;                  // h
    unsigned int tag;           // marks of this iteration
};
// Device bytes of the splash buffers of a graph of N variables (256-aligned parts).
size_t splash_bytes(int num_nodes);
hipError_t launch_rs_gate(DevState* st, const CounterLine* ctr, int slot_idx, hipStream_t s);
// variable keys, top-k roots (ties by id), level marks and lists
hipError_t launch_rs_select(const RsArgs& r, unsigned int k, int all, unsigned int* block_ties,
                            hipStream_t s);
// the updates of level d (evaluate the level's out-messages, then commit them)
hipError_t launch_rs_level(const RsArgs& r, int d, hipStream_t s);
hipError_t launch_fill_u32(unsigned int* p, unsigned int v, long long n, hipStream_t s);

// Host side (bp_api.cpp) used by other translation units of the library.
// bp_run with its per-run device scratch (iteration state, counters, top-k
// tie counts) taken from `scratch` instead of the graph's memory, and without
// creating events or buffers.
size_t run_scratch_bytes(long long num_messages, long long num_nodes);
int run_with_scratch(bp_graph* g, int schedule, double eps, double p, uint64_t seed,
                     const bp_run_opts* opts, bp_run_stats* stats, char* scratch,
                     size_t scratch_bytes);
int graph_device(const bp_graph* g);
// Record an error for bp_last_error() and return `code`.
int report_error(int code, const char* msg);

}  // namespace bp
