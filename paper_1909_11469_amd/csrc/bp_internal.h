// Internal declarations shared by the host side (bp_api.cpp) and the kernels
// (bp_kernels.hip) of libbp.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bp {

// Tile limits of the evaluation kernel.  A tile is a run of consecutive target
// nodes whose incoming messages (a contiguous slot range) are processed by one
// 256-thread block; the slot limit depends on the message layout.
constexpr int kBlock = 256;
constexpr int kTileSlotsLogOdds = 2048;  // K = 2 log-odds layout: 8 slots per thread
constexpr int kTileFloatsGeneric = 4096; // [E][K] layout: tile slots = this / K
constexpr int kTileNodesMax = 2048;      // nodes per tile (owner index fits in u16)
constexpr int kMaxK = 64;

enum Layout : int { kLayoutLogOdds = 0, kLayoutGeneric = 1 };
enum PairDev : int { kPairIsing = 0, kPairShared = 1, kPairSharedAsym = 2, kPairDense = 3 };
enum Mode : int { kModeLBP = 0, kModeRnBP = 1, kModeRBP = 2, kModeEvalOnly = 3 };

// Per-run scalar state on the device.  Per-iteration accumulators are indexed
// by t & 3 so that iteration t can read n_{t-1} while iteration t+1 accumulates.
struct DevState {
    unsigned long long active[4];   // n_t: residual > eps
    unsigned long long sel_a[4];    // frontier size under the larger keep threshold
    unsigned long long sel_b[4];    // frontier size under the smaller keep threshold
    unsigned int rmax[4];           // max residual as FP32 bits (residuals are >= 0)
    unsigned int revert_len[4];     // entries of the revert list
    unsigned int done;              // set once an evaluation finds n_t == 0
    unsigned int pad0;
    long long conv_t;               // t of that evaluation, -1 if none
    long long last_t;               // t of the last evaluation
    unsigned long long last_active; // n_t of the last evaluation
    unsigned long long evaluated;   // Eq. (2) evaluations in this run
    unsigned long long committed;   // committed messages in this run
    unsigned long long iterations;  // commits in this run
    unsigned int last_rmax;
    unsigned int pad1;
    unsigned long long evals;       // evaluations in this run
    long long last_prev;            // n_{t-1} as seen by the last evaluation (-1 if none)
    // greedy top-k selection (frontier residual BP)
    unsigned int hist[4][256];      // digit histograms of the 4 radix passes
    unsigned int sel_prefix;        // key bits fixed so far
    unsigned int sel_mask;
    unsigned int sel_krem;          // how many more keys to take among the prefix
    unsigned int sel_ties;          // keys equal to the final threshold
    unsigned int sel_rank_ties;     // 1 if ties must be ranked by slot
    unsigned int pad2[3];
};

struct EvalArgs {
    const int* tile_start;      // [T+1] first node of each tile
    int num_tiles;
    int tiles_per_xcd;          // ceil(T / 8): block -> tile remap for XCD locality
    const int* in_ptr;          // [N+1] slot range of each target node
    const int* rev;             // [E] slot of the reverse message
    const int* src;             // [E] source node of the message in each slot
    const float* coupling;      // [E] Ising J per slot
    const float* unary;         // log-odds [N] (K = 2 log-odds layout) or log psi [N][K]
    const float* pair;          // shared [K][K] (and its transpose after it) or dense [E][K][K]
    const unsigned char* orient;// [E] 1 if the shared table must be transposed for the slot
    const float* m_in;          // m^t
    float* m_out;               // m^{t+1} (LBP / RnBP); unused by RBP and eval-only
    float* cand;                // RBP candidates, same layout as m
    unsigned int* keys;         // RBP residual keys [E]
    int* revert_list;           // RnBP: slots to restore if p_t takes the smaller value
    DevState* st;
    int num_states;             // K
    int pair_kind;              // PairDev
    int slot_base;              // first slot of tile (unused, reserved)
    unsigned int t;             // global iteration number (RNG counter word 2)
    float eps;
    unsigned int thr_a;         // larger keep threshold on the 24-bit uniform
    unsigned int thr_b;         // smaller keep threshold
    unsigned int key0, key1;    // Philox key
    int slot_idx;               // t & 3
};

struct FinishArgs {
    DevState* st;
    int slot_idx;               // t & 3
    int prev_slot_idx;          // (t - 1) & 3
    int has_prev_in_run;        // n_{t-1} was counted on the device in this run
    long long prev_active_host; // n_{t-1} from the iteration state (first iteration)
    long long t;
    int mode;
    int dynamic_p;
    int low_is_a;               // 1 if p (low) has the larger threshold
    int thresholds_differ;      // thr_a != thr_b
    double ratio_threshold;
    int final_eval;             // evaluation after the last allowed commit
    unsigned long long num_messages;
    unsigned long long rbp_k;   // RBP frontier size
    const int* revert_list;
    const float* m_in;
    float* m_out;
    int row;                    // floats per message (1 or K)
    long long* trace;           // optional [cap][4]: t, n_t, |F_t|, rmax bits
    long long trace_cap;
    long long trace_base;       // index of this run's first iteration in the trace
};

// Launch wrappers (bp_kernels.hip).  All return the hipError_t of the launch.
hipError_t launch_init_state(DevState* st, hipStream_t s);
hipError_t launch_fill(float* p, float v, long long n, hipStream_t s);
hipError_t launch_eval(int layout, int kp, int mode, const EvalArgs& a, hipStream_t s);
hipError_t launch_finish(const FinishArgs& a, hipStream_t s);
hipError_t launch_marginals(int layout, int kp, const int* in_ptr, const float* unary,
                            const float* m, float* out, int N, int K, hipStream_t s);
// frontier residual BP selection
hipError_t launch_rbp_select(DevState* st, const unsigned int* keys, int E, unsigned int k,
                             int slot_idx, unsigned int* block_ties, hipStream_t s);
hipError_t launch_rbp_commit(DevState* st, const unsigned int* keys, const float* cand,
                             float* m, int E, int row, int all, int slot_idx,
                             const unsigned int* block_ties, hipStream_t s);

}  // namespace bp
