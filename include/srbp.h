/*
 * srbp.h -- C ABI of libsrbp: serial residual belief propagation on the host
 * CPU, the paper's serial baseline (SRBP, Sec. II-B and Sec. III-B).
 *
 * Residual BP updates one message at a time, always the message with the
 * largest residual (Eq. (4), L-infinity norm of the change of the normalised
 * message), and every update uses the newest messages (asynchronous BP,
 * Sec. II-B).  After m_{i->j} is committed, only the messages j -> k (k != i)
 * read it, so only their candidates and residuals are recomputed; a priority
 * queue (an indexed binary heap here) yields the next message.  Ties are taken
 * in (target, source) ascending order.  The solve stops when the largest
 * residual is <= eps (converged), after max_updates commits, or when the time
 * limit has passed.
 *
 * The problem is described by bp_graph_desc of bp.h (N, K <= 64, edges, log
 * unaries, Ising / shared / dense pairwise potentials; stream, workspace and
 * flags are ignored; var_states must be NULL).  Messages start uniform and are FP64; each candidate is
 * the literal product of Eq. (2) (no log domain, no division), so a solve is
 * reproducible bit for bit.  All arrays are host memory owned by the caller.
 * The library holds no state between calls and is thread-safe; the error
 * string is per thread.
 */
#ifndef SRBP_H
#define SRBP_H

#include <stdint.h>

#include "bp.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct srbp_stats {
    int64_t updates;       /* messages committed */
    int32_t converged;     /* 1 if the largest residual reached <= eps */
    int32_t timed_out;     /* 1 if the time limit stopped the solve */
    double max_residual;   /* largest residual when the solve stopped */
    double seconds;        /* wall time of the solve loop (setup excluded) */
    int64_t evaluations;   /* Eq. (2) evaluations, the E initial ones included */
} srbp_stats;

/* Solve desc with serial residual BP.
 *   eps           convergence threshold, finite and >= 0
 *   max_updates   cap on commits (>= 0)
 *   time_limit_s  wall-clock cap in seconds (<= 0: none); checked every 1024 commits
 *   out_marginals host [N][K] FP64 Eq. (3) beliefs at the end, or NULL
 *   out_msgs      host [E][K] FP64 messages at the end in canonical order
 *                 (row 2u = edges[u][0] -> edges[u][1], 2u + 1 the reverse), or NULL
 *   trace         host [trace_len]: message ids of the first trace_len commits, or NULL
 *   stats         or NULL
 * Returns BP_OK if converged, BP_NOT_CONVERGED if a cap stopped it, BP_EINVAL
 * for an invalid problem or argument, BP_ENOMEM if host memory runs out. */
int srbp_solve(const bp_graph_desc* desc, double eps, int64_t max_updates, double time_limit_s,
               double* out_marginals, double* out_msgs, int64_t* trace, int64_t trace_len,
               srbp_stats* stats);

/* Description of the last error in the calling thread ("" if none). */
const char* srbp_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* SRBP_H */
