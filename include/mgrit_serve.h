/*
 * mgrit_serve.h -- continuous-batching server of libmgrit: many MGRIT solves
 * (uneven n_x, n_t, order, Courant number, precision) share one GPU.
 *
 * A request is one space-time solve of the problem of mgrit.h (Sec. 2.1-2.2
 * of De Sterck et al., arXiv:1910.03726) with the least-squares coarse
 * operators of Sec. 4 (rule MGRIT_PSI_AUTO).  Life of a request:
 *   submit   -> the server copies u0 and queues the host setup of Psi on a
 *               worker thread.  Psi is cached per (scheme, Courant
 *               number, m): a request whose n_x divides the n_x of a cached
 *               hierarchy with enough levels takes its stencils folded onto
 *               n_x points, otherwise it gets its own fit, which is cached.
 *               Psi decides only how fast a solve converges, not what it
 *               converges to (the fine system's solution, Sec. 2.2);
 *   admit    -> when a slot is free and the plan's device footprint
 *               (mgrit_plan_estimate_bytes) fits the HBM budget next to the
 *               plans already resident; requests whose setup is done are
 *               admitted in submission order, a later request may pass one
 *               that does not fit yet at most `max_bypass` times before
 *               admission waits for it (setup itself runs on several threads,
 *               so a request may become ready before an earlier one); the
 *               admitted request takes the slot together with up to
 *               max_batch-1 later ready requests of the same shape (n_x,
 *               n_t, scheme, m, levels, cycle, relaxation, precision) that
 *               fit, each of which passes the requests between it and the
 *               first (counted against the same bypass limit);
 *   run      -> the slot's group on the slot's own HIP stream as one
 *               mgrit_solve_batch (relaxation launches of the group merged),
 *               so the kernels of all admitted requests overlap on the
 *               device; the solve state stays in device memory until the
 *               group completes;
 *   complete -> the final time level is copied to the host, the plan and
 *               its memory are released and the next request can enter.
 * Conventions: return 0 or a negative MGRIT_E* code (mgrit.h); all
 * pointers are host pointers; the server owns its threads, streams and
 * device memory; calls on one server may come from any host thread.
 */
#ifndef MGRIT_SERVE_H
#define MGRIT_SERVE_H

#include <stddef.h>

#include "mgrit.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mgrit_server_s* mgrit_server_t;

typedef struct {
    int nx, nt, scheme, m;
    int levels;          /* <= 0: coarsen while the coarsest level keeps >= 8
                            points (at least 2 levels)                       */
    int cycle, relax, precision;  /* MGRIT_CYCLE_*, MGRIT_RELAX_*, MGRIT_FP*  */
    double alpha, cfl;   /* wave speed and Courant number                     */
    double tol;          /* residual tolerance (discrete L2 norm)             */
    int maxit;
    unsigned long long seed;  /* U[0,1) initial iterate (splitmix64 stream)   */
    const double* u0;    /* n_x initial values, copied by mgrit_server_submit */
} mgrit_request;

typedef struct {
    long long id;
    int status;          /* MGRIT_OK, MGRIT_ENOTCONV, MGRIT_EDIVERGED or the
                            error of plan creation / setup                  */
    int iterations;
    int levels;
    double final_residual;
    double queue_ms;     /* submit -> admit                                   */
    double run_ms;       /* admit -> complete                                 */
    double latency_ms;   /* submit -> complete                                */
    size_t hbm_bytes;    /* device bytes the request held while resident      */
    long long admit_seq; /* 0-based rank of its admission on this server, -1
                            if it never ran (setup error)                   */
} mgrit_result;

typedef struct {
    long long submitted, completed, active, waiting;
    size_t hbm_in_use, hbm_peak, hbm_budget;
    long long psi_cache_hits, psi_cache_misses;
    long long batches;           /* groups of two or more requests run    */
    long long batched_requests;  /* requests in those groups               */
} mgrit_server_stats;

/* Start a server: `hbm_budget` device bytes for resident plans, `slots`
 * groups running at once (each with its own HIP stream and host thread),
 * `setup_threads` host threads for the coarse-operator setup, `max_bypass`
 * and `max_batch` (1..8; 1 runs every request alone) as above. */
int mgrit_server_create(mgrit_server_t* server, size_t hbm_budget, int slots,
                        int setup_threads, int max_bypass, int max_batch);

/* Queue one request; *id receives its id.  Fails with MGRIT_EINVAL for an
 * invalid request and MGRIT_EBUSY if its footprint exceeds the whole budget. */
int mgrit_server_submit(mgrit_server_t server, const mgrit_request* request,
                        long long* id);

/* Wait up to timeout_ms (< 0: forever) for request `id`; on completion fill
 * *result and, if u_final is not NULL, the n_x values of u^{n_t}, and forget
 * the request.  MGRIT_EBUSY on timeout, MGRIT_EINVAL for an unknown id. */
int mgrit_server_wait(mgrit_server_t server, long long id, int timeout_ms,
                      mgrit_result* result, double* u_final);

int mgrit_server_get_stats(mgrit_server_t server, mgrit_server_stats* stats);

/* Finish every submitted request, then stop the threads and free the
 * streams (NULL is a no-op).  Results not collected are discarded. */
void mgrit_server_destroy(mgrit_server_t server);

#ifdef __cplusplus
}
#endif

#endif /* MGRIT_SERVE_H */
