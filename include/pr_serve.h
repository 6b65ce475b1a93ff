/*
 * pr_serve.h -- a PageRank / PPR query server over graphs resident in device
 * memory (part of libpr.so).
 *
 * Queries are global PageRank (p = e/n) or single-source PPR (p = e_s), both
 * solved by IFP2 (Algorithm 3 of Zhang, Tang, Yao, Liang, arXiv 2302.03245)
 * with the certified L1 stop.  Each registered graph gets an engine: a host
 * thread with its own HIP stream.  An idle engine looks at its queue: with
 * fewer than batch_min waiting queries it solves the oldest one alone (the
 * pr_ppr / pr_solve_ifp2 path); otherwise it starts a batched IFP2 run whose
 * columns are query slots, 8 wide, or 16 wide when more than 8 queries wait
 * and slots is 16.  Between rounds of sweeps a run finishes the columns that
 * met their bound (dangling phase + normalisation for those columns only) and
 * admits waiting queries into free columns while the other columns keep
 * iterating (continuous batching).  A round's sweeps are ordered sweeps over
 * the graph's vertex groups (as in pr_ppr) when the last sweep's frontiers
 * were dense, else synchronous.  A run ends when its last column retires;
 * an 8-wide run whose queue outgrows its free slots stops admitting so that
 * the next run can be 16 wide.  Engines of different graphs run concurrently
 * on the device.
 *
 * Admission by memory footprint.  The budget covers the registered graphs'
 * device bytes (CSR, plans and the caches the server adds) and the query
 * workspaces.  A query runs in its engine's workspace: a column of a 16- or
 * 8-wide batched run (pr_server_footprint(.., 16 or 8, ..) bytes for the run)
 * or a single-vector solve (width 1).  Before each run an engine takes the
 * workspace of the width its queue asks for when the budget has room for it
 * next to the graphs and the other engines' workspaces; else the widest
 * narrower one that fits (8, then 1); else its queries wait.  Engines that wait
 * for memory get it in arrival order: while one waits, idle engines and engines
 * between runs give their workspace back, and running batched runs stop
 * admitting new columns so that they end.  A graph is registered only if it and
 * one single-query workspace fit next to the graphs already registered, so every
 * query can run eventually; a query fails with PR_ENOMEM only when the device
 * refuses the allocation with no other workspace left to wait for.
 *
 * Results equal those of pr_ppr / pr_solve_ifp2 on the same graph within the
 * certified tolerance (the rounding order differs).
 */
#ifndef PR_SERVE_H
#define PR_SERVE_H

#include <stdint.h>

#include "pr.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pr_server pr_server;

typedef struct {
    double c;                 /* damping factor, 0 < c < 1 */
    double l1_tol;            /* certified L1 bound per query, > 0 */
    int32_t residual;         /* PR_RES_FP32 or PR_RES_FP64 */
    int32_t slots;            /* widest batched run per graph engine: 8 or 16 */
    int32_t batch_min;        /* queue length at which an idle engine batches; >= 1 (1: always batch) */
    int32_t sweeps_per_round; /* sweeps between two admission / retirement points, >= 1 */
    int32_t max_sweeps;       /* per query; 0 -> 100000 (a query reaching it ends with PR_ENOCONV) */
    int64_t memory_budget;    /* device bytes for the registered graphs plus the query workspaces;
                                 0 -> 90 % of the device's memory */
} pr_server_opts;

typedef struct {
    int64_t submitted, completed;
    double p50_ms, p99_ms, mean_ms, max_ms; /* submit-to-completion latency of completed queries */
    double edges_per_second;                /* sum of m over completed queries / (last completion - first submit) */
    int64_t device_bytes;                   /* graphs + query workspaces held now */
    int64_t graph_bytes;                    /* registered graphs */
    int64_t peak_bytes;                     /* highest device_bytes so far (<= budget) */
    int64_t budget;                         /* the memory budget in force */
    int64_t memory_waits;                   /* times an engine's queries waited for workspace memory */
    int64_t narrowed_runs;                  /* runs narrower than the queue asked for, for lack of memory */
    int64_t rejected;                       /* queries failed with PR_ENOMEM */
} pr_server_stats;

/* defaults: c 0.85, l1_tol 1e-6, FP32 residuals, 16 slots, batch_min 2, 4 sweeps per round, budget 0 */
void pr_server_opts_default(pr_server_opts *o);

/* PR_EINVAL on invalid options. */
pr_status pr_server_create(const pr_server_opts *o, pr_server **out);

/*
 * Register an uploaded graph; its engine starts immediately.  The graph stays
 * owned by the caller and must outlive the server.  Registration builds the
 * graph's batch plans and stop-rule weights (kept on the graph).  PR_ENOMEM if
 * the graphs registered so far, this one and the largest single-query workspace
 * exceed the budget; PR_EBUSY while the graph is being tuned; PR_EINVAL for a
 * graph uploaded with PR_PEEL.
 */
pr_status pr_server_add_graph(pr_server *s, const pr_graph *g, int32_t *graph_id);

/*
 * Device bytes of one run's workspace on a registered graph: width 1 is a
 * single-vector solve (one query), 8 and 16 a batched run of that many query
 * slots.  PR_EINVAL for an unknown graph id or another width.
 */
pr_status pr_server_footprint(pr_server *s, int32_t graph_id, int32_t width, int64_t *bytes);

/*
 * Queue a query.  source = -1: global PageRank; else single-source PPR from that
 * vertex (original id).  pi_device: device buffer of n doubles receiving the
 * result, owned by the caller, untouched until the query completes.
 */
pr_status pr_server_submit(pr_server *s, int32_t graph_id, int32_t source, double *pi_device, int64_t *request_id);

/*
 * Wait for a query (timeout_seconds < 0: no limit).  Returns the query's status
 * (PR_OK, PR_ENOCONV, or a negative error); PR_EDEVICE with "timeout" when the
 * limit expires first (the query stays queued).  st (optional) receives its
 * statistics; seconds_solve is its submit-to-completion latency.  A completed
 * query can be waited for once.
 */
pr_status pr_server_wait(pr_server *s, int64_t request_id, double timeout_seconds, pr_stats *st);

pr_status pr_server_get_stats(pr_server *s, pr_server_stats *out);

/* Stop the engines (queued queries complete with PR_EINVAL) and free the server. */
pr_status pr_server_destroy(pr_server *s);

#ifdef __cplusplus
}
#endif

#endif /* PR_SERVE_H */
