/*
 * pr_set.h -- many independent graphs solved together (part of libpr.so).
 *
 * A graph set holds k directed graphs uploaded as one block-diagonal union in
 * device memory.  pr_set_solve_ifp2 runs IFP2 (Algorithm 3 of Zhang, Tang,
 * Yao, Liang, arXiv 2302.03245) on all of them at once: every sweep is one
 * launch sequence over the union (reserve, management, push or pull), with the
 * damping factor, the push threshold, the stop rule and the final
 * normalisation (Eq. 4) kept per graph.  Each graph's result is its global
 * PageRank (uniform p) with its own certified L1 bound; a graph that meets its
 * bound stops moving mass while the others continue.
 *
 * Graph g's vertices are 0 .. n[g]-1 in its own CSR; in the solution array they
 * sit at offset off[g] = n[0] + ... + n[g-1].
 */
#ifndef PR_SET_H
#define PR_SET_H

#include <stdint.h>

#include "pr.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pr_graph_set pr_graph_set;

typedef struct {
    int64_t k;                  /* graphs in the set */
    int64_t n, m;               /* totals over the set */
    int64_t n_dangling, m_dangling;
    int64_t device_bytes;
    double seconds_upload;
    int64_t groups;             /* vertex groups of ordered sweeps per graph (1: none) */
    int64_t tile_items;         /* rows + edges per sweep tile */
    int64_t ordered;            /* 1 if set solves use ordered sweeps */
} pr_set_info_t;

/*
 * Upload k >= 1 graphs.  n[g] >= 1 vertices; row_ptr[g] (host, n[g] + 1 int64,
 * non-decreasing, row_ptr[g][0] = 0) and col[g] (host, row_ptr[g][n[g]] int32,
 * each in [0, n[g])) give graph g in CSR with out-edges per row.  Duplicate
 * edges count with multiplicity.  Totals must stay below 2^31 vertices and 2^31
 * edges.  flags: PR_TILE_SHIFT, PR_GROUPS(q) (vertex groups per graph for ordered
 * sweeps, as for one graph: 1 = none; 0 selects 4).  The inputs are copied.
 * PR_EINVAL on a malformed graph (nothing is uploaded), PR_ENOMEM / PR_EDEVICE
 * on allocation or device failure.
 */
pr_status pr_set_upload(int32_t k, const int64_t *n, const int64_t *const *row_ptr, const int32_t *const *col,
                        uint32_t flags, pr_graph_set **out);
pr_status pr_set_free(pr_graph_set *s);
pr_status pr_set_info(const pr_graph_set *s, pr_set_info_t *out);

/*
 * IFP2 on every graph of the set, uniform personalisation.
 *   c    k damping factors in (0, 1), or NULL for o->c on every graph.
 *   o    o->stop PR_STOP_L1: graph g stops once its certified L1 bound is
 *        <= o->l1_tol (thresholds xi_g derived per graph); PR_STOP_XI: every
 *        graph uses threshold o->xi and stops when no vertex exceeds it.
 *        o->residual, o->max_sweeps (for the whole set), o->stream; flags
 *        PR_OUT_DEVICE, PR_FORCE_PUSH, PR_FORCE_PULL, PR_JACOBI.
 *        With vertex groups, sweeps over a dense frontier are ordered: group
 *        by group (in every graph at once), each takes its residuals and
 *        gathers its pushes before the next group takes its own, as in
 *        pr_solve_ifp2; a forced scatter mode or PR_JACOBI keeps synchronous
 *        sweeps.
 *   pi   sum of n[g] doubles (host, or device with PR_OUT_DEVICE), graph g at
 *        offset off[g]; written only when the status is not negative.
 *   st   k entries or NULL: per-graph sweeps, pushes, edges, residual and bound;
 *        seconds_solve is the time of the whole set solve.
 * Returns PR_OK when every graph converged, PR_ENOCONV when some graph reached
 * max_sweeps first (its entry of st says how far it got).
 */
pr_status pr_set_solve_ifp2(const pr_graph_set *s, const double *c, const pr_opts *o, double *pi, pr_stats *st);

/*
 * Autotuner of the set's sweep schedule, as pr_graph_tune for one graph: times
 * pr_set_solve_ifp2 with the damping factors c (or NULL) and options o for every
 * tile size s in {2, 3, 4} with synchronous and, when the set has vertex groups,
 * ordered sweeps, `reps` solves each after one warm-up (reps <= 0: 2), and keeps
 * the fastest.  rep->sweeps holds the largest per-graph sweep count of each
 * candidate.  Results do not change beyond rounding order.  No other call may use
 * the set meanwhile.  rep may be NULL.  PR_EINVAL on bad options or forced modes.
 */
pr_status pr_set_tune(pr_graph_set *s, const double *c, const pr_opts *o, int32_t reps, pr_tune_report *rep);

#ifdef __cplusplus
}
#endif

#endif /* PR_SET_H */
