/*
 * pr_warm.h -- resuming IFP2 after the graph changes (part of libpr.so).
 *
 * A state holds what a forward-push solve has accumulated: the reserve pibar and
 * the residual h of every vertex (original ids, device memory, FP64), in the form
 * of Algorithm 2 (IFP1), where the exact unnormalised PageRank is
 * pibar + (I - cP)^{-1} h for the current graph (Eq. 4; every push of section 3
 * keeps this sum fixed).  IFP2 solves read and write it in that form: at the end
 * of a solve the mass its vertices took has also been passed on to dangling
 * vertices, as IFP2's phase 2 does.
 *
 * After edges change, pr_state_update adds c (P_new - P_old) pibar to h, which
 * restores the identity for the new graph; a warm solve then pushes only what the
 * change disturbed.  Residuals may become negative: warm solves take a vertex
 * when |h_i| > xi, and their certified bound accounts for signed residuals.
 */
#ifndef PR_WARM_H
#define PR_WARM_H

#include <stdint.h>

#include "pr.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pr_state pr_state;

/*
 * A cold state for graphs of n >= 1 vertices: pibar = 0, h = n p / sum(p) with
 * p the host array of n personalisation weights (non-negative, finite, positive
 * sum), or uniform p when p is NULL (h = 1 everywhere, as Algorithms 2 and 3
 * start).  Single-source PPR: p = e_s.  PR_EINVAL on bad arguments.
 */
pr_status pr_state_create(int64_t n, const double *p, pr_state **out);
pr_status pr_state_free(pr_state *s);

/*
 * IFP2 (Algorithm 3) on g, starting from the state s and leaving its final
 * reserve and residual in it.  g must have the state's n; the first solve fixes
 * the damping factor o->c of the state, later solves and updates must use the
 * same one.  Options as pr_solve_ifp2 except p (taken from the state) and
 * PR_IFP2_LITERAL (rejected); graphs uploaded with PR_PEEL are rejected.  The
 * stop rule and pi / st as pr_solve_ifp2; the bound covers negative residuals.
 */
pr_status pr_solve_ifp2_warm(const pr_graph *g, const pr_opts *o, pr_state *s, double *pi, pr_stats *st);

/*
 * Carry the state from g_old (the graph of its last solve) to g_new (same n):
 * h += c (P_new - P_old) pibar over the k sources in `changed` (host array of
 * original ids whose out-edge lists differ), or over every vertex when changed is
 * NULL.  A source left out although its edges changed leaves the state wrong for
 * g_new.  PR_EINVAL if no solve has fixed c yet, on size mismatch, bad ids or
 * a graph uploaded with PR_PEEL.
 */
pr_status pr_state_update(pr_state *s, const pr_graph *g_old, const pr_graph *g_new, const int32_t *changed,
                          int32_t k);

/* Copy the state to host arrays of n doubles (either may be NULL). */
pr_status pr_state_read(const pr_state *s, double *pibar, double *h);

#ifdef __cplusplus
}
#endif

#endif /* PR_WARM_H */
