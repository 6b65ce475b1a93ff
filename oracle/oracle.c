/*
 * oracle.c -- plain serial FP64 CPU oracle for PageRank / personalized
 * PageRank and for the IFP1 / IFP2 forward-push algorithms of
 * Zhang, Tang, Yao, Liang, "Two Parallel PageRank Algorithms via Improving
 * Forward Push" (arXiv 2302.03245).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may call, link or
 * load this file: only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark use it.  It shares no code, header or table with the GPU
 * library; it builds its own degrees and dangling flags from the CSR it is
 * given.
 *
 * Graph input: n vertices, CSR row_ptr[n+1] (int64), col[m] (int32); the
 * edges i -> col[row_ptr[i] .. row_ptr[i+1]) with multiplicity.  deg(i) is the
 * row length (a self-loop counts).  A vertex with deg 0 is dangling.
 * p == NULL means the uniform vector e/n; otherwise p >= 0 with sum > 0 and
 * it is used as p / sum(p).
 *
 * Definitions followed (section 2.1 of the paper): P is the adjacency matrix
 * normalised by out-degree with zero columns at dangling vertices,
 * P' = P + p d^T, P'' = c P' + (1-c) p e^T, and the PageRank vector solves
 * pi = P'' pi with sum(pi) = 1 (Eq. 1); equivalently (I - cP') pi = (1-c) p
 * (Eq. 2) and pi = normalize((I - cP)^{-1} p) (Eq. 4).
 *
 * All sums of many terms use Neumaier's compensated summation.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { OR_OK = 0, OR_NOCONV = 1, OR_EINVAL = -1, OR_ENOMEM = -2 };

typedef struct { double s, comp; } nsum;
static inline void nadd(nsum *a, double v) {
    double t = a->s + v;
    if (fabs(a->s) >= fabs(v)) a->comp += (a->s - t) + v;
    else a->comp += (v - t) + a->s;
    a->s = t;
}
static inline double nval(const nsum *a) { return a->s + a->comp; }

static int check_graph(int64_t n, const int64_t *rp, const int32_t *col) {
    if (n < 1 || !rp) return 0;
    if (rp[0] != 0) return 0;
    for (int64_t i = 0; i < n; ++i)
        if (rp[i + 1] < rp[i]) return 0;
    int64_t m = rp[n];
    if (m > 0 && !col) return 0;
    for (int64_t e = 0; e < m; ++e)
        if (col[e] < 0 || col[e] >= n) return 0;
    return 1;
}

/* normalised personalization vector (e/n when p == NULL) */
static int make_p(int64_t n, const double *p, double *out) {
    if (!p) {
        for (int64_t i = 0; i < n; ++i) out[i] = 1.0 / (double)n;
        return 1;
    }
    nsum s = {0, 0};
    for (int64_t i = 0; i < n; ++i) {
        if (!(p[i] >= 0.0) || !isfinite(p[i])) return 0;
        nadd(&s, p[i]);
    }
    double tot = nval(&s);
    if (!(tot > 0.0)) return 0;
    for (int64_t i = 0; i < n; ++i) out[i] = p[i] / tot;
    return 1;
}

/*
 * Power method on P'' (Eq. 1); the serial power method the paper compares
 * against and takes its ground truth from (experiment section).
 *   x0 = p;  repeat  x' = c P x + (c d^T x + (1-c) e^T x) p,  x' /= sum(x'),
 *   delta = ||x' - x||_1,  until delta <= tol or max_iter iterations.
 * P'' is column-stochastic and contracts by c in the L1 norm, so the returned
 * x satisfies ||x - pi||_1 <= c/(1-c) * delta.
 */
int oracle_power(int64_t n, const int64_t *rp, const int32_t *col, double c, const double *p,
                 double tol, int64_t max_iter, double *x_out, int64_t *iters_out, double *delta_out) {
    if (!check_graph(n, rp, col) || !(c > 0.0 && c < 1.0) || !(tol >= 0.0) || max_iter < 1 || !x_out)
        return OR_EINVAL;
    double *pv = malloc(sizeof(double) * n), *x = malloc(sizeof(double) * n), *y = malloc(sizeof(double) * n);
    if (!pv || !x || !y) { free(pv); free(x); free(y); return OR_ENOMEM; }
    if (!make_p(n, p, pv)) { free(pv); free(x); free(y); return OR_EINVAL; }
    memcpy(x, pv, sizeof(double) * n);
    double delta = INFINITY;
    int64_t it = 0;
    while (it < max_iter) {
        nsum dsum = {0, 0}, xsum = {0, 0};
        for (int64_t i = 0; i < n; ++i) {
            nadd(&xsum, x[i]);
            if (rp[i + 1] == rp[i]) nadd(&dsum, x[i]);
        }
        for (int64_t i = 0; i < n; ++i) y[i] = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            int64_t deg = rp[i + 1] - rp[i];
            if (deg == 0) continue;
            double share = c * x[i] / (double)deg;
            for (int64_t e = rp[i]; e < rp[i + 1]; ++e) y[col[e]] += share;
        }
        double jump = c * nval(&dsum) + (1.0 - c) * nval(&xsum);
        nsum ysum = {0, 0};
        for (int64_t i = 0; i < n; ++i) {
            y[i] += jump * pv[i];
            nadd(&ysum, y[i]);
        }
        double ys = nval(&ysum);
        nsum d = {0, 0};
        for (int64_t i = 0; i < n; ++i) {
            y[i] /= ys;
            nadd(&d, fabs(y[i] - x[i]));
        }
        delta = nval(&d);
        double *t = x; x = y; y = t;
        ++it;
        if (delta <= tol) break;
    }
    memcpy(x_out, x, sizeof(double) * n);
    if (iters_out) *iters_out = it;
    if (delta_out) *delta_out = delta;
    free(pv); free(x); free(y);
    return delta <= tol ? OR_OK : OR_NOCONV;
}

/*
 * Serial IFP1 (Algorithm 2 run by a single calculation thread, section 3.2).
 * Reserve 100 % of the mass, push only from non-dangling vertices, stop when
 * no non-dangling vertex holds more than xi, normalise (pibar + h) once
 * (Eq. 4).  Units: h starts at n * p, i.e. h_i = 1 for the uniform p, as in
 * the algorithm's initialisation.  A vertex is processed when h_i > xi; its
 * mass v is taken and h_i cleared before the pushes, so a self-loop keeps its
 * share.  One pass visits the vertices in id order; the loop ends after a
 * pass that processed nothing, or after max_passes passes (return 1).
 * Outputs (each may be NULL): pibar[n], h[n] (final state), pi[n].
 * counts[3] = {passes, vertex pushes, edge pushes}.
 */
int oracle_ifp1(int64_t n, const int64_t *rp, const int32_t *col, double c, const double *p,
                double xi, int64_t max_passes, double *pibar_out, double *h_out, double *pi_out,
                int64_t *counts) {
    if (!check_graph(n, rp, col) || !(c > 0.0 && c < 1.0) || !(xi > 0.0) || max_passes < 1)
        return OR_EINVAL;
    double *pv = malloc(sizeof(double) * n), *pb = calloc(n, sizeof(double)), *h = malloc(sizeof(double) * n);
    if (!pv || !pb || !h) { free(pv); free(pb); free(h); return OR_ENOMEM; }
    if (!make_p(n, p, pv)) { free(pv); free(pb); free(h); return OR_EINVAL; }
    for (int64_t i = 0; i < n; ++i) h[i] = p ? (double)n * pv[i] : 1.0;
    int64_t passes = 0, vpush = 0, epush = 0;
    int active = 1;
    while (active && passes < max_passes) {
        active = 0;
        for (int64_t i = 0; i < n; ++i) {
            int64_t deg = rp[i + 1] - rp[i];
            if (deg == 0 || !(h[i] > xi)) continue;
            double v = h[i];
            h[i] = 0.0;
            pb[i] += v;
            double share = c * v / (double)deg;
            for (int64_t e = rp[i]; e < rp[i + 1]; ++e) h[col[e]] += share;
            ++vpush;
            epush += deg;
            active = 1;
        }
        ++passes;
    }
    int rc = active ? OR_NOCONV : OR_OK;
    if (rc == OR_NOCONV) {
        /* converged means: a full pass found no vertex above xi */
        rc = OR_OK;
        for (int64_t i = 0; i < n; ++i)
            if (rp[i + 1] > rp[i] && h[i] > xi) { rc = OR_NOCONV; break; }
    }
    if (pi_out) {
        nsum s = {0, 0};
        for (int64_t i = 0; i < n; ++i) nadd(&s, pb[i] + h[i]);
        double tot = nval(&s);
        for (int64_t i = 0; i < n; ++i) pi_out[i] = (pb[i] + h[i]) / tot;
    }
    if (pibar_out) memcpy(pibar_out, pb, sizeof(double) * n);
    if (h_out) memcpy(h_out, h, sizeof(double) * n);
    if (counts) { counts[0] = passes; counts[1] = vpush; counts[2] = epush; }
    free(pv); free(pb); free(h);
    return rc;
}

/*
 * Serial IFP2 (Algorithm 3 run by a single calculation thread, section 3.4).
 * Preprocessing invalidates every edge whose target is dangling.  Phase 1 is
 * IFP1 restricted to the remaining edges, still dividing by the ORIGINAL
 * out-degree (the mass a dangling vertex receives is c/deg(u) of its source's
 * reserve, as the motivation of IFP2 states).  Phase 2 runs once: every
 * dangling vertex d gets
 *     x_d = h_d + sum over edges u -> d of c * z_u / deg(u),
 * then the result is normalised.  Default (literal == 0): z = pibar + h and
 * x = z on non-dangling vertices, i.e. the leftover residual is kept as in
 * IFP1's normalisation.  literal != 0: z = pibar and x = pibar on
 * non-dangling vertices, exactly as the algorithm's phase 2 and final
 * normalisation are written.
 * Outputs: pibar[n], h[n] = phase-1 state (dangling entries keep their
 * initial mass), x[n] = unnormalised phase-2 result, pi[n].  counts[4] =
 * {passes, vertex pushes, edge pushes (phase 1), edge reads (phase 2)}.
 */
int oracle_ifp2(int64_t n, const int64_t *rp, const int32_t *col, double c, const double *p,
                double xi, int64_t max_passes, int literal, double *pibar_out, double *h_out,
                double *x_out, double *pi_out, int64_t *counts) {
    if (!check_graph(n, rp, col) || !(c > 0.0 && c < 1.0) || !(xi > 0.0) || max_passes < 1)
        return OR_EINVAL;
    double *pv = malloc(sizeof(double) * n), *pb = calloc(n, sizeof(double)), *h = malloc(sizeof(double) * n),
           *x = malloc(sizeof(double) * n);
    if (!pv || !pb || !h || !x) { free(pv); free(pb); free(h); free(x); return OR_ENOMEM; }
    if (!make_p(n, p, pv)) { free(pv); free(pb); free(h); free(x); return OR_EINVAL; }
    for (int64_t i = 0; i < n; ++i) h[i] = p ? (double)n * pv[i] : 1.0;
    /* phase 1 */
    int64_t passes = 0, vpush = 0, epush = 0, ereads = 0;
    int active = 1;
    while (active && passes < max_passes) {
        active = 0;
        for (int64_t i = 0; i < n; ++i) {
            int64_t deg = rp[i + 1] - rp[i];
            if (deg == 0 || !(h[i] > xi)) continue;
            double v = h[i];
            h[i] = 0.0;
            pb[i] += v;
            double share = c * v / (double)deg;
            for (int64_t e = rp[i]; e < rp[i + 1]; ++e) {
                int32_t j = col[e];
                if (rp[j + 1] == rp[j]) continue; /* invalidated edge: target is dangling */
                h[j] += share;
                ++epush;
            }
            ++vpush;
            active = 1;
        }
        ++passes;
    }
    int rc = OR_OK;
    for (int64_t i = 0; i < n; ++i)
        if (rp[i + 1] > rp[i] && h[i] > xi) { rc = OR_NOCONV; break; }
    /* phase 2 */
    for (int64_t i = 0; i < n; ++i) {
        if (rp[i + 1] > rp[i]) x[i] = literal ? pb[i] : pb[i] + h[i];
        else x[i] = h[i];
    }
    for (int64_t u = 0; u < n; ++u) {
        int64_t deg = rp[u + 1] - rp[u];
        if (deg == 0) continue;
        double z = literal ? pb[u] : pb[u] + h[u];
        double share = c * z / (double)deg;
        for (int64_t e = rp[u]; e < rp[u + 1]; ++e) {
            int32_t d = col[e];
            if (rp[d + 1] != rp[d]) continue;
            x[d] += share;
            ++ereads;
        }
    }
    if (pi_out) {
        nsum s = {0, 0};
        for (int64_t i = 0; i < n; ++i) nadd(&s, x[i]);
        double tot = nval(&s);
        for (int64_t i = 0; i < n; ++i) pi_out[i] = x[i] / tot;
    }
    if (pibar_out) memcpy(pibar_out, pb, sizeof(double) * n);
    if (h_out) memcpy(h_out, h, sizeof(double) * n);
    if (x_out) memcpy(x_out, x, sizeof(double) * n);
    if (counts) { counts[0] = passes; counts[1] = vpush; counts[2] = epush; counts[3] = ereads; }
    free(pv); free(pb); free(h); free(x);
    return rc;
}

/* Gaussian elimination with partial pivoting on a dense row-major a[n*n] x = b (in place). */
static int gauss_solve(int64_t n, double *a, double *b) {
    for (int64_t k = 0; k < n; ++k) {
        int64_t piv = k;
        for (int64_t r = k + 1; r < n; ++r)
            if (fabs(a[r * n + k]) > fabs(a[piv * n + k])) piv = r;
        if (a[piv * n + k] == 0.0) return 0;
        if (piv != k) {
            for (int64_t j = 0; j < n; ++j) { double t = a[k * n + j]; a[k * n + j] = a[piv * n + j]; a[piv * n + j] = t; }
            double t = b[k]; b[k] = b[piv]; b[piv] = t;
        }
        for (int64_t r = k + 1; r < n; ++r) {
            double f = a[r * n + k] / a[k * n + k];
            if (f == 0.0) continue;
            for (int64_t j = k; j < n; ++j) a[r * n + j] -= f * a[k * n + j];
            b[r] -= f * b[k];
        }
    }
    for (int64_t k = n - 1; k >= 0; --k) {
        double s = b[k];
        for (int64_t j = k + 1; j < n; ++j) s -= a[k * n + j] * b[j];
        b[k] = s / a[k * n + k];
    }
    return 1;
}

/*
 * Dense direct solve for small graphs (n <= 256).
 * form == 0: (I - c P') pi = (1-c) p with P' = P + p d^T      (Eq. 2)
 * form == 1: (I - c P) y = p, pi = y / sum(y)                 (Eq. 4)
 */
int oracle_dense(int64_t n, const int64_t *rp, const int32_t *col, double c, const double *p, int form,
                 double *pi_out) {
    if (!check_graph(n, rp, col) || n > 256 || !(c > 0.0 && c < 1.0) || !pi_out || (form != 0 && form != 1))
        return OR_EINVAL;
    double *pv = malloc(sizeof(double) * n), *a = calloc((size_t)(n * n), sizeof(double)), *b = malloc(sizeof(double) * n);
    if (!pv || !a || !b) { free(pv); free(a); free(b); return OR_ENOMEM; }
    if (!make_p(n, p, pv)) { free(pv); free(a); free(b); return OR_EINVAL; }
    /* a = -c P (column j is the source), then the dangling correction, then + I */
    for (int64_t j = 0; j < n; ++j) {
        int64_t deg = rp[j + 1] - rp[j];
        if (deg == 0) {
            if (form == 0)
                for (int64_t i = 0; i < n; ++i) a[i * n + j] -= c * pv[i];
            continue;
        }
        for (int64_t e = rp[j]; e < rp[j + 1]; ++e) a[(int64_t)col[e] * n + j] -= c / (double)deg;
    }
    for (int64_t i = 0; i < n; ++i) {
        a[i * n + i] += 1.0;
        b[i] = form == 0 ? (1.0 - c) * pv[i] : pv[i];
    }
    int ok = gauss_solve(n, a, b);
    if (ok) {
        nsum s = {0, 0};
        for (int64_t i = 0; i < n; ++i) nadd(&s, b[i]);
        double tot = nval(&s);
        for (int64_t i = 0; i < n; ++i) pi_out[i] = form == 0 ? b[i] : b[i] / tot;
    }
    free(pv); free(a); free(b);
    return ok ? OR_OK : OR_EINVAL;
}
