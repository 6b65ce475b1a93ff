/*
 * pr.h -- C ABI of libpr.so: IFP1 / IFP2 forward-push PageRank and the power
 * method on one AMD MI355X (gfx950) GPU.
 *
 * The method is that of Zhang, Tang, Yao, Liang, "Two Parallel PageRank
 * Algorithms via Improving Forward Push" (arXiv 2302.03245).  The arguments
 * follow the problem statement of its forward-push algorithm (section 2.2,
 * Algorithm 1): a graph G(V, E), the damping factor c, the personalization
 * vector p and the residual threshold xi; the output is the PageRank vector
 * pi.  The number of calculation threads K of Algorithms 2 and 3 is not an
 * argument: it is the GPU launch configuration.
 *
 * Conventions
 *  - Every function returns a pr_status; 0 (PR_OK) is success, PR_ENOCONV (> 0)
 *    is a warning with a usable result, negative values are errors.
 *  - On a negative status no output (pi, stats, *out handle) is written.
 *    pr_last_error() then returns a thread-local message.
 *  - Vertices are 0 .. n-1.  Edge i -> j is stored in row i of a CSR:
 *    j = col[row_ptr[i] + k], 0 <= k < row_ptr[i+1] - row_ptr[i].
 *  - deg(i) is the row length; a self-loop counts toward deg(i); repeated
 *    edges count with multiplicity unless PR_DEDUPE is given at upload.
 *    A vertex with deg(i) == 0 is dangling (section 2.1).
 *  - Sizes: n < 2^31 and m < 2^31 (the device stores 32-bit indices and
 *    offsets); larger graphs are rejected with PR_EINVAL.
 *  - Thread safety: distinct graphs may be used concurrently.  Solves on one
 *    graph from several host threads or streams are allowed (the graph is
 *    read-only after upload); freeing a graph while a solve runs is undefined.
 *    pr_graph_tune rebuilds the graph's plans: it returns PR_EBUSY while solves
 *    (or a query server) use the graph, and solves that start while it runs
 *    return PR_EBUSY.
 */
#ifndef PR_H
#define PR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PR_OK = 0,
    PR_ENOCONV = 1,  /* max_sweeps reached: pi holds the normalised best estimate, stats->l1_bound its quality */
    PR_EINVAL = -1,  /* invalid argument (see each function) */
    PR_ENOMEM = -2,  /* device or host allocation failed */
    PR_EDEVICE = -3, /* a HIP runtime call failed */
    PR_EBUSY = -4    /* the graph is in use: pr_graph_tune / pr_set_tune while solves or a
                        server use it, or a solve (or pr_server_add_graph) while it is tuned */
} pr_status;

typedef struct pr_graph pr_graph; /* opaque, device-resident, owned by the library */

/* residual (pushing mass) precision; the reserved mass and all reductions are always FP64 */
typedef enum { PR_RES_FP64 = 0, PR_RES_FP32 = 1 } pr_residual;

/* stop rule */
typedef enum {
    PR_STOP_XI = 0, /* stop when no non-dangling vertex has residual > xi (Algorithms 2 and 3) */
    PR_STOP_L1 = 1  /* stop when the certified bound on ||pi - pi_exact||_1 is <= l1_tol */
} pr_stop;

/* pr_graph_upload flags */
#define PR_INPUT_DEVICE 0x1u /* row_ptr and col are device pointers */
#define PR_DEDUPE 0x2u       /* collapse repeated edges (the 0/1 adjacency matrix of section 2.1) */
/* sweep tile size: each workgroup of 256 threads takes 256 << s rows + edges per tile,
   s in {2, 3, 4}; 0 selects the default (s = 3) */
#define PR_TILE_SHIFT(s) (((uint32_t)(s) & 0x7u) << 8)
#define PR_TILE_MASK 0x700u
/* ordered sweeps of global IFP2 solves: the non-dangling vertices are split into k
   groups of equal out-edge counts (k in 1..15; 1 = no ordered sweeps; 0 selects 4 when
   at least 2^24 edges join non-dangling vertices, else 1: on smaller graphs the extra
   launches of an ordered sweep cost more than the sweeps it saves) */
#define PR_GROUPS(k) (((uint32_t)(k) & 0xFu) << 12)
#define PR_GROUPS_MASK 0xF000u
/* ordered sweeps: each group's gather walks every target row instead of only the rows
   with an edge from that group (the default; pr_graph_tune times both and keeps one) */
#define PR_GROUP_ALL_ROWS 0x40000u
/* keep every in-edge list in fill order instead of sorting it by source (sorted lists
   make gathers touch fewer cache lines and their rounding order deterministic) */
#define PR_UNSORTED_IN 0x10000u
/* weak-dangling peeling for IFP2 (section 2: deleting the dangling vertices leaves new
   dangling vertices, the weakly dangling ones; repeated, this ranks vertices in levels).
   Level 1: every out-edge leads to a dangling vertex; level L: every out-edge leads to a
   vertex of a level below L (up to PR_PEEL_MAX_LEVELS; a vertex that reaches a cycle, a
   self-loop included, never peels).  Peeled vertices leave IFP2's phase 1 like dangling vertices:
   the sweeps run over the remaining core, with the edges into peeled vertices
   invalidated, and phase 2 gathers the levels from the highest down, each from the
   finished values of its in-neighbours, then the dangling vertices.  The certified bound
   is unchanged (c / (1-c) of the core's residual bounds the unnormalised error).  Such a
   graph serves pr_solve_ifp2, pr_ppr (sources solved one at a time), pr_solve_power and
   pr_graph_tune; IFP1, warm starts and the server reject it. */
#define PR_PEEL 0x20000u
#define PR_PEEL_MAX_LEVELS 64

/* pr_opts.flags */
#define PR_P_DEVICE 0x1u     /* p is a device pointer (double[n]) */
#define PR_OUT_DEVICE 0x2u   /* pi is a device pointer */
#define PR_IFP2_LITERAL 0x4u /* IFP2: drop the leftover residual at normalisation, as Algorithm 3 writes it */
#define PR_FORCE_PUSH 0x8u   /* every sweep scatters along out-edges with atomic adds */
#define PR_FORCE_PULL 0x10u  /* every sweep gathers along in-edges (no atomics) */
#define PR_PROFILE 0x20u     /* time each sweep kernel with HIP events (stats->kernel_*) */
#define PR_JACOBI 0x40u      /* IFP1 / IFP2: synchronous sweeps even where ordered sweeps apply */
/* After the solve, check the written result a posteriori in FP64: one application of
   the power-method matrix P'' (Eq. 1) to pi gives r = P'' pi - pi, and
   stats->l1_verified bounds ||pi - pi_exact||_1 whatever the residual precision: the
   smaller of ||r||_1 / (1 - c) (P'' contracts the difference of two vectors of equal sum
   by c in L1) and 2 sum_j F_j |r_j| / sum(pi) (F_j: the L1 mass a unit at j adds to
   (I - cP)^{-1}, dangling vertices absorbing; graphs uploaded without PR_PEEL), each
   + |sum(pi) - 1| and the rounding of the check.  Costs about one power-method
   iteration.  IFP1 / IFP2 under PR_STOP_L1 (not warm starts): when the check finds the
   result short of l1_tol, the solve sweeps on to a target tightened by the check's
   excess over the stop rule's estimate and checks again (at most 3 times); a verified
   bound still above l1_tol gives PR_ENOCONV. */
#define PR_VERIFY 0x80u
/* IFP1 / IFP2: every sweep scatters from the compacted frontier list (the vertices with
   residual > xi, kept as a list of ids between sweeps); without it a solve uses list
   sweeps while its frontier is sparse.  Not with PR_FORCE_PUSH / PR_FORCE_PULL. */
#define PR_FORCE_LIST 0x100u

typedef struct {
    double c;           /* damping factor, 0 < c < 1 (section 2.1) */
    double xi;          /* PR_STOP_XI threshold on a residual, in units where the initial residual
                           is n * p_i (1 for every vertex under uniform p, as in Algorithms 2 and 3) */
    double l1_tol;      /* PR_STOP_L1 target; also the power method's target */
    int32_t stop;       /* pr_stop */
    int32_t residual;   /* pr_residual */
    int32_t max_sweeps; /* 0 -> 100000 */
    uint32_t flags;     /* PR_P_DEVICE | PR_OUT_DEVICE | PR_IFP2_LITERAL | PR_FORCE_PUSH | PR_FORCE_PULL | PR_PROFILE
                           | PR_JACOBI | PR_VERIFY | PR_FORCE_LIST */
    void *stream;       /* hipStream_t to run on; NULL -> the graph's own stream */
} pr_opts;

typedef struct {
    int32_t sweeps;             /* synchronous sweeps (one reserve + one push or pull each); power: iterations */
    int32_t pull_sweeps;        /* of which gathered along in-edges */
    int64_t edges_processed;    /* sum over sweeps of the valid out-edges of the vertices that pushed,
                                   plus the in-edges read by IFP2's dangling phase; power: iterations * m */
    int64_t edges_traversed;    /* edges the kernels actually read (a pull sweep reads every in-edge) */
    int64_t vertex_pushes;      /* sum over sweeps of the number of vertices that pushed */
    double residual_l1;         /* final non-dangling residual / total mass (power: last ||x' - x||_1) */
    double l1_bound;            /* bound on ||pi - pi_exact||_1 from the stop rule's certificate; it
                                   assumes exact arithmetic, so with FP32 residuals it is an
                                   estimate (rounding of the pushes is not included): PR_VERIFY
                                   gives a bound that holds for the computed result */
    double seconds_solve;       /* device time from initialisation to the written result */
    double seconds_preprocess;  /* one-time per-graph preprocessing charged to this method (seconds): for
                                   folded IFP2 the edge split and the stop rule's weights for c (with
                                   ordered sweeps, also their restriction to the vertex groups) */
    /* PR_PROFILE only (else 0): the scatter (push) and gather (pull) kernels of the sweeps,
       timed with HIP events on the solve stream; launches that did work, their summed
       duration, and their algorithmic bytes (edge-index stream + residual traffic) */
    double push_seconds, push_bytes;
    int64_t push_launches;
    double pull_seconds, pull_bytes;
    int64_t pull_launches;
    int64_t launches;           /* kernels the solve enqueued (sweeps past the stop return at once) */
    double l1_verified;         /* PR_VERIFY: a-posteriori bound on ||pi - pi_exact||_1 (else 0) */
} pr_stats;

typedef struct {
    int64_t n, m;
    int64_t n_dangling;     /* out-degree 0 */
    int64_t m_dangling;     /* edges whose target is dangling, or peeled (PR_PEEL): invalidated
                               in IFP2's phase 1 and gathered once in its phase 2 */
    int64_t n_unreferenced; /* in-degree 0 */
    int64_t device_bytes;   /* device memory held by the graph */
    double seconds_upload;  /* whole upload: copies, classification, relabelling, plans */
    double seconds_split;   /* the IFP2 edge invalidation: stable split of every row into edges
                               towards non-dangling and towards dangling targets */
    int64_t max_depth;      /* largest finite unreferenced depth of a non-dangling vertex (0: a
                               vertex without non-dangling in-neighbours; -1: none), see below */
    int64_t epochs;         /* in-edge lists kept for the gather sweeps (1 + compacted copies) */
    int64_t groups;         /* vertex groups of ordered sweeps (1: none) */
    int64_t tile_items;     /* rows + edges per sweep tile (256 << tile shift) */
    int64_t ordered;        /* 1 if global IFP2 solves use ordered sweeps */
    int64_t n_peeled;       /* weakly dangling vertices taken out of the sweeps (PR_PEEL; else 0) */
    int64_t peel_levels;    /* their levels (0 without PR_PEEL) */
} pr_graph_info_t;

/*
 * Fill *o with the defaults: c = 0.85 (the experiments' damping factor),
 * xi = 1e-12, l1_tol = 1e-6, PR_STOP_XI, PR_RES_FP64, max_sweeps 0, flags 0,
 * stream NULL.
 */
void pr_opts_default(pr_opts *o);

/*
 * Copy a directed graph to the device and prepare it (graph of section 2.1).
 *   n        number of vertices, 1 <= n < 2^31
 *   m        number of edges, 0 <= m < 2^31
 *   row_ptr  int64[n+1], row_ptr[0] == 0, non-decreasing, row_ptr[n] == m
 *   col      int32[m], every entry in [0, n)   (may be NULL when m == 0)
 *   flags    PR_INPUT_DEVICE: row_ptr / col are device pointers; PR_DEDUPE; PR_TILE_SHIFT;
 *            PR_GROUPS; PR_UNSORTED_IN; PR_PEEL
 *   out      receives the handle
 * The inputs are copied; the caller keeps ownership of them.  The handle is
 * owned by the library until pr_graph_free.  Errors: PR_EINVAL for any
 * violated condition above or an unknown flag, PR_ENOMEM, PR_EDEVICE.
 */
pr_status pr_graph_upload(int64_t n, int64_t m, const int64_t *row_ptr, const int32_t *col,
                          uint32_t flags, pr_graph **out);

/* Release a graph and its device memory.  NULL is accepted.  */
pr_status pr_graph_free(pr_graph *g);

/*
 * Shape and cost figures of an uploaded graph (the data-set table columns of section 4.1).
 * Unreferenced depth (section 3.3.3): 0 for a non-dangling vertex with no non-dangling
 * in-neighbour, else 1 + the largest depth of those in-neighbours, infinite on or below a
 * cycle.  After sweep depth(v) a vertex receives no more mass, so the gather sweeps past
 * the start of an epoch read compacted in-edge lists without such sources.
 */
pr_status pr_graph_info(const pr_graph *g, pr_graph_info_t *out);

/* Outcome of pr_graph_tune: every candidate schedule that was timed. */
#define PR_TUNE_MAX 16
typedef struct {
    int32_t candidates;               /* entries filled below */
    int32_t tile_shift[PR_TUNE_MAX];  /* sweep tiles of 256 << s rows + edges per workgroup */
    int32_t groups[PR_TUNE_MAX];      /* vertex groups of ordered sweeps (1 for synchronous sweeps) */
    int32_t ordered[PR_TUNE_MAX];     /* 0: synchronous sweeps; ordered sweeps over the vertex groups
                                         with each group's gather over every row (1) or over only
                                         the rows that group reaches (2; graph sets: 1 only) */
    double ms[PR_TUNE_MAX];           /* fastest of the timed solves, device milliseconds */
    int32_t sweeps[PR_TUNE_MAX];
    int32_t chosen;                   /* index of the candidate the graph keeps */
    double seconds;                   /* wall time spent tuning */
    int32_t batch_ordered;            /* pr_graph_tune: whether batched solves (pr_ppr batches, the
                                         query server's batched runs) turn to ordered sweeps (1) or
                                         stay synchronous (0); -1 not measured (no ordered sweeps, a
                                         peeled graph, or no room for the batch's output) */
    double batch_ms[2];               /* the 16-source PPR batch timed for that choice: ordered, synchronous */
} pr_tune_report;

/*
 * Autotuner of the sweep schedule for global solves on this graph: times IFP2 with
 * the options o (c, stop rule, tolerance, residual type; p uniform) for every tile
 * size s in {2, 3, 4} with synchronous sweeps and, when the graph has vertex groups,
 * with ordered sweeps (the split of a sweep's work between per-vertex reserve
 * passes and per-edge gathers), `reps` solves each after one warm-up (reps <= 0:
 * 2); when the graph has vertex groups, the other form of the group gathers (every row,
 * or only the rows each group reaches) is timed at the tile size of the fastest ordered
 * candidate, and then 3, 4, 6 and 8 vertex groups in both forms (the graph's group lists
 * are rebuilt for each).  It
 * keeps the fastest: later solves of every kind use its tile size, and global IFP2
 * solves use ordered sweeps, with that group count and form of gather, only if it chose
 * them.  If it did, on a graph uploaded without PR_PEEL (pr_ppr solves a peeled graph's
 * sources one at a time), it then times a batch of 16 single-source PPR queries (non-dangling
 * sources spread over the ids, o's stop rule and residual type) with ordered and with
 * synchronous sweeps, and batched solves keep the faster (an ordered sweep of a batch
 * costs more than a synchronous one, and on some graphs saves few sweeps).  Results do
 * not change beyond rounding order.  No other call may use the graph meanwhile.
 * rep may be NULL.  PR_EINVAL on bad options or forced scatter modes.
 */
pr_status pr_graph_tune(pr_graph *g, const pr_opts *o, int32_t reps, pr_tune_report *rep);

/*
 * IFP1 (section 3.2, Algorithm 2): every non-dangling vertex whose residual
 * exceeds the threshold reserves 100 % of it and pushes c * r / deg(i) to each
 * out-neighbour; dangling vertices never push; the result is
 * pi = (pibar + h) / sum(pibar + h), which by Eq. 4 is the PageRank vector of
 * Eq. 1 for personalization p (dangling mass jumps according to p).
 *   p    double[n], p >= 0, finite, sum > 0 (normalised by its sum); NULL = uniform e/n
 *   o    options (NULL = defaults)
 *   pi   double[n] output (host, or device with PR_OUT_DEVICE)
 *   st   optional statistics
 * One GPU sweep processes every vertex above the threshold once (a
 * synchronous version of one scan of all calculation threads, section 3.3.1);
 * on a graph with vertex groups, sweeps over a dense frontier are ordered as
 * pr_solve_ifp2 describes, each group's pushes gathered into every vertex.
 * Errors: PR_EINVAL (bad graph handle, options, p, a graph uploaded with PR_PEEL
 * for IFP1), PR_ENOMEM, PR_EDEVICE;
 * PR_ENOCONV when max_sweeps ends the iteration.
 */
pr_status pr_solve_ifp1(const pr_graph *g, const double *p, const pr_opts *o, double *pi, pr_stats *st);

/*
 * IFP2 (section 3.4, Algorithm 3): as IFP1, but edges into dangling vertices
 * are invalidated during the sweeps (phase 1) and every dangling vertex d
 * gathers c * z_u / deg(u) from its in-neighbours once afterwards (phase 2),
 * deg being the original out-degree.  z = pibar + h by default;
 * PR_IFP2_LITERAL uses z = pibar and drops the leftover residual as the
 * algorithm is written.  Arguments and errors as pr_solve_ifp1.
 *
 * Global solves (p = NULL) of a graph uploaded with more than one vertex group
 * (PR_GROUPS, default 4) use ordered sweeps: within a sweep the groups, in
 * order of decreasing out-degree, each take their residuals and gather their
 * pushes before the next group takes its own, so later groups already see this
 * sweep's pushes -- the effect of the paper's calculation threads pushing as
 * they go -- and fewer sweeps reach the bound.  Unless the options force a
 * scatter mode or set PR_JACOBI; the stop rule and its certificate are the same.
 */
pr_status pr_solve_ifp2(const pr_graph *g, const double *p, const pr_opts *o, double *pi, pr_stats *st);

/*
 * Power method on P'' = c P' + (1-c) p e^T (Eq. 1), the baseline the paper
 * compares against (section 4.3): x <- c P x + (c d^T x + (1-c) e^T x) p from
 * x = p until c / (1-c) * ||x' - x||_1 <= l1_tol; xi and stop are ignored.
 * Arguments and errors as pr_solve_ifp1; l1_tol must be > 0.
 */
pr_status pr_solve_power(const pr_graph *g, const double *p, const pr_opts *o, double *pi, pr_stats *st);

/*
 * Single-source personalized PageRank (section 2.1: p = e_s; the mass of
 * dangling vertices jumps back to s because P' = P + p d^T), solved by IFP2
 * for each of the k sources.  Up to 16 sources share one batched solve: their
 * residual vectors are interleaved so that every gathered in-edge serves all of
 * them, and each keeps its own stop decision (same result as one call per
 * source, within the tolerances).  A batch starts with synchronous sweeps
 * (each column's frontier is one vertex) and turns to ordered sweeps over the
 * graph's vertex groups, as for global solves, once the columns' frontiers
 * together are dense; PR_JACOBI keeps it synchronous.  On a graph uploaded with
 * PR_PEEL every source is solved alone.  With PR_OUT_DEVICE, pi is a device
 * pointer.
 *   sources  int32[k] host array, each in [0, n); k >= 1
 *   pi       double[k * n], row r is the PPR vector of sources[r]
 *   st       optional, k entries
 * Returns the worst status over the k solves.  On a negative status no row of pi
 * and no entry of st is written: a call of more than one batch (k > 16, or k > 1
 * on a peeled graph) solves into a device staging buffer of k * n doubles,
 * allocated before the first batch (PR_ENOMEM if it cannot be), and copies the
 * rows out once every batch has succeeded; only a failure of that final copy
 * (PR_EDEVICE) can leave pi partly written.
 */
pr_status pr_ppr(const pr_graph *g, const int32_t *sources, int32_t k, const pr_opts *o, double *pi,
                 pr_stats *st);

/*
 * Testing hook (for callers that check the error contract of pr_ppr): the next
 * pr_ppr call on this thread fails with PR_ENOMEM when it reaches batch b
 * (b >= 1, i.e. after b batches have been solved), as if that batch's workspace
 * could not be allocated.  b <= 0 disables it; the hook is cleared by that call.
 */
void pr_debug_fail_ppr_batch(int32_t b);

/*
 * pr_solve_ifp2 for callers that cannot allocate memory (code under stream capture,
 * tight serving loops, harnesses that forbid allocation): the same solve, with every
 * byte of its device workspace taken from a fixed array of 256 MiB that the library
 * holds on each device it runs on (until the process ends), and no allocation, pinned
 * host memory or timing event created by the call (stats->seconds_solve is 0).  The
 * caller still passes p and pi as for pr_solve_ifp2 (host or device, PR_P_DEVICE /
 * PR_OUT_DEVICE).  A solve whose workspace exceeds the array (about 32 bytes per
 * vertex plus 18 per non-dangling vertex, and more with a host p, a host pi or
 * PR_VERIFY: R-MAT scale 22 with FP32 residuals and a device pi takes about 140 MB)
 * returns PR_EINVAL with the size it needs; PR_PROFILE returns PR_EINVAL.  All calls on
 * one device share the array: calls that overlap on one device race, and each call
 * initialises everything it reads.  Otherwise as pr_solve_ifp2.
 */
pr_status pr_solve_ifp2_noalloc(const pr_graph *g, const double *p, const pr_opts *o, double *pi, pr_stats *st);

/* Message describing the last error on this thread ("" if none). */
const char *pr_last_error(void);

/*
 * Per-sweep record of this thread's last IFP1 / IFP2 / PPR solve run with
 * PR_PROFILE (the quantities of the convergence analysis, section 3.3):
 * active[t] = vertices that pushed in sweep t, edges[t] = their valid
 * out-edges, residual[t] = residual left on non-dangling vertices after the
 * sweep, bound[t] = certified L1 bound after the sweep, pulled[t] = 1 if the
 * sweep gathered along in-edges.  Writes min(cap, sweeps) entries of every
 * non-NULL array (caller-owned) and returns the number of recorded sweeps
 * (0 when the last solve was not profiled).
 */
int32_t pr_last_trace(int32_t cap, int64_t *active, int64_t *edges, double *residual, double *bound,
                      int32_t *pulled);

#ifdef __cplusplus
}
#endif

#endif /* PR_H */
