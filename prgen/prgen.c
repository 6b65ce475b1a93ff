/*
 * prgen.c -- seeded synthetic graph generators (input generation only).
 *
 * This module produces the directed graphs on which both the GPU solver and
 * the CPU oracle run.  It contains none of the PageRank arithmetic: it only
 * draws edges, removes self-loops and duplicates, applies the dangling /
 * unreferenced transforms of the workload recipes and emits a CSR
 * (row_ptr int64[n+1], col int32[m], rows sorted by target id).
 *
 * Randomness: every random number is a SplitMix64 output addressed by a
 * counter, i.e. the k-th output of the stream with state s is
 * mix64(s + (k+1) * 0x9E3779B97F4A7C15) (Steele, Lea, Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014).  One stream key per
 * (root seed, workload id, purpose), so the output is identical for any
 * OpenMP thread count.
 *
 * Purposes: 0 edges, 1 dangling set, 2 unreferenced set / redirect targets,
 * 3 final vertex relabel permutation, 4 DAG layer assignment, 5 Zipf degrees,
 * 6 DAG forward targets, 7 back edges.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define GAMMA 0x9E3779B97F4A7C15ULL

static inline uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}
static inline uint64_t rnd_at(uint64_t key, uint64_t ctr) { return mix64(key + (ctr + 1) * GAMMA); }
static uint64_t stream_key(uint64_t seed, uint32_t wl, uint32_t purpose) {
    return mix64(seed * GAMMA ^ mix64(((uint64_t)wl << 32) | (uint64_t)purpose));
}
static inline double unif01(uint64_t x) { return (double)(x >> 11) * 0x1.0p-53; }
/* uniform integer in [0, n): high half of the 128-bit product (bias < n / 2^64) */
static inline uint64_t bounded(uint64_t x, uint64_t n) {
    return (uint64_t)(((unsigned __int128)x * n) >> 64);
}

/* ------------------------------------------------------------------------ */
/* result handle                                                             */
/* ------------------------------------------------------------------------ */
typedef struct {
    int64_t n, m;
    int64_t *row_ptr; /* n + 1 */
    int32_t *col;     /* m */
    double aux;       /* recipe-specific scalar (DAG: the degree scale lambda) */
    int64_t draws;    /* edges drawn before self-loop / duplicate removal */
} prgen_graph;

void prgen_free(prgen_graph *g) {
    if (!g) return;
    free(g->row_ptr);
    free(g->col);
    free(g);
}

/* ------------------------------------------------------------------------ */
/* stable LSD radix sort of 64-bit keys (deterministic for any thread count) */
/* ------------------------------------------------------------------------ */
static void radix_sort_u64(uint64_t *a, uint64_t *tmp, int64_t n, int key_bits) {
    const int RB = 11, R = 1 << RB;
    int nthreads = 1;
#ifdef _OPENMP
    nthreads = omp_get_max_threads();
#endif
    int64_t *hist = (int64_t *)malloc(sizeof(int64_t) * (size_t)nthreads * R);
    uint64_t *src = a, *dst = tmp;
    int passes = (key_bits + RB - 1) / RB;
    for (int pass = 0; pass < passes; ++pass) {
        int shift = pass * RB;
        memset(hist, 0, sizeof(int64_t) * (size_t)nthreads * R);
#pragma omp parallel num_threads(nthreads)
        {
            int t = 0;
#ifdef _OPENMP
            t = omp_get_thread_num();
#endif
            int64_t lo = n * t / nthreads, hi = n * (t + 1) / nthreads;
            int64_t *h = hist + (size_t)t * R;
            for (int64_t i = lo; i < hi; ++i) h[(src[i] >> shift) & (R - 1)]++;
#pragma omp barrier
#pragma omp single
            {
                int64_t run = 0;
                for (int d = 0; d < R; ++d)
                    for (int tt = 0; tt < nthreads; ++tt) {
                        int64_t c = hist[(size_t)tt * R + d];
                        hist[(size_t)tt * R + d] = run;
                        run += c;
                    }
            }
            for (int64_t i = lo; i < hi; ++i) {
                uint64_t v = src[i];
                dst[h[(v >> shift) & (R - 1)]++] = v;
            }
        }
        uint64_t *s = src; src = dst; dst = s;
    }
    if (src != a) memcpy(a, src, sizeof(uint64_t) * (size_t)n);
    free(hist);
}

static int bits_for(int64_t n) {
    int b = 1;
    while (((int64_t)1 << b) < n) ++b;
    return b;
}

/* sort (src<<32|dst) keys, drop duplicates; returns new count */
static int64_t sort_unique(uint64_t *keys, int64_t cnt, int64_t n) {
    if (cnt == 0) return 0;
    uint64_t *tmp = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)cnt);
    radix_sort_u64(keys, tmp, cnt, 32 + bits_for(n));
    free(tmp);
    int64_t w = 1;
    for (int64_t i = 1; i < cnt; ++i)
        if (keys[i] != keys[w - 1]) keys[w++] = keys[i];
    return w;
}

/* Fisher-Yates permutation of [0, n) driven by a counter stream */
static int32_t *permutation(int64_t n, uint64_t key) {
    int32_t *p = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) p[i] = (int32_t)i;
    for (int64_t i = n - 1; i > 0; --i) {
        int64_t j = (int64_t)bounded(rnd_at(key, (uint64_t)i), (uint64_t)i + 1);
        int32_t t = p[i]; p[i] = p[j]; p[j] = t;
    }
    return p;
}

/* relabel every endpoint through perm, sort, and emit CSR */
static prgen_graph *to_csr(uint64_t *keys, int64_t cnt, int64_t n, const int32_t *perm) {
    if (perm) {
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < cnt; ++i) {
            uint64_t s = keys[i] >> 32, d = keys[i] & 0xffffffffULL;
            keys[i] = ((uint64_t)(uint32_t)perm[s] << 32) | (uint64_t)(uint32_t)perm[d];
        }
        cnt = sort_unique(keys, cnt, n);
    }
    prgen_graph *g = (prgen_graph *)calloc(1, sizeof(prgen_graph));
    g->n = n;
    g->m = cnt;
    g->row_ptr = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    g->col = (int32_t *)malloc(sizeof(int32_t) * (size_t)(cnt > 0 ? cnt : 1));
    for (int64_t i = 0; i < cnt; ++i) g->row_ptr[(keys[i] >> 32) + 1]++;
    for (int64_t i = 0; i < n; ++i) g->row_ptr[i + 1] += g->row_ptr[i];
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < cnt; ++i) g->col[i] = (int32_t)(keys[i] & 0xffffffffULL);
    return g;
}

/* one R-MAT draw at the given scale: quadrant probabilities a (src 0, dst 0),
 * b (src 0, dst 1), c (src 1, dst 0), d = 1 - a - b - c (Chakrabarti, Zhan,
 * Faloutsos, SDM 2004) */
static inline uint64_t rmat_draw(uint64_t key, uint64_t k, int scale, double a, double ab, double abc) {
    uint64_t s = 0, t = 0;
    for (int l = 0; l < scale; ++l) {
        double u = unif01(rnd_at(key, k * 64 + (uint64_t)l));
        uint64_t bs, bt;
        if (u < a) { bs = 0; bt = 0; }
        else if (u < ab) { bs = 0; bt = 1; }
        else if (u < abc) { bs = 1; bt = 0; }
        else { bs = 1; bt = 1; }
        s = (s << 1) | bs;
        t = (t << 1) | bt;
    }
    return (s << 32) | t;
}

/* ------------------------------------------------------------------------ */
/* Small R-MAT workload: draw at `scale`, reject endpoints >= n, self-loops  */
/* and repeats, until `target_m` distinct edges exist (draw order), then     */
/* drop all out-edges of `n_dangling` uniformly chosen vertices, relabel.    */
/* ------------------------------------------------------------------------ */
/* stable LSD radix sort of 64-bit keys carrying 32-bit payloads */
static void radix_sort_kv(uint64_t *k, uint32_t *v, int64_t n, int key_bits) {
    const int RB = 11, R = 1 << RB;
    int nthreads = 1;
#ifdef _OPENMP
    nthreads = omp_get_max_threads();
#endif
    int64_t *hist = (int64_t *)malloc(sizeof(int64_t) * (size_t)nthreads * R);
    uint64_t *tk = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(n > 0 ? n : 1));
    uint32_t *tv = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(n > 0 ? n : 1));
    uint64_t *sk = k, *dk = tk;
    uint32_t *sv = v, *dv = tv;
    int passes = (key_bits + RB - 1) / RB;
    for (int pass = 0; pass < passes; ++pass) {
        int shift = pass * RB;
        memset(hist, 0, sizeof(int64_t) * (size_t)nthreads * R);
#pragma omp parallel num_threads(nthreads)
        {
            int t = 0;
#ifdef _OPENMP
            t = omp_get_thread_num();
#endif
            int64_t lo = n * t / nthreads, hi = n * (t + 1) / nthreads;
            int64_t *h = hist + (size_t)t * R;
            for (int64_t i = lo; i < hi; ++i) h[(sk[i] >> shift) & (R - 1)]++;
#pragma omp barrier
#pragma omp single
            {
                int64_t run = 0;
                for (int d = 0; d < R; ++d)
                    for (int tt = 0; tt < nthreads; ++tt) {
                        int64_t c = hist[(size_t)tt * R + d];
                        hist[(size_t)tt * R + d] = run;
                        run += c;
                    }
            }
            for (int64_t i = lo; i < hi; ++i) {
                int64_t o = h[(sk[i] >> shift) & (R - 1)]++;
                dk[o] = sk[i];
                dv[o] = sv[i];
            }
        }
        uint64_t *s = sk; sk = dk; dk = s;
        uint32_t *s2 = sv; sv = dv; dv = s2;
    }
    if (sk != k) {
        memcpy(k, sk, sizeof(uint64_t) * (size_t)n);
        memcpy(v, sv, sizeof(uint32_t) * (size_t)n);
    }
    free(tk);
    free(tv);
    free(hist);
}

/* ------------------------------------------------------------------------ */
/* Small R-MAT workload: draw at `scale`, reject endpoints >= n, self-loops  */
/* and repeats, until `target_m` distinct edges exist (draw order), then     */
/* drop all out-edges of `n_dangling` uniformly chosen vertices, relabel.    */
/* The first target_m distinct valid draws are found in parallel: draws     */
/* 0..K-1 are sorted stably by edge, which leaves each edge's first draw at  */
/* the head of its run; a scan in draw order then takes the first target_m   */
/* such heads (K grows until enough exist).                                  */
/* ------------------------------------------------------------------------ */
prgen_graph *prgen_rmat_exact(int64_t n, int scale, int64_t target_m, int64_t n_dangling,
                              double a, double b, double c, uint64_t seed, uint32_t wl) {
    if (n < 1 || n > ((int64_t)1 << scale) || scale > 31 || target_m < 0 ||
        target_m > n * (n - 1) || n_dangling < 0 || n_dangling > n)
        return NULL;
    uint64_t ke = stream_key(seed, wl, 0), kd = stream_key(seed, wl, 1), kr = stream_key(seed, wl, 3);
    const double ab = a + b, abc = a + b + c;
    const uint64_t INVALID = (uint64_t)1 << (32 + scale); /* above every valid key */
    uint64_t *keys = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(target_m > 0 ? target_m : 1));
    int64_t have = 0, k_used = 0;
    int64_t K = target_m + target_m / 4 + 1024;
    while (have < target_m) {
        if (K > ((int64_t)1 << 32) - 1) { free(keys); return NULL; }
        uint64_t *e = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)K);
        uint32_t *idx = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)K);
#pragma omp parallel for schedule(static)
        for (int64_t k = 0; k < K; ++k) {
            uint64_t d = rmat_draw(ke, (uint64_t)k, scale, a, ab, abc);
            uint64_t s = d >> 32, t = d & 0xffffffffULL;
            e[k] = ((int64_t)s >= n || (int64_t)t >= n || s == t) ? INVALID : d;
            idx[k] = (uint32_t)k;
        }
        radix_sort_kv(e, idx, K, 33 + scale);
        /* head[k] = edge of draw k if draw k is its edge's first valid draw */
        uint64_t *head = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)K);
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < K; ++i)
            head[idx[i]] = (e[i] != INVALID && (i == 0 || e[i] != e[i - 1])) ? e[i] : INVALID;
        free(idx);
        free(e);
        have = 0;
        int64_t k = 0;
        for (; k < K && have < target_m; ++k)
            if (head[k] != INVALID) keys[have++] = head[k];
        k_used = k;
        free(head);
        K += K / 2;
    }
    /* dangling set: first n_dangling entries of a permutation of V */
    int32_t *pd = permutation(n, kd);
    uint8_t *isd = (uint8_t *)calloc((size_t)n, 1);
    for (int64_t i = 0; i < n_dangling; ++i) isd[pd[i]] = 1;
    free(pd);
    int64_t w = 0;
    for (int64_t i = 0; i < have; ++i)
        if (!isd[keys[i] >> 32]) keys[w++] = keys[i];
    free(isd);
    int32_t *pr = permutation(n, kr);
    prgen_graph *g = to_csr(keys, w, n, pr);
    g->draws = k_used;
    free(pr);
    free(keys);
    return g;
}

/* ------------------------------------------------------------------------ */
/* Large R-MAT workload: (edge_factor << scale) draws, self-loops and        */
/* duplicates removed.  A permutation of V picks the dangling set (first     */
/* dangling_frac * n: out-edges dropped) and the unreferenced set (next      */
/* unref_frac * n): every edge into it is redirected to a uniform vertex     */
/* outside it, redrawn on self-loop or repeat within the row.  Relabel last. */
/* ------------------------------------------------------------------------ */
prgen_graph *prgen_rmat(int scale, int64_t edge_factor, double a, double b, double c,
                        double dangling_frac, double unref_frac, uint64_t seed, uint32_t wl) {
    if (scale < 1 || scale > 30 || edge_factor < 0) return NULL;
    const int64_t n = (int64_t)1 << scale;
    const int64_t draws = edge_factor << scale;
    uint64_t ke = stream_key(seed, wl, 0), kd = stream_key(seed, wl, 1),
             ku = stream_key(seed, wl, 2), kr = stream_key(seed, wl, 3);
    uint64_t *keys = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(draws > 0 ? draws : 1));
    const double ab = a + b, abc = a + b + c;
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < draws; ++k) keys[k] = rmat_draw(ke, (uint64_t)k, scale, a, ab, abc);
    int64_t cnt = 0;
    for (int64_t k = 0; k < draws; ++k)
        if ((keys[k] >> 32) != (keys[k] & 0xffffffffULL)) keys[cnt++] = keys[k];
    cnt = sort_unique(keys, cnt, n);

    int64_t nd = (int64_t)floor(dangling_frac * (double)n);
    int64_t nu = (int64_t)floor(unref_frac * (double)n);
    if (nd + nu > n) nu = n - nd;
    int32_t *pd = permutation(n, kd);
    uint8_t *cls = (uint8_t *)calloc((size_t)n, 1); /* 1 dangling, 2 unreferenced */
    for (int64_t i = 0; i < nd; ++i) cls[pd[i]] = 1;
    for (int64_t i = nd; i < nd + nu; ++i) cls[pd[i]] = 2;
    free(pd);
    int64_t w = 0;
    for (int64_t i = 0; i < cnt; ++i)
        if (cls[keys[i] >> 32] != 1) keys[w++] = keys[i];
    cnt = w;

    if (nu > 0) {
        int32_t *keep = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n - nu));
        int64_t nk = 0;
        for (int64_t v = 0; v < n; ++v)
            if (cls[v] != 2) keep[nk++] = (int32_t)v;
        /* row boundaries of the (sorted) edge list */
        int64_t *rs = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
        for (int64_t i = 0; i < cnt; ++i) rs[(keys[i] >> 32) + 1]++;
        for (int64_t v = 0; v < n; ++v) rs[v + 1] += rs[v];
#pragma omp parallel
        {
            int64_t cap = 0;
            uint32_t *tab = NULL;
#pragma omp for schedule(dynamic, 1024)
            for (int64_t v = 0; v < n; ++v) {
                int64_t lo = rs[v], hi = rs[v + 1], len = hi - lo;
                if (len == 0) continue;
                int need = 0;
                for (int64_t i = lo; i < hi; ++i)
                    if (cls[keys[i] & 0xffffffffULL] == 2) { need = 1; break; }
                if (!need) continue;
                int64_t want = 16;
                while (want < 2 * len) want <<= 1;
                if (want > cap) { free(tab); cap = want; tab = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)cap); }
                memset(tab, 0xff, sizeof(uint32_t) * (size_t)want);
                const uint64_t mask = (uint64_t)want - 1;
                /* targets that stay */
                for (int64_t i = lo; i < hi; ++i) {
                    uint32_t t = (uint32_t)(keys[i] & 0xffffffffULL);
                    if (cls[t] == 2) continue;
                    uint64_t h = mix64(t) & mask;
                    while (tab[h] != 0xffffffffu) h = (h + 1) & mask;
                    tab[h] = t;
                }
                for (int64_t i = lo; i < hi; ++i) {
                    uint32_t t = (uint32_t)(keys[i] & 0xffffffffULL);
                    if (cls[t] != 2) continue;
                    for (uint64_t att = 0;; ++att) {
                        uint32_t cand = (uint32_t)keep[bounded(rnd_at(ku, (uint64_t)i * 4096 + att), (uint64_t)nk)];
                        if ((int64_t)cand == v) continue;
                        uint64_t h = mix64(cand) & mask;
                        int dup = 0;
                        while (tab[h] != 0xffffffffu) {
                            if (tab[h] == cand) { dup = 1; break; }
                            h = (h + 1) & mask;
                        }
                        if (dup) continue;
                        tab[h] = cand;
                        keys[i] = ((uint64_t)v << 32) | cand;
                        break;
                    }
                }
            }
            free(tab);
        }
        free(rs);
        free(keep);
    }
    free(cls);
    int32_t *pr = permutation(n, kr);
    prgen_graph *g = to_csr(keys, cnt, n, pr);
    g->draws = draws;
    free(pr);
    free(keys);
    return g;
}

/* ------------------------------------------------------------------------ */
/* Layered DAG workload.  A permutation assigns n_layers * layer_size        */
/* vertices to layers.  Every vertex outside the last layer draws z from a   */
/* Zipf(s) law on [1, zmax] and takes out-degree min(zmax, ceil(lambda z));  */
/* lambda is bisected so the total is target_edges (within 0.1 %).  Targets  */
/* are uniform over all vertices of later layers, without repeats.  Then     */
/* round(back_frac * target_edges) back edges: source uniform in layers      */
/* 2..L-2, target uniform in layers 1..layer(source)-1, so layer 0 stays      */
/* unreferenced and layer L-1 dangling.  Relabel last.                       */
/* ------------------------------------------------------------------------ */
prgen_graph *prgen_dag(int n_layers, int64_t layer_size, double zipf_s, int64_t zmax,
                       int64_t target_edges, double back_frac, uint64_t seed, uint32_t wl) {
    if (n_layers < 4 || layer_size < 1 || zmax < 1 || zmax > layer_size) return NULL;
    const int64_t n = (int64_t)n_layers * layer_size;
    if (n > ((int64_t)1 << 31) - 1) return NULL;
    const int64_t nsrc = n - layer_size; /* vertices with forward edges */
    uint64_t kl = stream_key(seed, wl, 4), kz = stream_key(seed, wl, 5), kt = stream_key(seed, wl, 6),
             kb = stream_key(seed, wl, 7), kr = stream_key(seed, wl, 3);
    int32_t *order = permutation(n, kl); /* order[pos]: vertex at position pos; layer = pos / layer_size */
    /* Zipf inverse CDF table */
    double *cdf = (double *)malloc(sizeof(double) * (size_t)zmax);
    double acc = 0.0;
    for (int64_t k = 1; k <= zmax; ++k) { acc += pow((double)k, -zipf_s); cdf[k - 1] = acc; }
    for (int64_t k = 0; k < zmax; ++k) cdf[k] /= acc;
    int32_t *z = (int32_t *)malloc(sizeof(int32_t) * (size_t)nsrc);
#pragma omp parallel for schedule(static)
    for (int64_t pos = 0; pos < nsrc; ++pos) {
        double u = unif01(rnd_at(kz, (uint64_t)pos));
        int64_t lo = 0, hi = zmax - 1;
        while (lo < hi) { int64_t mid = (lo + hi) / 2; if (cdf[mid] > u) hi = mid; else lo = mid + 1; }
        z[pos] = (int32_t)(lo + 1);
    }
    free(cdf);
    /* bisect lambda */
    double lo_l = 0.0, hi_l = (double)zmax, lam = 1.0;
    for (int it = 0; it < 200; ++it) {
        lam = 0.5 * (lo_l + hi_l);
        int64_t tot = 0;
#pragma omp parallel for reduction(+ : tot) schedule(static)
        for (int64_t pos = 0; pos < nsrc; ++pos) {
            double d = ceil(lam * (double)z[pos]);
            tot += d > (double)zmax ? zmax : (int64_t)d;
        }
        if (fabs((double)(tot - target_edges)) <= 1e-3 * (double)target_edges) break;
        if (tot < target_edges) lo_l = lam; else hi_l = lam;
    }
    int64_t *off = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nsrc + 1));
    off[0] = 0;
    for (int64_t pos = 0; pos < nsrc; ++pos) {
        double d = ceil(lam * (double)z[pos]);
        off[pos + 1] = off[pos] + (d > (double)zmax ? zmax : (int64_t)d);
    }
    free(z);
    const int64_t nfwd = off[nsrc];
    const int64_t nback = (int64_t)llround(back_frac * (double)target_edges);
    uint64_t *keys = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(nfwd + nback + 1));
#pragma omp parallel
    {
        int64_t cap = 0;
        uint32_t *tab = NULL;
#pragma omp for schedule(dynamic, 4096)
        for (int64_t pos = 0; pos < nsrc; ++pos) {
            int64_t layer = pos / layer_size;
            int64_t base = (layer + 1) * layer_size, pool = n - base;
            int64_t deg = off[pos + 1] - off[pos];
            int64_t want = 16;
            while (want < 2 * deg) want <<= 1;
            if (want > cap) { free(tab); cap = want; tab = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)cap); }
            memset(tab, 0xff, sizeof(uint32_t) * (size_t)want);
            const uint64_t mask = (uint64_t)want - 1;
            uint64_t ctr = (uint64_t)off[pos] * 4;
            uint32_t s = (uint32_t)order[pos];
            for (int64_t j = 0; j < deg; ++j) {
                for (;;) {
                    uint32_t t = (uint32_t)order[base + (int64_t)bounded(rnd_at(kt, ctr++), (uint64_t)pool)];
                    uint64_t h = mix64(t) & mask;
                    int dup = 0;
                    while (tab[h] != 0xffffffffu) {
                        if (tab[h] == t) { dup = 1; break; }
                        h = (h + 1) & mask;
                    }
                    if (dup) continue;
                    tab[h] = t;
                    keys[off[pos] + j] = ((uint64_t)s << 32) | t;
                    break;
                }
            }
        }
        free(tab);
    }
    /* back edges */
    const int64_t src_lo = 2 * layer_size, src_cnt = (int64_t)(n_layers - 3) * layer_size;
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < nback; ++k) {
        int64_t spos = src_lo + (int64_t)bounded(rnd_at(kb, 2 * (uint64_t)k), (uint64_t)src_cnt);
        int64_t layer = spos / layer_size;
        int64_t tpos = layer_size + (int64_t)bounded(rnd_at(kb, 2 * (uint64_t)k + 1), (uint64_t)((layer - 1) * layer_size));
        keys[nfwd + k] = ((uint64_t)(uint32_t)order[spos] << 32) | (uint64_t)(uint32_t)order[tpos];
    }
    free(off);
    free(order);
    int64_t cnt = sort_unique(keys, nfwd + nback, n);
    int32_t *pr = permutation(n, kr);
    prgen_graph *g = to_csr(keys, cnt, n, pr);
    g->aux = lam;
    g->draws = nfwd + nback;
    free(pr);
    free(keys);
    return g;
}
