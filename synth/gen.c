/*
 * Seeded synthetic graph generators.
 *
 * This file only draws random graphs.  It holds none of the k-clique method's
 * arithmetic and is shared, as an input source, by the CPU oracle's tests and
 * by the GPU path's tests and benchmark.
 *
 * Randomness: SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom
 * number generators", OOPSLA 2014).  Every generator derives an independent
 * stream per row / per item from (seed, index), so a graph depends only on its
 * parameters and seed.
 *
 * Output: an array of undirected pairs (u, v) with u != v, possibly with
 * duplicates when several generators are unioned; the Python side canonicalises
 * the pairs into a sorted, simple, symmetric CSR.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct { uint64_t s; } sm64;

static uint64_t sm64_next(sm64* r) {
    uint64_t z = (r->s += 0x9e3779b97f4a7c15ULL);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

/* Stream for (seed, index): the state is a mix of both, so neighbouring indices
 * give unrelated streams. */
static sm64 sm64_stream(uint64_t seed, uint64_t index) {
    sm64 a = { seed * 0x632be59bd9b4e019ULL + 0x8cb92ba72f3d8dd7ULL };
    uint64_t h = sm64_next(&a);
    sm64 b = { h ^ (index * 0xd1342543de82ef95ULL + 0x9e3779b97f4a7c15ULL) };
    sm64_next(&b);
    return b;
}

/* Uniform double in [0, 1). */
static double sm64_unif(sm64* r) { return (double)(sm64_next(r) >> 11) * 0x1.0p-53; }

/* Growable pair buffer. */
typedef struct { int32_t* p; int64_t n, cap; } pairbuf;

static int pb_push(pairbuf* b, int32_t u, int32_t v) {
    if (b->n == b->cap) {
        int64_t nc = b->cap ? b->cap * 2 : 1024;
        int32_t* q = (int32_t*)realloc(b->p, (size_t)nc * 2 * sizeof(int32_t));
        if (!q) return -1;
        b->p = q; b->cap = nc;
    }
    b->p[2 * b->n] = u; b->p[2 * b->n + 1] = v; b->n++;
    return 0;
}

void synth_free(void* p) { free(p); }

/* Random permutation of 0..n-1 (Fisher-Yates). */
void synth_permutation(int32_t n, uint64_t seed, int32_t* out) {
    for (int32_t i = 0; i < n; i++) out[i] = i;
    sm64 r = sm64_stream(seed, 0x7065726dULL);
    for (int32_t i = n - 1; i > 0; i--) {
        int32_t j = (int32_t)(sm64_next(&r) % (uint64_t)(i + 1));
        int32_t t = out[i]; out[i] = out[j]; out[j] = t;
    }
}

/* Erdos-Renyi G(n, p): every pair {u, v} is an edge independently with
 * probability p.  Uses geometric skipping over the pair sequence (Batagelj and
 * Brandes, "Efficient generation of large random networks", Phys. Rev. E 2005),
 * one stream per row v so rows are independent.  Returns the pair count, or -1
 * on allocation failure; *out receives a malloc'd array of 2*count int32. */
int64_t synth_er(int32_t n, double p, uint64_t seed, int32_t** out) {
    pairbuf b = {0, 0, 0};
    *out = NULL;
    if (n < 2 || p <= 0.0) return 0;
    for (int32_t v = 1; v < n; v++) {
        sm64 r = sm64_stream(seed, (uint64_t)v);
        if (p >= 1.0) {
            for (int32_t w = 0; w < v; w++)
                if (pb_push(&b, v, w)) { free(b.p); return -1; }
            continue;
        }
        double lq = log1p(-p);
        int64_t w = -1;
        for (;;) {
            double u = 1.0 - sm64_unif(&r);           /* (0, 1] */
            w += 1 + (int64_t)floor(log(u) / lq);
            if (w >= v) break;
            if (pb_push(&b, v, (int32_t)w)) { free(b.p); return -1; }
        }
    }
    *out = b.p;
    return b.n;
}

/* i.i.d. weights from a power law with density proportional to w^(-gamma) on
 * [xmin, xmax] (inverse-CDF sampling), one draw per vertex. */
void synth_powerlaw_weights(int32_t n, double gamma, double xmin, double xmax,
                            uint64_t seed, double* w) {
    double a = 1.0 - gamma;
    double lo = pow(xmin, a), hi = pow(xmax, a);
    sm64 r = sm64_stream(seed, 0x776569ULL);
    for (int32_t i = 0; i < n; i++) {
        double u = sm64_unif(&r);
        w[i] = pow(lo + u * (hi - lo), 1.0 / a);
    }
}

static int cmp_desc(const void* x, const void* y) {
    double a = *(const double*)x, b = *(const double*)y;
    return (a < b) - (a > b);
}

/* Chung-Lu graph: pair {u, v} is an edge independently with probability
 * min(1, w_u w_v / sum(w)).  Generated in O(n + m) by the method of Miller and
 * Hagberg ("Efficient generation of networks with given expected degrees",
 * WAW 2011) over the weights sorted in decreasing order; sorted position i is
 * then mapped to vertex id perm[i] (perm a random permutation) so that hubs are
 * scattered over the id space.  `w` is not modified. */
int64_t synth_chung_lu(int32_t n, const double* w, uint64_t seed, int32_t** out) {
    pairbuf b = {0, 0, 0};
    *out = NULL;
    if (n < 2) return 0;
    double* ws = (double*)malloc((size_t)n * sizeof(double));
    int32_t* perm = (int32_t*)malloc((size_t)n * sizeof(int32_t));
    if (!ws || !perm) { free(ws); free(perm); return -1; }
    memcpy(ws, w, (size_t)n * sizeof(double));
    qsort(ws, (size_t)n, sizeof(double), cmp_desc);
    synth_permutation(n, seed ^ 0x5a5a5a5aULL, perm);
    double S = 0.0;
    for (int32_t i = 0; i < n; i++) S += ws[i];
    for (int32_t u = 0; u < n - 1; u++) {
        sm64 r = sm64_stream(seed, (uint64_t)u);
        int64_t v = u + 1;
        double p = fmin(ws[u] * ws[v] / S, 1.0);
        while (v < n && p > 0.0) {
            if (p < 1.0) {
                double x = 1.0 - sm64_unif(&r);
                v += (int64_t)floor(log(x) / log1p(-p));
            }
            if (v < n) {
                double q = fmin(ws[u] * ws[v] / S, 1.0);
                if (sm64_unif(&r) < q / p)
                    if (pb_push(&b, perm[u], perm[v])) { free(b.p); free(ws); free(perm); return -1; }
                p = q;
                v++;
            }
        }
    }
    free(ws); free(perm);
    *out = b.p;
    return b.n;
}

/* Planted communities: `nc` disjoint vertex subsets of sizes drawn uniformly from
 * [smin, smax] (consecutive chunks of a random permutation), each intra-community
 * pair an edge independently with probability p.  Returns -2 if the sizes do not
 * fit in n. */
int64_t synth_communities(int32_t n, int32_t nc, int32_t smin, int32_t smax, double p,
                          uint64_t seed, int32_t* sizes_out, int32_t** out) {
    pairbuf b = {0, 0, 0};
    *out = NULL;
    int32_t* perm = (int32_t*)malloc((size_t)n * sizeof(int32_t));
    if (!perm) return -1;
    synth_permutation(n, seed ^ 0xc0ffeeULL, perm);
    sm64 rs = sm64_stream(seed, 0x73697a65ULL);
    int64_t off = 0;
    for (int32_t c = 0; c < nc; c++) {
        int32_t sz = smin + (int32_t)(sm64_next(&rs) % (uint64_t)(smax - smin + 1));
        if (off + sz > n) { free(perm); free(b.p); return -2; }
        if (sizes_out) sizes_out[c] = sz;
        const int32_t* mem = perm + off;
        for (int32_t i = 0; i < sz; i++) {
            sm64 r = sm64_stream(seed ^ ((uint64_t)c << 32), (uint64_t)i);
            for (int32_t j = i + 1; j < sz; j++)
                if (sm64_unif(&r) < p)
                    if (pb_push(&b, mem[i], mem[j])) { free(perm); free(b.p); return -1; }
        }
        off += sz;
    }
    free(perm);
    *out = b.p;
    return b.n;
}

/* Uniform double in [0, 1) for draw `i` of stream `seed` (used by the Python side
 * for per-graph parameters of batched and served workloads). */
double synth_uniform(uint64_t seed, uint64_t i) {
    sm64 r = sm64_stream(seed, i);
    return sm64_unif(&r);
}

/* ------------------------------------------------------------------ batch */

static int cmp_i32(const void* a, const void* b) {
    int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
    return (x > y) - (x < y);
}

/* Rows sorted ascending: insertion sort for short rows, qsort otherwise. */
static void sort_row(int32_t* r, int64_t len) {
    if (len > 48) { qsort(r, (size_t)len, sizeof(int32_t), cmp_i32); return; }
    for (int64_t i = 1; i < len; i++) {
        int32_t x = r[i];
        int64_t j = i - 1;
        while (j >= 0 && r[j] > x) { r[j + 1] = r[j]; j--; }
        r[j + 1] = x;
    }
}

/* Parameters of graph g of a batch: vertex count log-uniform on [nmin, nmax],
 * kind 0 = Erdos-Renyi / 1 = Chung-Lu (50/50), mean degree uniform on
 * [dmin, dmax] capped at n - 1. */
void synth_batch_params(int32_t g, uint64_t seed, int32_t nmin, int32_t nmax, double dmin, double dmax,
                        int32_t* n, int32_t* kind, double* deg) {
    sm64 r = sm64_stream(seed, (uint64_t)g);
    double u = sm64_unif(&r);
    int32_t nn = (int32_t)floor(exp(log((double)nmin) + u * (log((double)nmax + 1.0) - log((double)nmin))));
    if (nn < nmin) nn = nmin;
    if (nn > nmax) nn = nmax;
    *n = nn;
    *kind = (int32_t)(sm64_next(&r) & 1u);
    double d = dmin + sm64_unif(&r) * (dmax - dmin);
    if (d > nn - 1) d = nn - 1;
    *deg = d;
}

/* Pairs of one batch graph (local ids).  Chung-Lu weights follow a power law
 * w^(-gamma) with the given mean, capped at w_max = n - 1 (the largest degree a
 * simple graph allows); pairs with w_u w_v >= sum w are edges with probability 1. */
static int64_t batch_graph_pairs(int32_t g, uint64_t seed, int32_t n, int32_t kind, double deg, double gamma,
                                 int32_t** out) {
    uint64_t gs = seed * 1000003ULL + (uint64_t)g * 7919ULL + 17ULL;
    if (kind == 0 || n < 3) return synth_er(n, n > 1 ? deg / (n - 1) : 0.0, gs, out);
    double wmax = n - 1;
    /* x_min by bisection on the truncated power-law mean */
    double lo = 1e-6, hi = deg;
    for (int it = 0; it < 200; it++) {
        double xm = 0.5 * (lo + hi);
        double a = 1.0 - gamma, b = 2.0 - gamma;
        double norm = (pow(wmax, a) - pow(xm, a)) / a;
        double first = (pow(wmax, b) - pow(xm, b)) / b;
        if (first / norm < deg) lo = xm; else hi = xm;
    }
    double* w = (double*)malloc((size_t)n * sizeof(double));
    if (!w) return -1;
    synth_powerlaw_weights(n, gamma, 0.5 * (lo + hi), wmax, gs, w);
    int64_t c = synth_chung_lu(n, w, gs, out);
    free(w);
    return c;
}

/* Total vertex count of a batch (to size buffers). */
int64_t synth_batch_vertices(int32_t ngraphs, uint64_t seed, int32_t nmin, int32_t nmax, double dmin, double dmax) {
    int64_t tot = 0;
    for (int32_t g = 0; g < ngraphs; g++) {
        int32_t n, kind;
        double d;
        synth_batch_params(g, seed, nmin, nmax, dmin, dmax, &n, &kind, &d);
        tot += n;
    }
    return tot;
}

/* Build the packed CSR of a batch: voff[ngraphs+1] (vertex offsets), row_ptr[N+1]
 * (global offsets, int64), and a malloc'd col array (global ids) in *col_out.
 * Returns the entry count (nnz) or -1. */
int64_t synth_batch(int32_t ngraphs, uint64_t seed, int32_t nmin, int32_t nmax, double dmin, double dmax,
                    double gamma, int32_t* voff, int64_t* row_ptr, int32_t** col_out) {
    *col_out = NULL;
    int64_t V = 0;
    voff[0] = 0;
    for (int32_t g = 0; g < ngraphs; g++) {
        int32_t n, kind;
        double d;
        synth_batch_params(g, seed, nmin, nmax, dmin, dmax, &n, &kind, &d);
        V += n;
        voff[g + 1] = (int32_t)V;
    }
    int64_t cap = 1 << 20, nnz = 0;
    int32_t* col = (int32_t*)malloc((size_t)cap * sizeof(int32_t));
    int64_t* deg = (int64_t*)calloc((size_t)(V + 1), sizeof(int64_t));
    if (!col || !deg) { free(col); free(deg); return -1; }
    row_ptr[0] = 0;
    for (int32_t g = 0; g < ngraphs; g++) {
        int32_t n = voff[g + 1] - voff[g], kind;
        double d;
        synth_batch_params(g, seed, nmin, nmax, dmin, dmax, &n, &kind, &d);
        int32_t* pairs = NULL;
        int64_t np = batch_graph_pairs(g, seed, n, kind, d, gamma, &pairs);
        if (np < 0) { free(col); free(deg); return -1; }
        int32_t base = voff[g];
        for (int32_t v = 0; v < n; v++) deg[base + v] = 0;
        for (int64_t e = 0; e < np; e++) { deg[base + pairs[2 * e]]++; deg[base + pairs[2 * e + 1]]++; }
        int64_t need = nnz + 2 * np;
        if (need > cap) {
            while (cap < need) cap *= 2;
            int32_t* q = (int32_t*)realloc(col, (size_t)cap * sizeof(int32_t));
            if (!q) { free(pairs); free(col); free(deg); return -1; }
            col = q;
        }
        /* offsets of this graph's rows, then scatter both directions */
        for (int32_t v = 0; v < n; v++) row_ptr[base + v + 1] = row_ptr[base + v] + deg[base + v];
        for (int32_t v = 0; v < n; v++) deg[base + v] = row_ptr[base + v];
        for (int64_t e = 0; e < np; e++) {
            int32_t a = pairs[2 * e], b = pairs[2 * e + 1];
            col[deg[base + a]++] = base + b;
            col[deg[base + b]++] = base + a;
        }
        for (int32_t v = 0; v < n; v++) sort_row(col + row_ptr[base + v], row_ptr[base + v + 1] - row_ptr[base + v]);
        nnz = need;
        free(pairs);
    }
    free(deg);
    *col_out = col;
    return nnz;
}
