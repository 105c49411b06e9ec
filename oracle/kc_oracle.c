/*
 * CPU ORACLE for exact k-clique counting -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, single-threaded and meant to be obviously correct.  Only the test
 * suite, the smoke check and the benchmark's CPU-baseline leg may load it; the
 * GPU library never does, and the two share no code.
 *
 * Paper: Almasri, El Hajj, Nagi, Xiong, Hwu, "Parallel K-clique Counting on GPUs"
 * (ICS 2022, arXiv 2104.13209).
 *
 * What it computes
 *   c_k(G) = number of k-vertex subsets of V that are pairwise adjacent (Sec. 1
 *   problem statement), by walking one of the paper's two search trees from each
 *   root, depth first with an explicit stack:
 *     - the orientation tree (Sec. 2.2): a node is a clique with the common
 *       out-neighbours of its vertices; vertex-rooted or edge-rooted;
 *     - the pivoting tree (Sec. 2.3) in the hybrid form of Sec. 2.3 / 2.4: the
 *       root level (vertex root) or two levels (edge root) follow the oriented
 *       graph, every level below works on undirected adjacency; a node branches
 *       only on the candidates outside its pivot's neighbourhood, and a leaf
 *       stands for a binomial number of cliques.
 *   All intersections are merges of sorted int vectors (or binary search when one
 *   list is far shorter); there is no blocking, fusion or bit encoding here.
 *
 * Readings of the paper (each also listed in the design notes):
 *   R1  Fig. 3's level variable counts the path vertices before the branch
 *       vertex, so a vertex root starts with one hold and an edge root with two;
 *       a leaf whose path has n_h holds and n_p pivots then adds
 *       C(n_p, n_h + n_p - k), which is Sec. 2.3's C(n_p, n_v - k).  The walk
 *       keeps the holds and pivots of the path itself.
 *   R2  Pivot = argmax over u in I of |I intersect Adj(u)|; ties go to the
 *       smallest vertex id.  (Any pivot in I gives the same count.)
 *   R3  The order "<" in Fig. 3's exclusion set is vertex id order.
 *   R4  Degree order: edge u->v iff (deg u, u) < (deg v, v).
 *   R5  Degeneracy order: repeatedly remove a vertex of minimum current degree,
 *       smallest id first on ties (Matula-Beck); edge u->v iff u is removed first.
 *   R8  Approximate degeneracy order (a relaxation of k-core, one of the
 *       orientation criteria of Sec. 2; the rule of ARB-COUNT's approximate
 *       peeling with eps = 1/10): in rounds r = 0, 1, ..., with L vertices left
 *       of total current degree D, every remaining vertex whose degree is at
 *       most 1.1 D / L (10 deg L <= 11 D, exact in integers) leaves in round r;
 *       then the remaining neighbours of the leavers lose one degree each.  The
 *       order is by (round, id).
 *   R9  Colouring order (graph colouring, one of the orientation criteria of
 *       Sec. 2): vertices are coloured greedily, each with the smallest colour
 *       absent from its already coloured neighbours, visiting them by decreasing
 *       priority p(v) and then decreasing id, where p(v) is SplitMix64's output
 *       for the counter value v (its mixing function applied to v plus the
 *       golden-ratio increment 0x9E3779B97F4A7C15; Steele, Lea and Flood,
 *       OOPSLA 2014).  The order is by (colour, id).
 *   R6  k = 1 gives n, k = 2 gives m (outside the pseudocode); counts[0] = 1 is
 *       the empty clique.
 *   R7  Counts are unsigned 128-bit; any carry out of bit 127 sets an overflow flag.
 *
 * Parity status: every function here is pinned by the CPU test suite against
 * brute-force enumeration, closed forms, a library routine, or the paper's
 * worked instance (see the tests); none is "parity unpinned".
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;

enum { KCO_OK = 0, KCO_EINVAL = -1, KCO_ENOMEM = -2, KCO_EOVERFLOW = -3 };
enum { KCO_DEGREE = 0, KCO_DEGENERACY = 1, KCO_APPROX_DEGENERACY = 2, KCO_COLOR = 3 };
enum { KCO_VC = 1, KCO_EC = 2 };

/* ------------------------------------------------------------------ input */

/* 0 if (row_ptr, col) is a simple symmetric graph with strictly increasing rows
 * and ids in range; KCO_EINVAL otherwise. */
int kco_validate(int32_t n, const int32_t* row_ptr, const int32_t* col) {
    if (n < 0 || row_ptr[0] != 0) return KCO_EINVAL;
    for (int32_t v = 0; v < n; v++) {
        if (row_ptr[v + 1] < row_ptr[v]) return KCO_EINVAL;
        for (int32_t e = row_ptr[v]; e < row_ptr[v + 1]; e++) {
            int32_t w = col[e];
            if (w < 0 || w >= n || w == v) return KCO_EINVAL;
            if (e > row_ptr[v] && col[e - 1] >= w) return KCO_EINVAL;
            /* symmetric: v must appear in w's row */
            int32_t lo = row_ptr[w], hi = row_ptr[w + 1];
            while (lo < hi) {
                int32_t mid = lo + (hi - lo) / 2;
                if (col[mid] < v) lo = mid + 1; else hi = mid;
            }
            if (lo == row_ptr[w + 1] || col[lo] != v) return KCO_EINVAL;
        }
    }
    return KCO_OK;
}

/* ------------------------------------------------------------ orientation */

static const int32_t* g_deg_for_sort;
static int cmp_degree_id(const void* a, const void* b) {
    int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
    if (g_deg_for_sort[x] != g_deg_for_sort[y]) return g_deg_for_sort[x] < g_deg_for_sort[y] ? -1 : 1;
    return (x > y) - (x < y);
}

/* R9: SplitMix64 output for counter value x: the mixing function of the
 * generator applied to x + 0x9E3779B97F4A7C15. */
uint64_t kco_splitmix64(uint64_t x) {
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static const uint64_t* g_prio_for_sort;
/* decreasing (priority, id) */
static int cmp_priority_desc(const void* a, const void* b) {
    int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
    uint64_t px = g_prio_for_sort[x], py = g_prio_for_sort[y];
    if (px != py) return px > py ? -1 : 1;
    return (x < y) - (x > y);
}

/* R9: greedy first-fit colouring in decreasing (priority, id) order; colour[v]
 * receives v's colour (0-based). */
int kco_colour(int32_t n, const int32_t* row_ptr, const int32_t* col, int32_t* colour) {
    int32_t* ids = (int32_t*)malloc((size_t)(n ? n : 1) * sizeof(int32_t));
    uint64_t* prio = (uint64_t*)malloc((size_t)(n ? n : 1) * sizeof(uint64_t));
    char* taken = (char*)calloc((size_t)n + 1, 1);
    if (!ids || !prio || !taken) { free(ids); free(prio); free(taken); return KCO_ENOMEM; }
    for (int32_t v = 0; v < n; v++) { prio[v] = kco_splitmix64((uint64_t)v); ids[v] = v; colour[v] = -1; }
    g_prio_for_sort = prio;
    qsort(ids, (size_t)n, sizeof(int32_t), cmp_priority_desc);
    for (int32_t i = 0; i < n; i++) {
        int32_t v = ids[i], c = 0;
        for (int32_t e = row_ptr[v]; e < row_ptr[v + 1]; e++)
            if (colour[col[e]] >= 0) taken[colour[col[e]]] = 1;
        while (taken[c]) c++;
        colour[v] = c;
        for (int32_t e = row_ptr[v]; e < row_ptr[v + 1]; e++)
            if (colour[col[e]] >= 0) taken[colour[col[e]]] = 0;
    }
    free(ids); free(prio); free(taken);
    return KCO_OK;
}

/* Binary min-heap of (key, id) with lazy deletion, for the degeneracy peel. */
typedef struct { int64_t* a; int64_t n, cap; } heap64;
static int heap_push(heap64* h, int64_t x) {
    if (h->n == h->cap) {
        int64_t nc = h->cap ? 2 * h->cap : 1024;
        int64_t* q = (int64_t*)realloc(h->a, (size_t)nc * sizeof(int64_t));
        if (!q) return -1;
        h->a = q; h->cap = nc;
    }
    int64_t i = h->n++;
    h->a[i] = x;
    while (i > 0) {
        int64_t p = (i - 1) / 2;
        if (h->a[p] <= h->a[i]) break;
        int64_t t = h->a[p]; h->a[p] = h->a[i]; h->a[i] = t; i = p;
    }
    return 0;
}
static int64_t heap_pop(heap64* h) {
    int64_t top = h->a[0];
    h->a[0] = h->a[--h->n];
    int64_t i = 0;
    for (;;) {
        int64_t l = 2 * i + 1, r = l + 1, s = i;
        if (l < h->n && h->a[l] < h->a[s]) s = l;
        if (r < h->n && h->a[r] < h->a[s]) s = r;
        if (s == i) break;
        int64_t t = h->a[s]; h->a[s] = h->a[i]; h->a[i] = t; i = s;
    }
    return top;
}

/* Orientation (Sec. 3.1): rank[] is the position of each vertex in the order
 * (R4 / R5); the DAG keeps edge u->v iff rank[u] < rank[v].  Out-lists are in
 * vertex id order.  out_ptr has n+1 entries, out_col m = nnz/2 entries.
 * *degeneracy receives the largest current degree seen at a removal (degeneracy
 * order) or -1 (degree and approximate degeneracy order). */
int kco_orient(int32_t n, const int32_t* row_ptr, const int32_t* col, int order,
               int32_t* out_ptr, int32_t* out_col, int32_t* rank,
               int32_t* d_max, int32_t* degeneracy) {
    if (n < 0 || (order != KCO_DEGREE && order != KCO_DEGENERACY && order != KCO_APPROX_DEGENERACY &&
                  order != KCO_COLOR))
        return KCO_EINVAL;
    int32_t* ids = (int32_t*)malloc((size_t)(n ? n : 1) * sizeof(int32_t));
    int32_t* deg = (int32_t*)malloc((size_t)(n ? n : 1) * sizeof(int32_t));
    if (!ids || !deg) { free(ids); free(deg); return KCO_ENOMEM; }
    for (int32_t v = 0; v < n; v++) deg[v] = row_ptr[v + 1] - row_ptr[v];
    *degeneracy = -1;
    if (order == KCO_DEGREE) {
        for (int32_t v = 0; v < n; v++) ids[v] = v;
        g_deg_for_sort = deg;
        qsort(ids, (size_t)n, sizeof(int32_t), cmp_degree_id);
    } else if (order == KCO_COLOR) {
        /* R9: sort by (colour, id); deg[] is reused to hold the colours */
        if (kco_colour(n, row_ptr, col, deg) != KCO_OK) { free(ids); free(deg); return KCO_ENOMEM; }
        for (int32_t v = 0; v < n; v++) ids[v] = v;
        g_deg_for_sort = deg;
        qsort(ids, (size_t)n, sizeof(int32_t), cmp_degree_id);
    } else if (order == KCO_APPROX_DEGENERACY) {
        /* R8: whole rounds of low-degree vertices, in id order within a round */
        int32_t* round = (int32_t*)malloc((size_t)(n ? n : 1) * sizeof(int32_t));
        if (!round) { free(ids); free(deg); return KCO_ENOMEM; }
        for (int32_t v = 0; v < n; v++) round[v] = -1;
        int32_t removed = 0;
        for (int32_t r = 0; removed < n; r++) {
            int64_t L = 0, D = 0;
            for (int32_t v = 0; v < n; v++)
                if (round[v] < 0) { L++; D += deg[v]; }
            int32_t first = removed;
            for (int32_t v = 0; v < n; v++)
                if (round[v] < 0 && 10 * (int64_t)deg[v] * L <= 11 * D) { round[v] = r; ids[removed++] = v; }
            for (int32_t i = first; i < removed; i++) {
                int32_t v = ids[i];
                for (int32_t e = row_ptr[v]; e < row_ptr[v + 1]; e++)
                    if (round[col[e]] < 0) deg[col[e]]--;
            }
        }
        free(round);
    } else {
        /* Matula-Beck peel: pop the (current degree, id) minimum; skip stale
         * heap entries; decrement the degrees of still-present neighbours. */
        char* gone = (char*)calloc((size_t)(n ? n : 1), 1);
        heap64 h = {0, 0, 0};
        int32_t removed = 0, degen = 0;
        if (!gone) { free(ids); free(deg); return KCO_ENOMEM; }
        for (int32_t v = 0; v < n; v++)
            if (heap_push(&h, ((int64_t)deg[v] << 32) | (uint32_t)v)) goto oom;
        while (removed < n) {
            int64_t x = heap_pop(&h);
            int32_t v = (int32_t)(x & 0xffffffff), d = (int32_t)(x >> 32);
            if (gone[v] || d != deg[v]) continue;       /* stale entry */
            gone[v] = 1;
            ids[removed++] = v;
            if (d > degen) degen = d;
            for (int32_t e = row_ptr[v]; e < row_ptr[v + 1]; e++) {
                int32_t w = col[e];
                if (!gone[w]) {
                    deg[w]--;
                    if (heap_push(&h, ((int64_t)deg[w] << 32) | (uint32_t)w)) goto oom;
                }
            }
        }
        *degeneracy = degen;
        free(h.a); free(gone);
        goto peeled;
    oom:
        free(h.a); free(gone); free(ids); free(deg);
        return KCO_ENOMEM;
    }
peeled:
    for (int32_t i = 0; i < n; i++) rank[ids[i]] = i;
    int32_t dm = 0, pos = 0;
    out_ptr[0] = 0;
    for (int32_t u = 0; u < n; u++) {
        for (int32_t e = row_ptr[u]; e < row_ptr[u + 1]; e++)
            if (rank[u] < rank[col[e]]) out_col[pos++] = col[e];
        out_ptr[u + 1] = pos;
        if (pos - out_ptr[u] > dm) dm = pos - out_ptr[u];
    }
    *d_max = dm;
    free(ids); free(deg);
    return KCO_OK;
}

/* ----------------------------------------------------------- set algebra */

static int32_t find_ge(const int32_t* b, int32_t nb, int32_t x) {
    int32_t lo = 0, hi = nb;
    while (lo < hi) {
        int32_t mid = lo + (hi - lo) / 2;
        if (b[mid] < x) lo = mid + 1; else hi = mid;
    }
    return lo;
}

/* out = a intersect b (both sorted ascending); returns |out|. */
static int32_t intersect(const int32_t* a, int32_t na, const int32_t* b, int32_t nb, int32_t* out) {
    int32_t c = 0;
    if ((int64_t)na * 16 < nb) {
        for (int32_t i = 0; i < na; i++) {
            int32_t j = find_ge(b, nb, a[i]);
            if (j < nb && b[j] == a[i]) out[c++] = a[i];
        }
        return c;
    }
    if ((int64_t)nb * 16 < na) {
        for (int32_t j = 0; j < nb; j++) {
            int32_t i = find_ge(a, na, b[j]);
            if (i < na && a[i] == b[j]) out[c++] = b[j];
        }
        return c;
    }
    int32_t i = 0, j = 0;
    while (i < na && j < nb) {
        if (a[i] < b[j]) i++;
        else if (a[i] > b[j]) j++;
        else { out[c++] = a[i]; i++; j++; }
    }
    return c;
}

static int contains(const int32_t* b, int32_t nb, int32_t x) {
    int32_t j = find_ge(b, nb, x);
    return j < nb && b[j] == x;
}

/* ------------------------------------------------------------ accumulation */

typedef struct {
    u128 total;
    u128* counts;      /* count_all: counts[0..cap] */
    int32_t cap;
    u128* local;       /* local counts, per vertex (original ids) */
    int overflow;
    uint64_t nodes;    /* tree nodes visited (one per intersection with Adj(v)) */
} acc_t;

static void add128(u128* x, u128 y, int* ovf) {
    u128 s = *x + y;
    if (s < *x) *ovf = 1;
    *x = s;
}

/* Pascal table C[i][j] for 0 <= j <= i <= N, with per-entry overflow marks. */
typedef struct { int32_t N; u128* c; char* big; } binom_t;
static int binom_init(binom_t* b, int32_t N) {
    b->N = N;
    b->c = (u128*)calloc((size_t)(N + 1) * (N + 1), sizeof(u128));
    b->big = (char*)calloc((size_t)(N + 1) * (N + 1), 1);
    if (!b->c || !b->big) return -1;
    for (int32_t i = 0; i <= N; i++) {
        b->c[(size_t)i * (N + 1)] = 1;
        for (int32_t j = 1; j <= i; j++) {
            u128 x = b->c[(size_t)(i - 1) * (N + 1) + j - 1];
            u128 y = j <= i - 1 ? b->c[(size_t)(i - 1) * (N + 1) + j] : 0;
            char big = b->big[(size_t)(i - 1) * (N + 1) + j - 1] |
                       (j <= i - 1 ? b->big[(size_t)(i - 1) * (N + 1) + j] : 0);
            u128 s = x + y;
            if (s < x) big = 1;
            b->c[(size_t)i * (N + 1) + j] = s;
            b->big[(size_t)i * (N + 1) + j] = big;
        }
    }
    return 0;
}
static void binom_free(binom_t* b) { free(b->c); free(b->big); }
static u128 binom(const binom_t* b, int32_t i, int32_t j, int* ovf) {
    if (j < 0 || j > i) return 0;
    if (b->big[(size_t)i * (b->N + 1) + j]) *ovf = 1;
    return b->c[(size_t)i * (b->N + 1) + j];
}

/* ---------------------------------------------------------------- graph */

typedef struct {
    int32_t n;
    const int32_t *optr, *ocol;   /* oriented DAG, out-lists sorted by id */
    const int32_t *uptr, *ucol;   /* undirected graph (pivoting levels) */
    int32_t d_max;
} graph_t;

static const int32_t* outN(const graph_t* g, int32_t v, int32_t* len) {
    *len = g->optr[v + 1] - g->optr[v];
    return g->ocol + g->optr[v];
}
static const int32_t* undN(const graph_t* g, int32_t v, int32_t* len) {
    *len = g->uptr[v + 1] - g->uptr[v];
    return g->ucol + g->uptr[v];
}

/* Per-level vertex buffers (two of d_max + 1 entries each), allocated when a
 * level is first reached. */
typedef struct { int32_t** buf; int32_t nlev; int32_t width; int failed; } levels_t;
static int32_t* level_buf(levels_t* L, int32_t l, int which) {
    if (l >= L->nlev) {
        int32_t nn = L->nlev ? L->nlev : 8;
        while (nn <= l) nn *= 2;
        int32_t** q = (int32_t**)realloc(L->buf, (size_t)nn * sizeof(int32_t*));
        if (!q) { L->failed = 1; return NULL; }
        for (int32_t i = L->nlev; i < nn; i++) q[i] = NULL;
        L->buf = q; L->nlev = nn;
    }
    if (!L->buf[l]) {
        L->buf[l] = (int32_t*)malloc((size_t)2 * L->width * sizeof(int32_t));
        if (!L->buf[l]) { L->failed = 1; return NULL; }
    }
    return L->buf[l] + (size_t)which * L->width;
}
static void levels_free(levels_t* L) {
    for (int32_t i = 0; i < L->nlev; i++) free(L->buf[i]);
    free(L->buf);
}

/* Path of the current branch: `holds` gets the non-pivot vertices (all of them
 * in graph orientation), `pivots` the pivots.  Grown on demand. */
typedef struct { int32_t* v; int32_t cap; } path_t;
static int path_set(path_t* p, int32_t i, int32_t x) {
    if (i >= p->cap) {
        int32_t nc = p->cap ? 2 * p->cap : 16;
        while (nc <= i) nc *= 2;
        int32_t* q = (int32_t*)realloc(p->v, (size_t)nc * sizeof(int32_t));
        if (!q) return -1;
        p->v = q; p->cap = nc;
    }
    p->v[i] = x;
    return 0;
}

enum { MODE_K = 0, MODE_ALL = 1, MODE_LOCAL = 2 };

typedef struct {
    const graph_t* g;
    int32_t k;
    int mode;
    const binom_t* bn;
    levels_t lev;
    path_t holds, pivots;
    int32_t* scratch;   /* d_max + 1 entries for intersections used at once */
    acc_t* acc;
} ctx_t;

/* ------------------------------------------------- search-tree walks */

/* Both walks visit the nodes of a search tree depth first with an explicit
 * stack of frames, one per depth.  A frame holds the node's candidate set, the
 * vertices it branches on and how far the branching has got.  The frame at
 * stack index i keeps its candidate set in buffer 0 of level i (the root's is
 * the caller's) and its branch list in buffer 1; a child is always built at
 * index i + 1, whose buffers no live frame uses.  Candidate sets stay sorted by
 * id: each is a filtered intersection of sorted lists. */
typedef struct {
    const int32_t* C; int32_t nC;   /* candidate set */
    int32_t* B; int32_t nB;         /* branch vertices, ascending */
    int32_t next;                   /* index of the next branch in B */
    int32_t p;                      /* pivot (pivoting walk) */
    int32_t nh, np;                 /* holds and pivots on the path to the node */
} frame_t;

typedef struct { frame_t* f; int32_t n, cap; } fstack_t;
static frame_t* fs_push(fstack_t* s) {
    if (s->n == s->cap) {
        int32_t nc = s->cap ? 2 * s->cap : 16;
        frame_t* q = (frame_t*)realloc(s->f, (size_t)nc * sizeof(frame_t));
        if (!q) return NULL;
        s->f = q; s->cap = nc;
    }
    return &s->f[s->n++];
}

/* Orientation tree (Sec. 2.2): a node is a clique Q, listed in holds[0..q), with
 * C = the common out-neighbours of Q.  Each x in C closes the (q+1)-clique
 * Q + x, so the node stands for |C| cliques of size q + 1; its children are
 * Q + v with candidates C cap N+(v), for every v in C.  For a fixed k the walk
 * stops at q = k - 1, where the |C| cliques are k-cliques; counting all sizes, it
 * adds |C| to c_(q+1) at every node and runs until the candidate sets are empty.
 * Every child costs one intersection: that is the node count reported. */
static void local_add_clique_node(ctx_t* c, int32_t q, const int32_t* C, int32_t nC) {
    /* each of the q vertices of Q is in all nC k-cliques, each x in C in one */
    for (int32_t i = 0; i < q; i++) add128(&c->acc->local[c->holds.v[i]], (u128)nC, &c->acc->overflow);
    for (int32_t j = 0; j < nC; j++) add128(&c->acc->local[C[j]], 1, &c->acc->overflow);
}

/* Applies the node's contribution; returns 1 when the node has children. */
static int orient_node(ctx_t* c, int32_t q, const int32_t* C, int32_t nC) {
    acc_t* a = c->acc;
    if (c->mode == MODE_ALL) {
        if (q + 1 >= 3 && q + 1 <= a->cap) add128(&a->counts[q + 1], (u128)nC, &a->overflow);
        return nC > 0;
    }
    if (q == c->k - 1) {
        if (c->mode == MODE_K) add128(&a->total, (u128)nC, &a->overflow);
        else local_add_clique_node(c, q, C, nC);
        return 0;
    }
    return nC > 0;
}

static void orient_walk(ctx_t* c, int32_t q0, const int32_t* C0, int32_t nC0) {
    fstack_t st = {0, 0, 0};
    if (!orient_node(c, q0, C0, nC0)) return;
    frame_t* f = fs_push(&st);
    if (!f) { c->lev.failed = 1; return; }
    *f = (frame_t){C0, nC0, NULL, 0, 0, -1, q0, 0};
    while (st.n > 0 && !c->lev.failed) {
        f = &st.f[st.n - 1];
        if (f->next == f->nC) { st.n--; continue; }
        const int32_t q = f->nh;
        const int32_t v = f->C[f->next++];
        if (path_set(&c->holds, q, v)) { c->lev.failed = 1; break; }
        int32_t* C1 = level_buf(&c->lev, st.n, 0);
        if (!C1) break;
        int32_t na;
        const int32_t* adj = outN(c->g, v, &na);
        int32_t n1 = intersect(f->C, f->nC, adj, na, C1);
        c->acc->nodes++;
        if (orient_node(c, q + 1, C1, n1)) {
            frame_t* g = fs_push(&st);
            if (!g) { c->lev.failed = 1; break; }
            *g = (frame_t){C1, n1, NULL, 0, 0, -1, q + 1, 0};
        }
    }
    free(st.f);
}

/* Pivoting tree (Sec. 2.3).  A node carries holds H and pivots P (its path) and
 * the candidate set C of common neighbours of the path, on the undirected
 * graph.  An empty C is a leaf: it stands for the cliques H + P' with P' any
 * subset of P, so it holds C(|P|, k - |H|) k-cliques.  Otherwise the node picks
 * a pivot p in C (reading R2) and branches only on B = C minus N(p) (p itself
 * included): the branch on p adds p to the pivots, any other branch v adds v to
 * the holds.  The child on v has candidates C cap N(v) without the vertices of
 * B that precede v (reading R3), so each clique is reached once.  For a fixed
 * k a branch whose holds would exceed k is skipped (reading R11). */
static void piv_leaf(ctx_t* c, int32_t nh, int32_t np) {
    acc_t* a = c->acc;
    int32_t k = c->k;
    if (c->mode == MODE_K) {
        if (nh + np >= k) add128(&a->total, binom(c->bn, np, nh + np - k, &a->overflow), &a->overflow);
    } else if (c->mode == MODE_ALL) {
        for (int32_t j = 0; j <= np; j++)
            if (nh + j <= a->cap) add128(&a->counts[nh + j], binom(c->bn, np, j, &a->overflow), &a->overflow);
    } else if (nh <= k && k - nh <= np) {
        /* a hold is in every one of the C(np, k - nh) k-cliques, a pivot in those
         * whose P' contains it: C(np - 1, k - nh - 1) */
        u128 per_hold = binom(c->bn, np, k - nh, &a->overflow);
        u128 per_pivot = binom(c->bn, np - 1, k - nh - 1, &a->overflow);
        for (int32_t q = 0; q < nh; q++) add128(&a->local[c->holds.v[q]], per_hold, &a->overflow);
        for (int32_t q = 0; q < np; q++) add128(&a->local[c->pivots.v[q]], per_pivot, &a->overflow);
    }
}

/* Fills frame `f` (stack index idx) for a node with a non-empty candidate set:
 * its pivot and branch list B. */
static int piv_open(ctx_t* c, frame_t* f, int32_t idx, const int32_t* C, int32_t nC, int32_t nh, int32_t np) {
    const graph_t* g = c->g;
    int32_t* B = level_buf(&c->lev, idx, 1);
    if (!B) return -1;
    /* R2: the candidate with the most neighbours inside C, smallest id on ties */
    int32_t p = C[0], best = -1;
    for (int32_t i = 0; i < nC; i++) {
        int32_t na;
        const int32_t* adj = undN(g, C[i], &na);
        int32_t inside = intersect(C, nC, adj, na, c->scratch);
        if (inside > best) { best = inside; p = C[i]; }
    }
    int32_t pa, nB = 0;
    const int32_t* padj = undN(g, p, &pa);
    for (int32_t i = 0; i < nC; i++)
        if (!contains(padj, pa, C[i])) B[nB++] = C[i];
    *f = (frame_t){C, nC, B, nB, 0, p, nh, np};
    return 0;
}

static void piv_walk(ctx_t* c, int32_t nh0, const int32_t* C0, int32_t nC0) {
    if (nC0 == 0) { piv_leaf(c, nh0, 0); return; }
    fstack_t st = {0, 0, 0};
    frame_t* f = fs_push(&st);
    if (!f || piv_open(c, f, 0, C0, nC0, nh0, 0)) { c->lev.failed = 1; free(st.f); return; }
    while (st.n > 0 && !c->lev.failed) {
        f = &st.f[st.n - 1];
        if (f->next == f->nB) { st.n--; continue; }
        const int32_t v = f->B[f->next++];
        const int is_pivot = v == f->p;
        const int32_t nh = f->nh + !is_pivot, np = f->np + is_pivot;
        if (c->mode == MODE_K && nh > c->k) continue;
        int32_t* C1 = level_buf(&c->lev, st.n, 0);
        if (!C1) break;
        int32_t na;
        const int32_t* adj = undN(c->g, v, &na);
        int32_t n1 = intersect(f->C, f->nC, adj, na, c->scratch);
        int32_t n2 = 0;
        for (int32_t j = 0; j < n1; j++)
            if (!(c->scratch[j] < v && contains(f->B, f->nB, c->scratch[j]))) C1[n2++] = c->scratch[j];
        c->acc->nodes++;
        if (is_pivot ? path_set(&c->pivots, f->np, v) : path_set(&c->holds, f->nh, v)) { c->lev.failed = 1; break; }
        if (n2 == 0) { piv_leaf(c, nh, np); continue; }
        frame_t* g = fs_push(&st);
        if (!g || piv_open(c, g, st.n - 1, C1, n2, nh, np)) { c->lev.failed = 1; break; }
    }
    free(st.f);
}

/* --------------------------------------------------------------- driver */

/* Count over the given roots (all roots when roots == NULL).
 *   scheme KCO_VC: roots are vertices (Sec. 3.2 vertex-centric);
 *   scheme KCO_EC: roots are DAG edge indices (Sec. 3.2 edge-centric).
 *   mode MODE_K: c_k into total; MODE_ALL: counts[] for every size;
 *   MODE_LOCAL: per-vertex counts.
 * The DAG (optr, ocol) and the undirected graph (uptr, ucol) share vertex ids. */
static int run(int32_t n, const int32_t* optr, const int32_t* ocol, const int32_t* uptr,
               const int32_t* ucol, int32_t d_max, int32_t k, int pivot, int scheme, int mode,
               const int64_t* roots, int64_t nroots, acc_t* acc) {
    graph_t g = {n, optr, ocol, uptr, ucol, d_max};
    int32_t m = optr[n];
    binom_t bn = {0, 0, 0};
    ctx_t c;
    memset(&c, 0, sizeof c);
    c.g = &g; c.k = k; c.mode = mode; c.bn = &bn; c.acc = acc;
    c.lev.width = d_max + 1;
    if (pivot && binom_init(&bn, d_max + 2)) return KCO_ENOMEM;
    int32_t* I = (int32_t*)malloc((size_t)(d_max + 1) * sizeof(int32_t));
    c.scratch = (int32_t*)malloc((size_t)(d_max + 1) * sizeof(int32_t));
    int32_t* esrc = NULL;
    if (scheme == KCO_EC) {
        esrc = (int32_t*)malloc((size_t)(m ? m : 1) * sizeof(int32_t));
        if (esrc)
            for (int32_t u = 0; u < n; u++)
                for (int32_t e = optr[u]; e < optr[u + 1]; e++) esrc[e] = u;
    }
    if (!I || !c.scratch || (scheme == KCO_EC && !esrc)) {
        free(I); free(c.scratch); free(esrc); binom_free(&bn);
        return KCO_ENOMEM;
    }
    int64_t nr = roots ? nroots : (scheme == KCO_VC ? n : m);
    for (int64_t r = 0; r < nr && !c.lev.failed; r++) {
        int64_t root = roots ? roots[r] : r;
        int32_t nI, l;
        if (scheme == KCO_VC) {
            int32_t u = (int32_t)root, na;
            const int32_t* a = outN(&g, u, &na);
            memcpy(I, a, (size_t)na * sizeof(int32_t));
            nI = na;
            l = 1;
            if (path_set(&c.holds, 0, u)) c.lev.failed = 1;
        } else {
            int32_t u = esrc[root], v = ocol[root], na, nb;
            const int32_t* a = outN(&g, u, &na);
            const int32_t* b = outN(&g, v, &nb);
            nI = intersect(a, na, b, nb, I);
            l = 2;
            if (path_set(&c.holds, 0, u) || path_set(&c.holds, 1, v)) c.lev.failed = 1;
        }
        if (c.lev.failed) break;
        /* the root node: Q = {u} with C = N+(u), or Q = {u, v} with
         * C = N+(u) cap N+(v); with pivoting the root vertices are holds and
         * every level below works on the undirected graph (Sec. 2.3's hybrid) */
        if (pivot) piv_walk(&c, l, I, nI);
        else if (mode == MODE_ALL || k >= 3) orient_walk(&c, l, I, nI);
    }
    int failed = c.lev.failed;
    levels_free(&c.lev);
    free(c.holds.v); free(c.pivots.v);
    free(esrc); free(I); free(c.scratch); binom_free(&bn);
    return failed ? KCO_ENOMEM : KCO_OK;
}

/* c_k over the given roots (all roots when roots == NULL).  Result as two u64
 * halves; returns KCO_EOVERFLOW when the true value needs more than 128 bits.
 * k = 1 and k = 2 follow R6 when roots == NULL.  *nodes receives the number of
 * tree nodes visited (intersections with an adjacency list). */
int kco_count(int32_t n, const int32_t* optr, const int32_t* ocol, const int32_t* uptr,
              const int32_t* ucol, int32_t d_max, int32_t k, int pivot, int scheme,
              const int64_t* roots, int64_t nroots, uint64_t* out_lo, uint64_t* out_hi,
              uint64_t* nodes) {
    if (k < 1 || (scheme != KCO_VC && scheme != KCO_EC)) return KCO_EINVAL;
    acc_t acc;
    memset(&acc, 0, sizeof acc);
    int st = KCO_OK;
    if (k == 1 && !roots) acc.total = (u128)n;
    else if (k == 2 && !roots) acc.total = (u128)optr[n];
    else st = run(n, optr, ocol, uptr, ucol, d_max, k, pivot, scheme, MODE_K, roots, nroots, &acc);
    *out_lo = (uint64_t)acc.total;
    *out_hi = (uint64_t)(acc.total >> 64);
    if (nodes) *nodes = acc.nodes;
    if (st) return st;
    return acc.overflow ? KCO_EOVERFLOW : KCO_OK;
}

/* counts[j] = c_j for j = 0..cap (as lo/hi pairs, 2*(cap+1) u64).  counts[0] = 1,
 * counts[1] = n, counts[2] = m; the rest come from the traversal with no k bound. */
int kco_count_all(int32_t n, const int32_t* optr, const int32_t* ocol, const int32_t* uptr,
                  const int32_t* ucol, int32_t d_max, int pivot, int scheme, int32_t cap,
                  uint64_t* counts, int32_t* omega) {
    if (cap < 2 || (scheme != KCO_VC && scheme != KCO_EC)) return KCO_EINVAL;
    acc_t acc;
    memset(&acc, 0, sizeof acc);
    acc.cap = cap;
    acc.counts = (u128*)calloc((size_t)cap + 1, sizeof(u128));
    if (!acc.counts) return KCO_ENOMEM;
    int st = run(n, optr, ocol, uptr, ucol, d_max, 0, pivot, scheme, MODE_ALL, NULL, 0, &acc);
    acc.counts[0] = 1;
    acc.counts[1] = (u128)n;
    acc.counts[2] = (u128)optr[n];
    int32_t om = n > 0 ? 1 : 0;
    for (int32_t j = 0; j <= cap; j++) {
        counts[2 * j] = (uint64_t)acc.counts[j];
        counts[2 * j + 1] = (uint64_t)(acc.counts[j] >> 64);
        if (j > 0 && acc.counts[j] != 0) om = j;
    }
    *omega = om;
    free(acc.counts);
    if (st) return st;
    return acc.overflow ? KCO_EOVERFLOW : KCO_OK;
}

/* local[v] = number of k-cliques containing v (lo/hi pairs, 2n u64). */
int kco_count_local(int32_t n, const int32_t* optr, const int32_t* ocol, const int32_t* uptr,
                    const int32_t* ucol, int32_t d_max, int32_t k, int pivot, int scheme,
                    uint64_t* local) {
    if (k < 1 || (scheme != KCO_VC && scheme != KCO_EC)) return KCO_EINVAL;
    acc_t acc;
    memset(&acc, 0, sizeof acc);
    acc.local = (u128*)calloc((size_t)(n ? n : 1), sizeof(u128));
    if (!acc.local) return KCO_ENOMEM;
    int st = KCO_OK;
    if (k == 1) {
        for (int32_t v = 0; v < n; v++) acc.local[v] = 1;
    } else if (k == 2) {
        for (int32_t v = 0; v < n; v++) acc.local[v] = (u128)(uptr[v + 1] - uptr[v]);
    } else {
        st = run(n, optr, ocol, uptr, ucol, d_max, k, pivot, scheme, MODE_LOCAL, NULL, 0, &acc);
    }
    for (int32_t v = 0; v < n; v++) {
        local[2 * v] = (uint64_t)acc.local[v];
        local[2 * v + 1] = (uint64_t)(acc.local[v] >> 64);
    }
    free(acc.local);
    if (st) return st;
    return acc.overflow ? KCO_EOVERFLOW : KCO_OK;
}
