// k-clique counting by search-tree traversal over bitset-encoded induced
// sub-graphs (paper Sec. 2.2 Fig. 2, Sec. 3.2 - 3.6), for gfx950 wave64.
//
// Work distribution (Sec. 3.2, 3.6): persistent workgroups pull roots from a
// device work queue.  A root is a vertex u (vertex-centric, VC) or a DAG edge
// u->v (edge-centric, EC).  Roots are split by the size bound of their candidate
// set S into a light list (|S| <= 64: one wavefront per root) and a heavy list
// (one 4-wavefront workgroup per root); roots whose S cannot hold k - |path|
// vertices are dropped.
//
// Extraction (Sec. 2.4, 3.4): S = N+(u) (VC) or N+(u) cap N+(v) (EC), kept
// sorted, so with the DAG's order-relabelled ids bit j of row i means S[j] is an
// out-neighbour of S[i], and only j > i can be set (upper-triangular rows).  Row
// bits come from binary searches of each out-neighbour in S (the paper's
// binary-search intersections).
//
// Traversal (Fig. 2 with the intra-block split of Sec. 3.2 and sub-warp groups
// of Sec. 3.5): the lanes of a wavefront form groups of G lanes; a group owns one
// subtree at a time (task i = the branch through S[i]), taken dynamically from an
// LDS counter, and walks it depth-first with an explicit stack (Sec. 3.3).  Each
// lane holds words glane, glane + G, ... of the current level's remaining set R.
// One step: the lowest set bit v of R is found with a ballot and one bpermute,
// cleared, and Y = R & B[v] is formed.  Because rows are upper triangular,
// R & B[v] (R holding only bits above v) equals I cap Adj(v) of Fig. 2.  At the
// last level the step adds popcount(Y); otherwise a non-empty Y is pushed.
// Every lane keeps its own 64-bit partial count; wavefronts reduce them exactly
// into a 128-bit device counter when they exit.
#include <climits>
#include <mutex>
#include <new>

#include "kc_extract.h"
#include "kc_count_impl.h"

namespace kc {
namespace {

constexpr int kBlock = 256;
constexpr int kWavesPerBlock = kBlock / 64;

struct GoParams {
    int n, m, k;
    const int* __restrict__ row_ptr;
    const int* __restrict__ col;
    const int* __restrict__ src;
    const int* __restrict__ roots;   // root ids of this list
    const int* __restrict__ nroots;  // device count of this list
    int* head;                       // device queue head of this list
    unsigned long long* acc;         // [lo, hi]
    unsigned long long* stats;       // [nodes, word_ops] (stats variant only)
    int s_cap;                       // LDS rows per team
    int levels;                      // stack levels per group
    int* flags;                      // CC_FLAGS word (kFlagCanceled)
    const int* cancel;               // caller's cancel flag (null: none)
    unsigned long long* gacc;        // batched: per-graph {lo, hi}; null otherwise
    const int* gid;                  // batched: graph of each DAG vertex
    const int* list_counts;          // batched: sizes of the width lists (roots = the lists back to back)
    int list_index;                  // batched: the width list this launch walks
};

__device__ __forceinline__ int ffs64(unsigned long long x) { return __ffsll(static_cast<long long>(x)) - 1; }

// Sizes of the per-team LDS regions, in 32-bit words.
struct TeamLayout {
    int s_words, b_stride, b_words, stack_words, total;
};

__host__ __device__ inline TeamLayout team_layout(int s_cap, int maxw, int groups, int levels) {
    TeamLayout t;
    t.s_words = s_cap;
    t.b_stride = b_stride_of(maxw);
    t.b_words = s_cap * t.b_stride;
    t.stack_words = groups * levels * maxw;
    t.total = 8 + t.s_words + t.b_words + t.stack_words;
    return t;
}

// ------------------------------------------------------------ classify

// Split roots into light / heavy lists by the bound on |S|; drop roots whose
// bound is below `need` (a k-clique needs |S| >= k - 1 for VC, >= k - 2 for EC).
template <bool EC>
__global__ void __launch_bounds__(kBlock) k_classify(int nroots_total, int need, const int* __restrict__ row_ptr,
                                                    const int* __restrict__ col, const int* __restrict__ src,
                                                    int* light, int* heavy, int* ctl) {
    const int lane = threadIdx.x & 63;
    for (int base = blockIdx.x * blockDim.x; base < nroots_total; base += gridDim.x * blockDim.x) {
        int r = base + threadIdx.x;
        int bound = -1;
        if (r < nroots_total) {
            if (EC) {
                int u = src[r], v = col[r];
                int du = row_ptr[u + 1] - row_ptr[u] - 1;
                int dv = row_ptr[v + 1] - row_ptr[v];
                bound = du < dv ? du : dv;
                if (du >= KC_MAX_DMAX) bound = -1;   // a wide root
            } else {
                bound = row_ptr[r + 1] - row_ptr[r];
                if (bound > KC_MAX_DMAX) bound = -1;                          // a wide root
            }
        }
        bool ok = r < nroots_total && bound >= need && bound >= 0;
        bool is_light = ok && bound <= kLightCap;
        bool is_heavy = ok && bound > kLightCap;
        unsigned long long ml = __ballot(is_light), mh = __ballot(is_heavy);
        int bl = 0, bh = 0;
        if (lane == 0) {
            if (ml) bl = atomicAdd(&ctl[CC_LIGHT_N], __popcll(ml));
            if (mh) bh = atomicAdd(&ctl[CC_HEAVY_N], __popcll(mh));
        }
        bl = __shfl(bl, 0);
        bh = __shfl(bh, 0);
        if (is_light) light[bl + __popcll(ml & lanemask_lt())] = r;
        if (is_heavy) heavy[bh + __popcll(mh & lanemask_lt())] = r;
    }
}

// Width lists: root r goes to list w when its |S| needs 2^w words per bitset
// row (1, 2, 4, 8, 16 or 32); pass 1 counts, pass 2 appends into consecutive
// segments of one array (the order inside a list is unspecified).
__device__ __forceinline__ int width_list(int bound) {
    return bound <= 32 ? 0 : bound <= 64 ? 1 : bound <= 128 ? 2 : bound <= 256 ? 3 : bound <= 512 ? 4 : 5;
}

// |S| of root r: |N+(u)| for a vertex root; for the edge root (u, v) the size
// of N+(u) ∩ N+(v), counted exactly (rows are ascending, and every common
// vertex lies after v in the row of u).  Sizes below `need` are only bounded.
// Wide roots (first vertex with more than KC_MAX_DMAX out-neighbours) give -1.
template <bool EC>
__device__ __forceinline__ int root_size(int r, int need, const int* __restrict__ row_ptr,
                                         const int* __restrict__ col, const int* __restrict__ src) {
    if (!EC) {
        const int s = row_ptr[r + 1] - row_ptr[r];
        return s > KC_MAX_DMAX ? -1 : s;
    }
    const int u = src[r], v = col[r];
    if (row_ptr[u + 1] - row_ptr[u] > KC_MAX_DMAX) return -1;
    const int a0 = r + 1, na = row_ptr[u + 1] - a0;
    const int b0 = row_ptr[v], nb = row_ptr[v + 1] - b0;
    if (na < need || nb < need) return na < nb ? na : nb;
    const int* x = col + (na <= nb ? a0 : b0);          // shorter row: probes
    const int* y = col + (na <= nb ? b0 : a0);          // longer row: searched
    const int nx = na <= nb ? na : nb, ny = na <= nb ? nb : na;
    int c = 0, lo = 0;
    for (int i = 0; i < nx && lo < ny; i++) {
        const int t = x[i];
        int hi = ny;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (y[mid] < t) lo = mid + 1; else hi = mid;
        }
        if (lo < ny && y[lo] == t) c++;
    }
    return c;
}

// Exact |S| of every edge root (u, v), one wavefront per source vertex u: the
// row N+(u) is staged in LDS, then four 16-lane groups take the row's edges in
// turn; a group reads N+(v) coalesced and binary-searches each entry in the tail
// of N+(u) past v.  lst_of[r] gets the root's width list (-1 when |S| < need,
// and for the wide roots of rows longer than KC_MAX_DMAX); the list sizes go to
// ctl[CC_WN0 + j].  cap >= the longest DAG row up to KC_MAX_DMAX.
constexpr int kSizeWaves = 4;   // wavefronts per block
__global__ void __launch_bounds__(64 * kSizeWaves) k_sizes_ec(int n, int need, const int* __restrict__ row_ptr,
                                                             const int* __restrict__ col,
                                                             const int* __restrict__ src, int* lst_of, int* ctl,
                                                             int cap) {
    extern __shared__ int su_all[];
    const int lane = threadIdx.x & 63;
    int* su = su_all + (threadIdx.x >> 6) * cap;
    const int g = lane >> 4, gl = lane & 15;
    const unsigned long long gmask = 0xFFFFull << (16 * g);
    int cnt[kWidthLists];
#pragma unroll
    for (int q = 0; q < kWidthLists; q++) cnt[q] = 0;
    const int nw = gridDim.x * kSizeWaves;
    for (int u = blockIdx.x * kSizeWaves + static_cast<int>(threadIdx.x >> 6); u < n; u += nw) {
        const int b = row_ptr[u], du = row_ptr[u + 1] - b;
        if (du == 0) continue;
        if (du > KC_MAX_DMAX) {
            for (int i = lane; i < du; i += 64) lst_of[b + i] = -1;   // wide roots
            continue;
        }
        if (du > cap) {
            // a row longer than the stated d_max: per-edge search in global memory
            for (int i = lane; i < du; i += 64) {
                const int size = root_size<true>(b + i, need, row_ptr, col, src);
                const int lst = size >= need ? width_list(size) : -1;
#pragma unroll
                for (int q = 0; q < kWidthLists; q++) cnt[q] += lst == q;
                lst_of[b + i] = lst;
            }
            continue;
        }
        for (int i = lane; i < du; i += 64) su[i] = col[b + i];
        wave_sync_lds();
        for (int j0 = 0; j0 < du; j0 += 4) {
            const int j = j0 + g;
            bool live = j < du;
            int vb = 0, len = 0;
            if (live) {
                const int v = su[j];
                vb = row_ptr[v];
                len = row_ptr[v + 1] - vb;
                if (du - j - 1 < need || len < need) live = false;
            }
            if (!live) len = 0;
            // rounds of 16 entries of N+(v) per group, as many as the longest row
            const int rounds = wave_max(len);
            int hits = 0;
            for (int t0 = 0; t0 < rounds; t0 += 16) {
                const int t = t0 + gl;
                bool hit = false;
                if (t < len) {
                    const int x = col[vb + t];
                    int lo = j + 1, hi = du;
                    while (lo < hi) {
                        const int mid = (lo + hi) >> 1;
                        if (su[mid] < x) lo = mid + 1; else hi = mid;
                    }
                    hit = lo < du && su[lo] == x;
                }
                hits += __popcll(__ballot(hit) & gmask);
            }
            if (gl == 0 && j < du) {
                const int lst = live && hits >= need ? width_list(hits) : -1;
#pragma unroll
                for (int q = 0; q < kWidthLists; q++) cnt[q] += lst == q;
                lst_of[b + j] = lst;
            }
        }
        wave_sync_lds();
    }
#pragma unroll
    for (int q = 0; q < kWidthLists; q++) {
        const int tot = wave_sum(cnt[q]);
        if (lane == 0 && tot) atomicAdd(&ctl[CC_WN0 + q], tot);
    }
}

template <bool EC, bool FILL>
__global__ void __launch_bounds__(kBlock) k_classify_w(int nroots_total, int need, const int* __restrict__ row_ptr,
                                                      const int* __restrict__ col, const int* __restrict__ src,
                                                      int* lists, int* ctl, int* lst_of) {
    const int lane = threadIdx.x & 63;
    int off[kWidthLists];
    if (FILL) {
        int run = 0;
        for (int j = 0; j < kWidthLists; j++) {
            off[j] = run;
            run += ctl[CC_WN0 + j];
        }
    }
    for (int base = blockIdx.x * blockDim.x; base < nroots_total; base += gridDim.x * blockDim.x) {
        const int r = base + threadIdx.x;
        int lst = -1;
        if (r < nroots_total) {
            if (FILL) {
                lst = lst_of[r];                    // from the counting pass
            } else {
                const int size = root_size<EC>(r, need, row_ptr, col, src);
                if (size >= need && size >= 0) lst = width_list(size);
                lst_of[r] = lst;
            }
        }
        for (int j = 0; j < kWidthLists; j++) {
            const unsigned long long m = __ballot(lst == j);
            if (m == 0ull) continue;
            int b = 0;
            if (lane == 0) b = atomicAdd(&ctl[(FILL ? CC_WC0 : CC_WN0) + j], __popcll(m));
            b = __shfl(b, 0);
            if (FILL && lst == j) lists[off[j] + b + __popcll(m & lanemask_lt())] = r;
        }
    }
}

// ------------------------------------------------------------- traversal

// G: lanes per group; MAXW: bitset words per row this instantiation handles;
// TW: wavefronts per team (1 = wave per root, 4 = workgroup per root);
// STATS: also count expanded nodes and their bitset words (measurement only).
template <int G, int MAXW, int TW, bool EC, bool STATS>
__global__ void __launch_bounds__(kBlock) k_go(GoParams P) {
    static_assert(G >= 1 && G <= 64 && (G & (G - 1)) == 0, "group size");
    constexpr int WPL = (MAXW + G - 1) / G;             // words per lane
    constexpr int TEAM_LANES = 64 * TW;
    constexpr int GROUPS = TEAM_LANES / G;              // groups per team
    extern __shared__ unsigned int lds[];

    const int lane = threadIdx.x & 63;
    const int team = threadIdx.x / TEAM_LANES;
    const int tl = threadIdx.x % TEAM_LANES;            // lane within team
    const int glane = lane & (G - 1);
    const int gbase = lane & ~(G - 1);
    const int group = tl / G;
    const unsigned long long gmask = G == 64 ? ~0ull : (((1ull << G) - 1ull) << gbase);

    const TeamLayout L = team_layout(P.s_cap, MAXW, GROUPS, P.levels);
    unsigned int* tbase = lds + team * L.total;
    int* ctl = reinterpret_cast<int*>(tbase);           // [0] task ctr, [1] s, [2] root
    int* S = reinterpret_cast<int*>(tbase + 8);
    unsigned int* B = tbase + 8 + L.s_words;
    unsigned int* stack = B + L.b_words + group * P.levels * MAXW;
    const int stride = L.b_stride;
    const int k = P.k;
    const int p0 = EC ? 3 : 2;                          // path length of a task's root branch
    const int* roots = P.roots;
    int nroots = *P.nroots;
    if (P.list_counts) {
        // one width list of lists stored back to back: its offset is the sum of
        // the sizes before it
        int off = 0;
        for (int j = 0; j < P.list_index; j++) off += P.list_counts[j];
        roots += off;
        nroots = P.list_counts[P.list_index];
    }

    unsigned long long acc = 0;
    unsigned long long st_nodes = 0, st_words = 0;

    for (;;) {
        // ---- fetch a root (none once the caller asked to cancel)
        if (tl == 0) {
            int r = atomicAdd(P.head, 1);
            if (P.cancel && r < nroots && cancel_requested(P.cancel)) {
                atomicOr(P.flags, kFlagCanceled);
                r = nroots;
            }
            ctl[2] = r;
        }
        team_sync<TW>();
        const int root = ctl[2];
        if (root >= nroots) break;
        const int rid = roots[root];
        // batched: every lane adds this root's partial count to the root's graph
        auto flush_graph = [&]() {
            if (P.gacc) {
                if (acc) {
                    const int g = P.gid[EC ? P.src[rid] : rid];
                    atomic_add_u128(P.gacc + 2 * g, P.gacc + 2 * g + 1, acc, 0ull);
                }
                acc = 0;
            }
        };

        // ---- candidate set S (sorted) and bitset rows B[i] (bit j <=> S[j] in N+(S[i]))
        extract_set<TW, EC>(rid, P.row_ptr, P.col, P.src, tl, S, &ctl[1]);
        const int s = ctl[1];
        if (EC && k == 3) {
            // every vertex of S closes a triangle with the root edge
            if (tl == 0) acc += static_cast<unsigned long long>(s);
            flush_graph();
            team_sync<TW>();
            continue;
        }
        if (tl == 0) ctl[0] = 0;
        extract_rows<TW, false>(s, P.row_ptr, P.col, tl, S, B, stride);

        // ---- traversal: groups take subtrees (tasks i = 0..s-1) dynamically
        unsigned int R[WPL];
#pragma unroll
        for (int t = 0; t < WPL; t++) R[t] = 0u;
        int depth = 0, p = p0;
        bool done = false;
        for (;;) {
            bool my_any = false;
#pragma unroll
            for (int t = 0; t < WPL; t++) my_any |= R[t] != 0u;
            const bool has = (__ballot(my_any) & gmask) != 0ull;
            const bool need = !has && !done;
            const bool fetch = need && depth == 0;
            if (need && depth > 0) {
                // pop
                depth--;
                p--;
#pragma unroll
                for (int t = 0; t < WPL; t++) {
                    const int wd = glane + t * G;
                    R[t] = wd < MAXW ? stack[depth * MAXW + wd] : 0u;
                }
            }
            int task = 0;
            if (fetch && glane == 0) task = atomicAdd(&ctl[0], 1);
            task = __shfl(task, gbase);
            if (fetch) {
                if (task < s) {
                    p = p0;
                    unsigned int c = 0;
#pragma unroll
                    for (int t = 0; t < WPL; t++) {
                        const int wd = glane + t * G;
                        R[t] = wd < MAXW ? B[task * stride + wd] : 0u;
                        c += __popc(R[t]);
                    }
                    if (p0 + 1 == k) {
                        acc += c;
#pragma unroll
                        for (int t = 0; t < WPL; t++) R[t] = 0u;
                    }
                } else {
                    done = true;
                }
            }
            if (__ballot(!done) == 0ull) break;
            if (!has) continue;   // popped or fetched: re-evaluate next step

            // ---- expand: lowest set bit of R over the group
            int tsel = WPL;
            int owner = gbase;
#pragma unroll
            for (int t = WPL - 1; t >= 0; t--) {
                const unsigned long long bt = __ballot(R[t] != 0u) & gmask;
                if (bt) { tsel = t; owner = ffs64(bt); }
            }
            unsigned int mine = 0u;
#pragma unroll
            for (int t = 0; t < WPL; t++) mine = (t == tsel) ? R[t] : mine;
            const unsigned int wv = static_cast<unsigned int>(__shfl(static_cast<int>(mine), owner));
            const int v = ((owner - gbase) + tsel * G) * 32 + (__ffs(wv) - 1);
            if (STATS && glane == 0) {
                st_nodes += 1;
                st_words += static_cast<unsigned long long>((s + 31) >> 5);
            }
            if (lane == owner) {
#pragma unroll
                for (int t = 0; t < WPL; t++)
                    if (t == tsel) R[t] &= R[t] - 1u;
            }
            unsigned int Y[WPL];
            bool y_any = false;
            unsigned int c = 0;
#pragma unroll
            for (int t = 0; t < WPL; t++) {
                const int wd = glane + t * G;
                Y[t] = (wd < MAXW && R[t]) ? (R[t] & B[v * stride + wd]) : 0u;
                y_any |= Y[t] != 0u;
                c += __popc(Y[t]);
            }
            if (p + 2 == k) {
                acc += c;
            } else {
                const bool push = (__ballot(y_any) & gmask) != 0ull;
                if (push) {
#pragma unroll
                    for (int t = 0; t < WPL; t++) {
                        const int wd = glane + t * G;
                        if (wd < MAXW) stack[depth * MAXW + wd] = R[t];
                        R[t] = Y[t];
                    }
                    depth++;
                    p++;
                }
            }
        }
        flush_graph();
        team_sync<TW>();
    }

    unsigned long long lo, hi;
    wave_sum_u128(acc, lo, hi);
    if (lane == 0) atomic_add_u128(P.acc, P.acc + 1, lo, hi);
    if (STATS) {
        st_nodes = wave_sum(st_nodes);
        st_words = wave_sum(st_words);
        if (lane == 0) {
            atomicAdd(P.stats, st_nodes);
            atomicAdd(P.stats + 1, st_words);
        }
    }
}

// --------------------------------------------------------------- launch

int levels_for(int k, bool ec) {
    const int p0 = ec ? 3 : 2;
    int lv = k - 2 - p0;
    return lv < 1 ? 1 : lv;
}

template <int G, int MAXW, int TW, bool EC>
int launch_go(const GoParams& base, int s_cap, bool stats, hipStream_t s) {
    constexpr int TEAMS = kWavesPerBlock / TW;
    constexpr int GROUPS = 64 * TW / G;
    GoParams P = base;
    P.s_cap = s_cap;
    P.levels = levels_for(P.k, EC);
    const TeamLayout L = team_layout(s_cap, MAXW, GROUPS, P.levels);
    const size_t lds_bytes = static_cast<size_t>(L.total) * TEAMS * sizeof(unsigned int);
    if (lds_bytes > 160 * 1024) return KC_EUNSUPPORTED;
    auto kern = stats ? k_go<G, MAXW, TW, EC, true> : k_go<G, MAXW, TW, EC, false>;
    if (lds_bytes > 64 * 1024)
        KC_CHECK(hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds_bytes)));
    int occ = 0;
    KC_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, kBlock, lds_bytes));
    if (occ < 1) return KC_EUNSUPPORTED;
    const int blocks = device_cus() * occ;
    kern<<<blocks, kBlock, lds_bytes, s>>>(P);
    KC_CHECK(hipGetLastError());
    return KC_OK;
}

template <bool EC>
int launch_light(const GoParams& P, int width, bool st, hipStream_t s) {
    switch (width) {
        case 1: return launch_go<1, 2, 1, EC>(P, kLightCap, st, s);
        case 2: return launch_go<2, 2, 1, EC>(P, kLightCap, st, s);
        case 4: return launch_go<4, 2, 1, EC>(P, kLightCap, st, s);
        case 8: return launch_go<8, 2, 1, EC>(P, kLightCap, st, s);
        default: return KC_EINVAL;
    }
}

template <bool EC, int MAXW>
int launch_heavy_w(const GoParams& P, int width, int s_cap, bool st, hipStream_t s) {
    switch (width) {
        case 4: return launch_go<4, MAXW, 4, EC>(P, s_cap, st, s);
        case 8: return launch_go<8, MAXW, 4, EC>(P, s_cap, st, s);
        case 16: return launch_go<16, MAXW, 4, EC>(P, s_cap, st, s);
        case 32: return launch_go<32, MAXW, 4, EC>(P, s_cap, st, s);
        default: return KC_EINVAL;
    }
}

template <bool EC>
int launch_heavy(const GoParams& P, int width, int d_max, bool st, hipStream_t s) {
    const int s_cap = ((d_max + 31) / 32) * 32;
    if (d_max <= 128) return launch_heavy_w<EC, 4>(P, width, s_cap, st, s);
    if (d_max <= 256) return launch_heavy_w<EC, 8>(P, width, s_cap, st, s);
    if (d_max <= 512) return launch_heavy_w<EC, 16>(P, width, s_cap, st, s);
    return launch_heavy_w<EC, 32>(P, width, s_cap, st, s);
}

}  // namespace

// Sub-wavefront group walk over one width list of a batched call (groups of
// `group` lanes; lists 0 and 1 run a wavefront per root with at most 8 lanes
// per group, wider lists a 4-wavefront team per root with at least 4).
int go_batch_launch(const GoBatchLaunch& B, hipStream_t s) {
    GoParams P;
    P.n = 0;
    P.m = 0;
    P.k = B.k;
    P.row_ptr = B.row_ptr;
    P.col = B.col;
    P.src = B.src;
    P.roots = B.lists;
    P.nroots = B.list_counts + B.list;
    P.head = B.head;
    P.acc = B.acc;
    P.stats = B.acc + 2;
    P.s_cap = 0;
    P.levels = 0;
    P.flags = B.flags;
    P.cancel = nullptr;
    P.gacc = B.gacc;
    P.gid = B.gid;
    P.list_counts = B.list_counts;
    P.list_index = B.list;
    if (B.list <= 1) {
        const int g = B.group <= 2 ? 2 : B.group <= 4 ? 4 : 8;
        return B.ec ? launch_light<true>(P, g, false, s) : launch_light<false>(P, g, false, s);
    }
    const int g = B.group <= 4 ? 4 : B.group <= 8 ? 8 : B.group <= 16 ? 16 : 32;
    const int s_cap = 32 << B.list;
    return B.ec ? launch_heavy<true>(P, g, s_cap, false, s) : launch_heavy<false>(P, g, s_cap, false, s);
}

namespace {

bool valid_dag(const kc_dag* d) {
    if (!d || d->n < 0 || d->m < 0 || d->d_max < 0) return false;
    if (!d->row_ptr) return false;
    if (d->m > 0 && (!d->col || !d->src)) return false;
    return true;
}

int pick_scheme(const kc_opts* o, int k) {
    int sc = o ? o->scheme : KC_SCHEME_AUTO;
    if (sc == KC_SCHEME_AUTO) sc = k < 6 ? KC_SCHEME_VC : KC_SCHEME_EC;   // Sec. 4.5 guideline
    return sc;
}

int pick_width(const kc_opts* o, int d_max, bool light) {
    int w = o ? o->width : 0;
    if (w == 0) {
        if (light) return 2;
        return d_max < 200 ? 4 : 8;   // Sec. 4.5: small groups for small d_max, 8 otherwise
    }
    return w;
}

// Classify roots, run the light and heavy kernels of one traversal, and read
// the results back.  `pivot_all` selects the pivot kernels (-1: graph
// orientation, 0: pivot with target k, 1: pivot count-all, 2: pivot per-vertex
// counts of size k into local_out, which the caller has zeroed).
int run_count(const kc_dag* d, int k, int pivot_all, const kc_opts* o, const CountWs& w, bool ec,
              unsigned long long preload, unsigned long long res[kAccWords], int hctl[CC_WORDS],
              unsigned long long* counts_out, int counts_len, hipStream_t s,
              unsigned long long* local_out = nullptr) {
    kc_profile* prof = o ? o->profile : nullptr;
    const bool stats = o && o->collect_stats;
    // timing events for kc_profile: a set from the per-device pool for this call
    ProfileGuard pg;
    ProfileEvents* pe = nullptr;
    if (prof) {
        int st0 = profile_acquire(&pg.e);
        if (st0 != KC_OK) return st0;
        pg.held = true;
        pe = &pg.e;
        KC_CHECK(hipEventRecord(pe->ev[0], s));
    }
    const int nroots = ec ? d->m : d->n;
    const int dm = bit_dmax(d->d_max);   // the on-chip kernels never see a wide root
    KC_CHECK(hipMemsetAsync(w.ctl, 0, CC_WORDS * sizeof(int), s));
    unsigned long long init[kAccWords] = {};
    init[0] = preload;
    for (int j = 0; j < kWidthLists; j++) init[6 + 4 * kWidthLists + 3 * j + 1] = ~0ull;   // min start of each list's timing
    KC_CHECK(hipMemcpyAsync(w.acc, init, sizeof(init), hipMemcpyHostToDevice, s));
    if (pivot_all >= 0) {
        KC_CHECK(hipMemsetAsync(w.counts, 0, 2 * sizeof(unsigned long long) * w.counts_len, s));
        // frame queues of the light and the heavy launch
        KC_CHECK(hipMemsetAsync(w.qctl, 0, sizeof(int) * kQueueCtlWords * 2, s));
        KC_CHECK(hipMemsetAsync(w.qready, 0, sizeof(int) * kQueueCap * 2, s));
        int st0 = pivot_binom_table(w, s);
        if (st0 != KC_OK) return st0;
    }
    // roots that cannot reach the target size are dropped (count-all: cliques of
    // size >= 3 need |S| >= 2 under a vertex root, >= 1 under an edge root)
    const int need = pivot_all == 1 ? (ec ? 1 : 2) : (ec ? k - 2 : k - 1);
    int cblocks = div_up(nroots, kBlock);
    if (cblocks > device_cus() * 8) cblocks = device_cus() * 8;
    if (cblocks < 1) cblocks = 1;
    const bool lists = pivot_all < 0 && o && (o->flags & KC_OPT_NO_BITSETS);
    bool lane_path = pivot_all < 0 && !lists && (o ? o->width : 0) <= 1;
    if (lane_path) {
        // the widest list must fit one wavefront's LDS; otherwise use the group walk
        int top = 0;
        while (top < kWidthLists - 1 && (32 << top) < dm) top++;
        const bool deep = k >= (ec ? 3 : 2) + 4;
        if (lane_lds_bytes(1 << top, k, ec, deep && top >= 1) > 160 * 1024) lane_path = false;
    }
    if (lane_path) {
        KC_CHECK(hipMemsetAsync(w.active, 0xff, 2 * sizeof(int) * w.nactive, s));
        if (k >= (ec ? 3 : 2) + 4) {
            KC_CHECK(hipMemsetAsync(w.task_ctr, 0, sizeof(int) * static_cast<size_t>(nroots), s));
            KC_CHECK(hipMemsetAsync(w.task_tot, 0, sizeof(int) * static_cast<size_t>(nroots), s));
            KC_CHECK(hipMemsetAsync(w.qctl, 0, sizeof(int) * kQueueCtlWords * kWidthLists, s));
            KC_CHECK(hipMemsetAsync(w.qready, 0, sizeof(int) * kQueueCap * kWidthLists, s));
        }
        if (ec) {
            const int cap = dm > 1 ? dm : 1;
            int sblocks = div_up(d->n, kSizeWaves);
            if (sblocks > device_cus() * 8) sblocks = device_cus() * 8;
            if (sblocks < 1) sblocks = 1;
            k_sizes_ec<<<sblocks, 64 * kSizeWaves, kSizeWaves * cap * sizeof(int), s>>>(
                d->n, need, d->row_ptr, d->col, d->src, w.heavy, w.ctl, cap);
        } else {
            k_classify_w<false, false><<<cblocks, kBlock, 0, s>>>(nroots, need, d->row_ptr, d->col, d->src, w.light, w.ctl, w.heavy);
        }
    } else if (ec) {
        k_classify<true><<<cblocks, kBlock, 0, s>>>(nroots, need, d->row_ptr, d->col, d->src, w.light, w.heavy, w.ctl);
    } else {
        k_classify<false><<<cblocks, kBlock, 0, s>>>(nroots, need, d->row_ptr, d->col, d->src, w.light, w.heavy, w.ctl);
    }
    KC_CHECK(hipGetLastError());
    if (prof && !lane_path) KC_CHECK(hipEventRecord(pe->ev[1], s));

    int st = KC_OK;
    int lane_grid[kWidthLists] = {0, 0, 0, 0, 0, 0};
    if (lane_path) {
        // lane walks over the width lists, widest first so that the largest roots
        // start early; profile: heavy = lists with >= 4 words, light = 1-2 words
        if (ec)
            k_classify_w<true, true><<<cblocks, kBlock, 0, s>>>(nroots, need, d->row_ptr, d->col, d->src, w.light, w.ctl, w.heavy);
        else
            k_classify_w<false, true><<<cblocks, kBlock, 0, s>>>(nroots, need, d->row_ptr, d->col, d->src, w.light, w.ctl, w.heavy);
        KC_CHECK(hipGetLastError());
        if (prof) KC_CHECK(hipEventRecord(pe->ev[1], s));
        const int p0 = ec ? 3 : 2;
        const bool deep = k >= p0 + 4;
        int top = 0;
        while (top < kWidthLists - 1 && (32 << top) < dm) top++;
        // deep trees: the widest list runs on a side stream beside the others, so
        // that the tail of its few large roots overlaps their work
        SideGuard side;
        LaneLaunch side_launch;
        if (deep && top >= 1 && !(o && (o->flags & KC_OPT_SINGLE_STREAM))) {
            st = side_acquire(&side.s);
            if (st != KC_OK) return st;
            side.held = true;
            KC_CHECK(hipEventRecord(side.s.fork, s));
            KC_CHECK(hipStreamWaitEvent(side.s.stream, side.s.fork, 0));
        }
        for (int lst = top; lst >= 0; lst--) {
            const bool on_side = side.held && lst == top;
            hipStream_t ls = on_side ? side.s.stream : s;
            if (lst == 1 && prof) KC_CHECK(hipEventRecord(pe->ev[2], s));
            LaneLaunch L;
            L.k = k;
            L.ec = ec;
            L.pair = deep && lst >= 1;
            L.stats = stats;
            L.maxw = 1 << lst;
            L.list = lst;
            L.row_ptr = d->row_ptr;
            L.col = d->col;
            L.src = d->src;
            L.lists = w.light;
            L.counts = w.ctl + CC_WN0;
            L.head = w.ctl + CC_WH0 + lst;
            L.task_ctr = w.task_ctr;
            L.task_tot = w.task_tot;
            L.active = on_side ? w.active + w.nactive : w.active;
            L.acc = w.acc;
            L.stats_ptr = w.acc + 6 + 2 * lst;
            L.iters_ptr = w.acc + 6 + 2 * kWidthLists + 2 * lst;
            L.timing_ptr = w.acc + 6 + 4 * kWidthLists + 3 * lst;
            L.cwords_ptr = w.acc + kAccCwords + lst;
            L.steal = L.pair && !(o && (o->flags & KC_OPT_NO_HANDOFF));
            L.qctl = w.qctl + kQueueCtlWords * lst;
            L.qready = w.qready + static_cast<size_t>(kQueueCap) * lst;
            L.qitems = w.qitems + (on_side ? static_cast<size_t>(kQueueCap) * kItemWords : 0);
            L.flags = w.ctl + CC_FLAGS;
            if (o) {
                L.steal_every = o->handoff_every > 0 ? o->handoff_every : kLaneStealEvery;
                L.steal_after = o->handoff_after > 0 ? o->handoff_after : kLaneStealAfter;
                L.cancel = const_cast<const int*>(reinterpret_cast<const volatile int*>(o->cancel));
            }
            if (prof) KC_CHECK(hipEventRecord(pe->wl[2 * lst], ls));
            L.grid_out = &lane_grid[lst];
            if (on_side) side_launch = L;
            st = lane_launch(L, ls);
            if (st != KC_OK) return st;
            if (prof) KC_CHECK(hipEventRecord(pe->wl[2 * lst + 1], ls));
        }
        if (side.held) {
            // once the other lists are done, the rest of the device joins the
            // widest list's tail: helpers take pair tasks and queued subtrees
            LaneLaunch H = side_launch;
            H.helper = true;
            H.grid_out = nullptr;
            H.timing_ptr = w.acc + 6 + 7 * kWidthLists;   // not part of the list's busy fraction
            st = lane_launch(H, s);
            if (st != KC_OK) return st;
            KC_CHECK(hipEventRecord(side.s.join, side.s.stream));
            KC_CHECK(hipStreamWaitEvent(s, side.s.join, 0));
        }
        if (prof && top < 1) KC_CHECK(hipEventRecord(pe->ev[2], s));
        if (prof)
            for (int lst = top + 1; lst < kWidthLists; lst++) {   // unlaunched lists: zero-length spans
                KC_CHECK(hipEventRecord(pe->wl[2 * lst], s));
                KC_CHECK(hipEventRecord(pe->wl[2 * lst + 1], s));
            }
    } else if (lists) {
        st = lists_launch(d, k, ec, w, o->cancel ? const_cast<const int*>(reinterpret_cast<const volatile int*>(o->cancel))
                                                 : nullptr, s);
        if (st != KC_OK) return st;
        if (prof) KC_CHECK(hipEventRecord(pe->ev[2], s));
    } else if (pivot_all < 0) {
        GoParams P;
        P.n = d->n;
        P.m = d->m;
        P.k = k;
        P.row_ptr = d->row_ptr;
        P.col = d->col;
        P.src = d->src;
        P.acc = w.acc;
        P.stats = w.acc + 2;
        P.s_cap = 0;
        P.levels = 0;
        P.flags = w.ctl + CC_FLAGS;
        P.cancel = o ? const_cast<const int*>(reinterpret_cast<const volatile int*>(o->cancel)) : nullptr;
        P.roots = w.light;
        P.nroots = w.ctl + CC_LIGHT_N;
        P.head = w.ctl + CC_LIGHT_HEAD;
        P.gacc = nullptr;
        P.gid = nullptr;
        P.list_counts = nullptr;
        P.list_index = 0;
        int lw = pick_width(o, dm, true);
        if (lw > 8) lw = 8;
        st = ec ? launch_light<true>(P, lw, stats, s) : launch_light<false>(P, lw, stats, s);
        if (st != KC_OK) return st;
        if (prof) KC_CHECK(hipEventRecord(pe->ev[2], s));
        if (dm > kLightCap) {
            P.roots = w.heavy;
            P.nroots = w.ctl + CC_HEAVY_N;
            P.head = w.ctl + CC_HEAVY_HEAD;
            P.stats = w.acc + 4;
            int wd = pick_width(o, dm, false);
            if (wd < 4) wd = 4;
            st = ec ? launch_heavy<true>(P, wd, dm, stats, s) : launch_heavy<false>(P, wd, dm, stats, s);
            if (st != KC_OK) return st;
        }
    } else {
        PivLaunch L;
        L.k = k;
        L.all = pivot_all == 1;
        if (pivot_all == 2) {
            L.local = local_out;
            L.perm = d->perm;
        }
        L.ec = ec;
        L.stats = stats;
        L.steal = !(o && (o->flags & KC_OPT_NO_HANDOFF));
        if (o) {
            L.steal_every = o->handoff_every > 0 ? o->handoff_every : 0;
            L.steal_after = o->handoff_after > 0 ? o->handoff_after : 0;
            L.cancel = const_cast<const int*>(reinterpret_cast<const volatile int*>(o->cancel));
        }
        L.d_max = dm;
        L.row_ptr = d->row_ptr;
        L.col = d->col;
        L.src = d->src;
        L.w = w;
        st = pivot_launch(L, false, s);
        if (st != KC_OK) return st;
        if (prof) KC_CHECK(hipEventRecord(pe->ev[2], s));
        if (dm > kLightCap) {
            st = pivot_launch(L, true, s);
            if (st != KC_OK) return st;
        }
    }
    if (d->d_max > KC_MAX_DMAX && !lists && pivot_all != 2) {
        // wide roots, after the others on the caller's stream
        const int* cancel = o ? const_cast<const int*>(reinterpret_cast<const volatile int*>(o->cancel)) : nullptr;
        st = wide_launch(d, k, pivot_all < 0 ? 0 : pivot_all == 0 ? 1 : 2, w, cancel, s);
        if (st != KC_OK) return st;
    }
    if (prof) {
        if (!lane_path && dm <= kLightCap) KC_CHECK(hipEventRecord(pe->ev[2], s));
        KC_CHECK(hipEventRecord(pe->ev[3], s));
    }
    KC_CHECK(hipMemcpyAsync(res, w.acc, kAccWords * sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
    KC_CHECK(hipMemcpyAsync(hctl, w.ctl, CC_WORDS * sizeof(int), hipMemcpyDeviceToHost, s));
    int hq[kQueueCtlWords * kWidthLists] = {};
    const bool queued = lane_path && k >= (ec ? 3 : 2) + 4;
    if (prof && queued)
        KC_CHECK(hipMemcpyAsync(hq, w.qctl, sizeof(hq), hipMemcpyDeviceToHost, s));
    if (counts_out)
        KC_CHECK(hipMemcpyAsync(counts_out, w.counts, 2 * sizeof(unsigned long long) * counts_len,
                                hipMemcpyDeviceToHost, s));
    KC_CHECK(hipStreamSynchronize(s));
    if (prof) {
        KC_CHECK(hipEventElapsedTime(&prof->ms_classify, pe->ev[0], pe->ev[1]));
        if (lane_path) {   // heavy lists run first
            KC_CHECK(hipEventElapsedTime(&prof->ms_heavy, pe->ev[1], pe->ev[2]));
            KC_CHECK(hipEventElapsedTime(&prof->ms_light, pe->ev[2], pe->ev[3]));
        } else {
            KC_CHECK(hipEventElapsedTime(&prof->ms_light, pe->ev[1], pe->ev[2]));
            KC_CHECK(hipEventElapsedTime(&prof->ms_heavy, pe->ev[2], pe->ev[3]));
        }
        KC_CHECK(hipEventElapsedTime(&prof->ms_total, pe->ev[0], pe->ev[3]));
        for (int i = 0; i < 2; i++) {
            prof->nodes[i] = stats ? res[2 + 2 * i] : 0;
            prof->word_ops[i] = stats ? res[3 + 2 * i] : 0;
        }
        for (int j = 0; j < kWidthLists; j++) {
            prof->ms_width[j] = 0.f;
            prof->roots_width[j] = lane_path ? hctl[CC_WN0 + j] : 0;
            prof->waves_width[j] = lane_path ? lane_grid[j] : 0;
            prof->nodes_width[j] = lane_path && stats ? res[6 + 2 * j] : 0;
            prof->words_width[j] = lane_path && stats ? res[7 + 2 * j] : 0;
            prof->iters_width[j] = lane_path && stats ? res[6 + 2 * kWidthLists + 2 * j] : 0;
            prof->items_width[j] = queued ? hq[kQueueCtlWords * j + 1] : 0;   // queue tail
            prof->expand_width[j] = lane_path && stats ? res[7 + 2 * kWidthLists + 2 * j] : 0;
            prof->cwords_width[j] = lane_path && stats ? res[kAccCwords + j] : 0;
            {
                const unsigned long long* tm = res + 6 + 4 * kWidthLists + 3 * j;
                const double span = tm[2] > tm[1] && tm[1] != ~0ull ? static_cast<double>(tm[2] - tm[1]) : 0.0;
                prof->busy_width[j] = lane_path && stats && span > 0 && prof->waves_width[j] > 0
                                          ? static_cast<float>(static_cast<double>(tm[0]) / (span * prof->waves_width[j]))
                                          : 0.f;
            }
            if (lane_path) KC_CHECK(hipEventElapsedTime(&prof->ms_width[j], pe->wl[2 * j], pe->wl[2 * j + 1]));
        }
        if (lane_path) {
            prof->light_roots = hctl[CC_WN0] + hctl[CC_WN0 + 1];
            prof->heavy_roots = 0;
            for (int j = 2; j < kWidthLists; j++) prof->heavy_roots += hctl[CC_WN0 + j];
            for (int i = 0; i < 2; i++) {
                prof->nodes[i] = 0;
                prof->word_ops[i] = 0;
            }
            for (int j = 0; j < kWidthLists; j++) {
                prof->nodes[j >= 2] += prof->nodes_width[j];
                prof->word_ops[j >= 2] += prof->words_width[j];
            }
        } else {
            prof->light_roots = hctl[CC_LIGHT_N];
            prof->heavy_roots = hctl[CC_HEAVY_N];
        }
    }
    return KC_OK;
}

}  // namespace

size_t device_lds_bytes() {
    int dev = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&per_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) != hipSuccess ||
        per_cu <= 0)
        per_cu = 160 * 1024;
    return static_cast<size_t>(device_cus()) * static_cast<size_t>(per_cu);
}

size_t count_lds_demand(const kc_dag* d, int k, int pivot) {
    if (!d || k < 3 || d->m <= 0 || k > d->d_max + 1) return 0;
    const int dm = bit_dmax(d->d_max);
    const bool ec = pick_scheme(nullptr, k) == KC_SCHEME_EC;
    const long long roots = ec ? d->m : d->n;
    size_t per_wave = 0;
    long long waves = 0;
    if (!pivot) {
        int top = 0;
        while (top < kWidthLists - 1 && (32 << top) < dm) top++;
        const bool deep = k >= (ec ? 3 : 2) + 4;
        per_wave = lane_lds_bytes(1 << top, k, ec, deep && top >= 1);
        waves = static_cast<long long>(device_cus()) * kLaneWavesPerCU;
    } else {
        const int s_cap = s_cap_for(dm), maxw = maxw_for(dm);
        per_wave = static_cast<size_t>(8 + s_cap + s_cap * b_stride_of(maxw)) * 4;
        waves = static_cast<long long>(device_cus()) * kPivBlocksPerCU;
    }
    if (roots < waves) waves = roots;
    const size_t total = per_wave * static_cast<size_t>(waves);
    const size_t cap = device_lds_bytes();
    return total < cap ? total : cap;
}

}  // namespace kc

using namespace kc;

extern "C" KC_API size_t kc_count_workspace(const kc_dag* d, int32_t k, int32_t pivot, const kc_opts* o) {
    (void)k;
    (void)o;
    if (!d || d->n < 0 || d->m < 0 || d->d_max < 0) return 0;
    size_t bytes = 0;
    carve_count(nullptr, d, pivot != 0, &bytes);
    return bytes;
}

namespace kc {
namespace {

// kc_count's body over a workspace the caller (or the fixed scratch array)
// provides.
int count_with_ws(const kc_dag* d, int32_t k, int32_t pivot, kc_u128* count, void* ws, size_t ws_bytes,
                  const kc_opts* o, hipStream_t s) {
    if (!valid_dag(d) || !count || k < 1) return KC_EINVAL;
    count->lo = count->hi = 0;
    const unsigned long long preload = o ? o->test_preload : 0ull;
    if (k == 1 || k == 2) {
        unsigned long long v = (k == 1 ? static_cast<unsigned long long>(d->n) : static_cast<unsigned long long>(d->m));
        unsigned long long sum = v + preload;
        count->lo = sum;
        count->hi = sum < v ? 1ull : 0ull;
        if (!pivot && count->hi) { count->hi = 0; return KC_EOVERFLOW; }
        return KC_OK;
    }
    if (d->d_max > KC_MAX_DMAX_WIDE) return KC_EUNSUPPORTED;
    size_t need = 0;
    CountWs w = carve_count(ws, d, pivot != 0, &need);
    if (!ws || ws_bytes < need) return KC_ENOMEM;
    if (k > d->d_max + 1 || d->m == 0) {
        count->lo = preload;
        return KC_OK;
    }
    const int scheme = pick_scheme(o, k);
    if (scheme != KC_SCHEME_VC && scheme != KC_SCHEME_EC) return KC_EINVAL;
    unsigned long long res[kAccWords];
    int hctl[CC_WORDS];
    int st = run_count(d, k, pivot ? 0 : -1, o, w, scheme == KC_SCHEME_EC, preload, res, hctl, nullptr, 0, s);
    if (st != KC_OK) return st;
    if (hctl[CC_FLAGS] & kFlagCanceled) return KC_ECANCELED;   // no valid count
    if (hctl[CC_FLAGS] & kFlagStalled) return KC_EDEVICE;      // subtree queue stalled: no valid count
    count->lo = res[0];
    count->hi = pivot ? res[1] : 0ull;
    if (pivot && (hctl[CC_FLAGS] & kFlagBigBinom)) return KC_EOVERFLOW;
    if (!pivot && res[1] != 0) return KC_EOVERFLOW;
    return KC_OK;
}

// Fixed device scratch of kc_count_noalloc: one copy per GPU, kept until the
// process ends.  Host code never uses the array's name as an address: the
// device address comes from hipGetSymbolAddress, once per device.
constexpr size_t kScratchBytes = static_cast<size_t>(KC_NOALLOC_SCRATCH_BYTES);
__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kScratchDevices];   // device address of `scratch` per device (null = not looked up)

int scratch_ptr(void** out) {
    int dev = 0;
    KC_CHECK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kScratchDevices) return KC_EUNSUPPORTED;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        KC_CHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return KC_EDEVICE;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return KC_OK;
}

}  // namespace
}  // namespace kc

namespace kc {
namespace {

// kc_count_all without pivoting: the graph-orientation traversal (Fig. 2) is
// run once per clique size, k = 3, 4, ..., until a size has no clique (at most
// d_max + 1, the largest size an orientation allows); each count is the exact
// 128-bit total of that traversal.
int count_all_orient(const kc_dag* d, kc_u128* counts, int32_t cap, int32_t* omega, void* ws, size_t ws_bytes,
                     const kc_opts* o, hipStream_t s) {
    size_t need = 0;
    CountWs w = carve_count(ws, d, false, &need);
    if (!ws || ws_bytes < need) return KC_ENOMEM;
    for (int j = 0; j <= cap; j++) counts[j].lo = counts[j].hi = 0;
    counts[0].lo = 1;
    counts[1].lo = static_cast<unsigned long long>(d->n);
    counts[2].lo = static_cast<unsigned long long>(d->m);
    int om = d->m > 0 ? 2 : (d->n > 0 ? 1 : 0);
    for (int k = 3; d->m > 0 && k <= d->d_max + 1; k++) {
        const int scheme = pick_scheme(o, k);
        if (scheme != KC_SCHEME_VC && scheme != KC_SCHEME_EC) return KC_EINVAL;
        unsigned long long res[kAccWords];
        int hctl[CC_WORDS];
        const int st = run_count(d, k, -1, o, w, scheme == KC_SCHEME_EC, 0ull, res, hctl, nullptr, 0, s);
        if (st != KC_OK) return st;
        if (hctl[CC_FLAGS] & kFlagCanceled) return KC_ECANCELED;
        if (hctl[CC_FLAGS] & kFlagStalled) return KC_EDEVICE;
        if ((res[0] | res[1]) == 0ull) break;
        om = k;
        if (k <= cap) {
            counts[k].lo = res[0];
            counts[k].hi = res[1];
        }
    }
    *omega = om;
    return KC_OK;
}

}  // namespace
}  // namespace kc

extern "C" KC_API int32_t kc_count(const kc_dag* d, int32_t k, int32_t pivot, kc_u128* count, void* ws,
                                   size_t ws_bytes, const kc_opts* o, void* stream) {
    return count_with_ws(d, k, pivot, count, ws, ws_bytes, o, static_cast<hipStream_t>(stream));
}

extern "C" KC_API int32_t kc_count_noalloc(const kc_dag* d, int32_t k, int32_t pivot, kc_u128* count,
                                           const kc_opts* o, void* stream) {
    if (!valid_dag(d) || !count || k < 1) return KC_EINVAL;
    // no side stream (its pool creates streams on first use) and no profile
    // (its events are created on first use): only the caller's stream is used
    kc_opts local{};
    if (o) local = *o;
    local.flags |= KC_OPT_SINGLE_STREAM;
    local.profile = nullptr;
    local.collect_stats = 0;
    void* ws = nullptr;
    if (k >= 3) {
        size_t need = 0;
        carve_count(nullptr, d, pivot != 0, &need);
        if (need > kScratchBytes) return KC_ENOMEM;   // beyond the fixed scratch
        const int st = scratch_ptr(&ws);
        if (st != KC_OK) return st;
    }
    return count_with_ws(d, k, pivot, count, ws, kScratchBytes, &local, static_cast<hipStream_t>(stream));
}

extern "C" KC_API int32_t kc_count_local(const kc_dag* d, int32_t k, int32_t pivot, uint64_t* local, void* ws,
                                         size_t ws_bytes, const kc_opts* o, void* stream) {
    if (!valid_dag(d) || !local || k < 1 || (d->n > 0 && !d->perm)) return KC_EINVAL;
    if (d->d_max > KC_MAX_DMAX) return KC_EUNSUPPORTED;
    size_t need = 0;
    CountWs w = carve_count(ws, d, pivot != 0, &need);
    if (!ws || ws_bytes < need) return KC_ENOMEM;
    if (d->n == 0) return KC_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int scheme = pick_scheme(o, k);
    if (scheme != KC_SCHEME_VC && scheme != KC_SCHEME_EC) return KC_EINVAL;
    const int* cancel = o ? const_cast<const int*>(reinterpret_cast<const volatile int*>(o->cancel)) : nullptr;
    KC_CHECK(hipMemsetAsync(w.ctl, 0, CC_WORDS * sizeof(int), s));
    int hctl[CC_WORDS];
    if (pivot && k >= 3 && k <= d->d_max + 1 && d->m > 0) {
        // the pivoting traversal of Fig. 3 with the per-vertex leaf rule
        KC_CHECK(hipMemsetAsync(local, 0, sizeof(uint64_t) * static_cast<size_t>(d->n), s));
        kc_opts lo{};
        if (o) lo = *o;
        lo.collect_stats = 0;
        lo.profile = nullptr;
        unsigned long long res[kAccWords];
        const int st = run_count(d, k, 2, &lo, w, scheme == KC_SCHEME_EC, 0ull, res, hctl, nullptr, 0, s,
                                 reinterpret_cast<unsigned long long*>(local));
        if (st != KC_OK) return st;
    } else {
        const int st = local_orient_launch(d, k, scheme == KC_SCHEME_EC, reinterpret_cast<unsigned long long*>(local),
                                           w.ctl, cancel, s);
        if (st != KC_OK) return st;
        KC_CHECK(hipMemcpyAsync(hctl, w.ctl, sizeof(hctl), hipMemcpyDeviceToHost, s));
        KC_CHECK(hipStreamSynchronize(s));
    }
    if (hctl[CC_FLAGS] & kFlagCanceled) return KC_ECANCELED;
    if (hctl[CC_FLAGS] & kFlagStalled) return KC_EDEVICE;
    if (hctl[CC_FLAGS] & (kFlagLocalOverflow | kFlagBigBinom)) return KC_EOVERFLOW;
    return KC_OK;
}

extern "C" KC_API int32_t kc_list(const kc_dag* d, int32_t k, int32_t* cliques, int64_t cap, uint64_t* total,
                                  void* ws, size_t ws_bytes, const kc_opts* o, void* stream) {
    if (!valid_dag(d) || !total || k < 1 || cap < 0 || (cap > 0 && !cliques) || (d->n > 0 && !d->perm))
        return KC_EINVAL;
    if (d->d_max > KC_MAX_DMAX) return KC_EUNSUPPORTED;
    *total = 0;
    size_t need = 0;
    CountWs w = carve_count(ws, d, false, &need);
    if (!ws || ws_bytes < need) return KC_ENOMEM;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (k == 1 || k == 2) {
        const int st = list_orient_launch(d, k, false, cliques, cap, nullptr, nullptr, nullptr, s);
        if (st != KC_OK) return st;
        KC_CHECK(hipStreamSynchronize(s));
        *total = k == 1 ? static_cast<uint64_t>(d->n) : static_cast<uint64_t>(d->m);
        return KC_OK;
    }
    const int scheme = pick_scheme(o, k);
    if (scheme != KC_SCHEME_VC && scheme != KC_SCHEME_EC) return KC_EINVAL;
    const int* cancel = o ? const_cast<const int*>(reinterpret_cast<const volatile int*>(o->cancel)) : nullptr;
    KC_CHECK(hipMemsetAsync(w.ctl, 0, CC_WORDS * sizeof(int), s));
    KC_CHECK(hipMemsetAsync(w.acc, 0, sizeof(unsigned long long), s));
    const int st = list_orient_launch(d, k, scheme == KC_SCHEME_EC, cliques, cap, w.acc, w.ctl, cancel, s);
    if (st != KC_OK) return st;
    int hctl[CC_WORDS];
    unsigned long long listed = 0;
    KC_CHECK(hipMemcpyAsync(hctl, w.ctl, sizeof(hctl), hipMemcpyDeviceToHost, s));
    KC_CHECK(hipMemcpyAsync(&listed, w.acc, sizeof(listed), hipMemcpyDeviceToHost, s));
    KC_CHECK(hipStreamSynchronize(s));
    if (hctl[CC_FLAGS] & kFlagCanceled) return KC_ECANCELED;
    if (hctl[CC_FLAGS] & kFlagStalled) return KC_EDEVICE;
    if (hctl[CC_FLAGS] & kFlagLocalOverflow) return KC_EOVERFLOW;
    *total = listed;
    return KC_OK;
}

extern "C" KC_API int32_t kc_count_all(const kc_dag* d, int32_t pivot, kc_u128* counts, int32_t cap,
                                       int32_t* omega, void* ws, size_t ws_bytes, const kc_opts* o,
                                       void* stream) {
    if (!valid_dag(d) || !counts || !omega || cap < 2) return KC_EINVAL;
    if (d->d_max > KC_MAX_DMAX_WIDE) return KC_EUNSUPPORTED;
    if (!pivot) return count_all_orient(d, counts, cap, omega, ws, ws_bytes, o, static_cast<hipStream_t>(stream));
    size_t need = 0;
    CountWs w = carve_count(ws, d, true, &need);
    if (!ws || ws_bytes < need) return KC_ENOMEM;
    hipStream_t s = static_cast<hipStream_t>(stream);
    for (int j = 0; j <= cap; j++) counts[j].lo = counts[j].hi = 0;
    int om = d->n > 0 ? 1 : 0;
    bool ovf = false;
    if (d->m > 0 && d->d_max >= 2) {
        const int scheme = o && o->scheme == KC_SCHEME_EC ? KC_SCHEME_EC : KC_SCHEME_VC;
        const int len = w.counts_len;
        unsigned long long* host = new (std::nothrow) unsigned long long[2 * static_cast<size_t>(len)];
        if (!host) return KC_ENOMEM;
        unsigned long long res[kAccWords];
        int hctl[CC_WORDS];
        int st = run_count(d, 0, 1, o, w, scheme == KC_SCHEME_EC, 0ull, res, hctl, host, len, s);
        if (st != KC_OK) { delete[] host; return st; }
        if (hctl[CC_FLAGS] & kFlagCanceled) { delete[] host; return KC_ECANCELED; }
        if (hctl[CC_FLAGS] & kFlagStalled) { delete[] host; return KC_EDEVICE; }   // frame queue stalled
        ovf = (hctl[CC_FLAGS] & kFlagBigBinom) != 0;
        for (int j = 3; j < len; j++) {
            if (host[2 * j] | host[2 * j + 1]) {
                om = j;
                if (j <= cap) {
                    counts[j].lo = host[2 * j];
                    counts[j].hi = host[2 * j + 1];
                }
            }
        }
        delete[] host;
    }
    counts[0].lo = 1;
    counts[1].lo = static_cast<unsigned long long>(d->n);
    counts[2].lo = static_cast<unsigned long long>(d->m);
    if (d->m > 0 && om < 2) om = 2;
    *omega = om;
    return ovf ? KC_EOVERFLOW : KC_OK;
}
