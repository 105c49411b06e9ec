// Graph-orientation traversal (Fig. 2) without binary encoding: the ablation
// of Sec. 4.3 (Fig. 7's "+BE" step removed).  Candidate sets are sorted vertex
// lists and every intersection I' = I cap Adj(v) is a parallel list
// intersection: each lane takes one member of I after v and binary-searches it
// in v's sorted out-list of the oriented CSR (no induced sub-graph, no bitsets).
//
// One wavefront owns one root and walks its tree depth first with all 64 lanes
// on each intersection; the lists of the open levels live in LDS (one buffer of
// up to d_max entries per level) with a size and a cursor per level.
#include "kc_count_impl.h"

namespace kc {
namespace {

struct ListParams {
    int k;
    int nroots;
    int need;                          // smallest root list that can hold a k-clique
    int s_cap;                         // entries per level buffer
    int levels;                        // level buffers per wavefront
    const int* __restrict__ row_ptr;
    const int* __restrict__ col;
    const int* __restrict__ src;
    int* head;                         // root queue head (zero at launch)
    unsigned long long* acc;           // [lo, hi]
    int* flags;                        // CC_FLAGS word
    const int* cancel;                 // caller's cancel flag (null: none)
};

// Members of a[i0, n) that occur in the sorted row col[b, e), compacted in order
// into out[] (when out is not null); returns how many there are.  Wave-wide.
__device__ __forceinline__ int intersect_wave(const int* a, int i0, int n, const int* __restrict__ col, int b, int e,
                                              int* out) {
    const int lane = __lane_id();
    const unsigned long long lt = lanemask_lt();
    int m = 0;
    for (int j0 = i0; j0 < n; j0 += 64) {
        const int j = j0 + lane;
        bool hit = false;
        if (j < n) {
            const int x = a[j];
            int lo = b, hi = e;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (col[mid] < x) lo = mid + 1; else hi = mid;
            }
            hit = lo < e && col[lo] == x;
        }
        const unsigned long long mk = __ballot(hit);
        if (out && hit) out[m + __popcll(mk & lt)] = a[j];
        m += __popcll(mk);
    }
    return m;
}

template <bool EC>
__global__ void __launch_bounds__(64) k_lists(ListParams P) {
    extern __shared__ __align__(16) int lds_l[];
    const int lane = threadIdx.x & 63;
    int* lvl_n = lds_l;                       // [levels] list sizes
    int* lvl_c = lds_l + P.levels;            // [levels] cursors
    int* buf = lds_l + 2 * P.levels + 2;      // [levels][s_cap]
    const int k = P.k;
    const int p_root = EC ? 2 : 1;            // path length of the root's own list
    unsigned long long cnt = 0;               // wave-uniform partial count (lane 0 flushes)
    unsigned long long hi_part = 0;

    for (;;) {
        int root = 0;
        if (lane == 0) {
            root = atomicAdd(P.head, 1);
            if (P.cancel && root < P.nroots && cancel_requested(P.cancel)) {
                atomicOr(P.flags, kFlagCanceled);
                root = P.nroots;
            }
        }
        root = __shfl(root, 0);
        if (root >= P.nroots) break;
        // level 0: the root's candidate list (N+(u), or N+(u) cap N+(v))
        int n0;
        if (EC) {
            const int u = P.src[root], v = P.col[root];
            const int a0 = root + 1, na = P.row_ptr[u + 1] - a0;      // N+(u) past v
            const int b0 = P.row_ptr[v], nb = P.row_ptr[v + 1] - b0;
            if (na < P.need || nb < P.need) continue;
            // members of N+(u) after v that are out-neighbours of v
            n0 = 0;
            for (int j0 = 0; j0 < na; j0 += 64) {
                const int j = j0 + lane;
                bool hit = false;
                int x = 0;
                if (j < na) {
                    x = P.col[a0 + j];
                    int lo = b0, hi = b0 + nb;
                    while (lo < hi) {
                        const int mid = (lo + hi) >> 1;
                        if (P.col[mid] < x) lo = mid + 1; else hi = mid;
                    }
                    hit = lo < b0 + nb && P.col[lo] == x;
                }
                const unsigned long long mk = __ballot(hit);
                if (hit) buf[n0 + __popcll(mk & lanemask_lt())] = x;
                n0 += __popcll(mk);
            }
        } else {
            const int b = P.row_ptr[root], e = P.row_ptr[root + 1];
            n0 = e - b;
            if (n0 < P.need) continue;
            for (int j = lane; j < n0; j += 64) buf[j] = P.col[b + j];
        }
        if (EC && k == 3) {
            cnt += static_cast<unsigned long long>(n0);
            wave_sync_lds();
            continue;
        }
        if (n0 < k - p_root) {
            wave_sync_lds();
            continue;
        }
        if (lane == 0) {
            lvl_n[0] = n0;
            lvl_c[0] = 0;
        }
        wave_sync_lds();
        int L = 0;
        int polls = 0;
        while (L >= 0) {
            if (P.cancel && ++polls == kCancelEvery) {
                polls = 0;
                int c = 0;
                if (lane == 0 && cancel_requested(P.cancel)) {
                    atomicOr(P.flags, kFlagCanceled);
                    c = 1;
                }
                if (__shfl(c, 0)) break;
            }
            const int p = p_root + L;                 // path length of level L's list
            const int n = lvl_n[L], c = lvl_c[L];
            // a list needs k - p more vertices; too few left: close the level
            if (n - c < k - p) {
                L--;
                continue;
            }
            const int v = buf[L * P.s_cap + c];
            if (lane == 0) lvl_c[L] = c + 1;
            const int rb = P.row_ptr[v], re = P.row_ptr[v + 1];
            if (p + 2 == k) {
                // children of v are the last level: count them
                cnt += static_cast<unsigned long long>(
                    intersect_wave(buf + L * P.s_cap, c + 1, n, P.col, rb, re, nullptr));
                wave_sync_lds();
                continue;
            }
            const int m = intersect_wave(buf + L * P.s_cap, c + 1, n, P.col, rb, re, buf + (L + 1) * P.s_cap);
            if (m >= k - p - 1) {
                if (lane == 0) {
                    lvl_n[L + 1] = m;
                    lvl_c[L + 1] = 0;
                }
                L++;
            }
            wave_sync_lds();
        }
        wave_sync_lds();
    }
    if (lane == 0) atomic_add_u128(P.acc, P.acc + 1, cnt, hi_part);
}

template <bool EC>
int launch_lists_t(const ListParams& P, hipStream_t s) {
    const size_t lds_bytes = (static_cast<size_t>(P.levels) * (P.s_cap + 2) + 2) * sizeof(int);
    if (lds_bytes > 160 * 1024) return KC_EUNSUPPORTED;
    auto kern = k_lists<EC>;
    if (lds_bytes > 64 * 1024)
        KC_CHECK(hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds_bytes)));
    int occ = 0;
    KC_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, 64, lds_bytes));
    if (occ < 1) return KC_EUNSUPPORTED;
    if (occ > 32) occ = 32;
    kern<<<device_cus() * occ, 64, lds_bytes, s>>>(P);
    KC_CHECK(hipGetLastError());
    return KC_OK;
}

}  // namespace

int lists_launch(const kc_dag* d, int k, bool ec, const CountWs& w, const int* cancel, hipStream_t s) {
    ListParams P;
    P.k = k;
    P.nroots = ec ? d->m : d->n;
    P.need = ec ? k - 2 : k - 1;
    P.s_cap = d->d_max > 1 ? d->d_max : 1;
    const int p_root = ec ? 2 : 1;
    P.levels = k - 1 - p_root > 1 ? k - 1 - p_root : 1;   // lists of path lengths p_root .. k - 2
    P.row_ptr = d->row_ptr;
    P.col = d->col;
    P.src = d->src;
    P.head = w.ctl + CC_LIGHT_HEAD;
    P.acc = w.acc;
    P.flags = w.ctl + CC_FLAGS;
    P.cancel = cancel;
    return ec ? launch_lists_t<true>(P, s) : launch_lists_t<false>(P, s);
}

}  // namespace kc
