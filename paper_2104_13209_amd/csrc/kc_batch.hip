// Batched counting: thousands of independent graphs in one pass (per-graph
// k-clique counts), capture-safe so the whole call can live in a HIP graph.
//
// The packed graphs form one disjoint union.  Orientation by degree order is
// done once for the union (each graph's order is the restriction of the union's,
// so every graph gets a valid orientation of its own).  Roots of every graph go
// through a classification into width lists, one pass per (root scheme,
// traversal) pair that the plan assigns to some size bucket: vertex or edge
// roots, and the lane walk or sub-wavefront groups of 2 to 32 lanes (Sec. 3.5).
// The persistent kernels pull roots from device queues and add the partial
// counts of a finished root to that root's graph counter.  No host
// synchronisation, no memset and no device allocation happen inside the call.
#include <cmath>

#include "kc_count_impl.h"

namespace kc {
namespace {

constexpr int kBlock = 256;

__global__ void __launch_bounds__(kBlock) k_fill_i32(int* p, int v, long long count) {
    for (long long i = blockIdx.x * static_cast<long long>(blockDim.x) + threadIdx.x; i < count;
         i += static_cast<long long>(gridDim.x) * blockDim.x)
        p[i] = v;
}

__global__ void __launch_bounds__(kBlock) k_fill_u64(unsigned long long* p, unsigned long long v, long long count) {
    for (long long i = blockIdx.x * static_cast<long long>(blockDim.x) + threadIdx.x; i < count;
         i += static_cast<long long>(gridDim.x) * blockDim.x)
        p[i] = v;
}

// Graph of every DAG vertex (binary search of perm[i] in voff) and the scheme
// of every graph's size bucket.
__global__ void __launch_bounds__(kBlock) k_gid(int n, const int* __restrict__ perm, const int* __restrict__ voff,
                                               int ngraphs, int* gid) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const int v = perm[i];
        int lo = 0, hi = ngraphs;                        // voff[lo] <= v < voff[hi]
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (voff[mid] <= v) lo = mid; else hi = mid;
        }
        gid[i] = lo;
    }
}

__global__ void __launch_bounds__(kBlock) k_graph_bucket(int ngraphs, const int* __restrict__ voff, kc_batch_plan plan,
                                                        unsigned char* bucket) {
    for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < ngraphs; g += gridDim.x * blockDim.x) {
        const int n = voff[g + 1] - voff[g];
        int b = plan.nbuckets - 1;
        for (int j = plan.nbuckets - 1; j >= 0; j--)
            if (n <= plan.n_hi[j]) b = j;
        bucket[g] = static_cast<unsigned char>(b);
    }
}

// k = 1 and k = 2: n_g and m_g directly.
__global__ void __launch_bounds__(kBlock) k_small_k(int ngraphs, int k, const int* __restrict__ voff,
                                                   const int* __restrict__ row_ptr, unsigned long long* counts) {
    for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < ngraphs; g += gridDim.x * blockDim.x) {
        const int a = voff[g], b = voff[g + 1];
        counts[2 * g] = k == 1 ? static_cast<unsigned long long>(b - a)
                               : static_cast<unsigned long long>(row_ptr[b] - row_ptr[a]) / 2ull;
        counts[2 * g + 1] = 0ull;
    }
}

__device__ __forceinline__ int width_list_b(int bound) {
    return bound <= 32 ? 0 : bound <= 64 ? 1 : bound <= 128 ? 2 : bound <= 256 ? 3 : bound <= 512 ? 4 : 5;
}

// Width-list classification of the roots of graphs whose size bucket is in
// `buckets` (a bit mask): pass 1 counts, pass 2 appends (as in the single-graph
// path).
template <bool EC, bool FILL>
__global__ void __launch_bounds__(kBlock) k_classify_batch(int nroots_total, int need, const int* __restrict__ row_ptr,
                                                          const int* __restrict__ col, const int* __restrict__ src,
                                                          const int* __restrict__ gid,
                                                          const unsigned char* __restrict__ bucket, unsigned buckets,
                                                          int* lists, int* ctl) {
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
            const int u = EC ? src[r] : r;
            if ((buckets >> bucket[gid[u]]) & 1u) {
                int bound;
                if (EC) {
                    const int v = col[r];
                    const int du = row_ptr[u + 1] - row_ptr[u] - 1;
                    const int dv = row_ptr[v + 1] - row_ptr[v];
                    bound = du < dv ? du : dv;
                } else {
                    bound = row_ptr[u + 1] - row_ptr[u];
                }
                if (bound >= need && bound >= 0) lst = width_list_b(bound);
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

struct BatchWs {
    void* orient_ws;
    int *dag_row_ptr, *dag_col, *dag_src, *perm, *gid;
    unsigned char* bucket;     // size bucket of every graph
    int* ctl[2];               // control words of alternate passes
    int* lists[2];
    int *task_ctr, *task_tot, *active;
    unsigned long long* acc;
    int nactive;
};

BatchWs carve_batch(void* ws, const kc_batch* b, size_t* bytes) {
    Carver c(ws);
    BatchWs w{};
    const int n = b->n > 0 ? b->n : 1;
    const int m = b->nnz / 2 > 0 ? b->nnz / 2 : 1;
    const size_t ows = orient_async_workspace(b->n > 0 ? b->n : 1, b->nnz);
    w.orient_ws = c.take<char>(ows);
    w.dag_row_ptr = c.take<int>(static_cast<size_t>(n) + 1);
    w.dag_col = c.take<int>(static_cast<size_t>(m));
    w.dag_src = c.take<int>(static_cast<size_t>(m));
    w.perm = c.take<int>(static_cast<size_t>(n));
    w.gid = c.take<int>(static_cast<size_t>(n));
    w.bucket = c.take<unsigned char>(static_cast<size_t>(b->ngraphs > 0 ? b->ngraphs : 1));
    const int nr = n > m ? n : m;
    for (int i = 0; i < 2; i++) w.ctl[i] = c.take<int>(CC_WORDS);
    for (int i = 0; i < 2; i++) w.lists[i] = c.take<int>(static_cast<size_t>(nr));
    w.task_ctr = c.take<int>(static_cast<size_t>(nr));
    w.task_tot = c.take<int>(static_cast<size_t>(nr));
    w.nactive = device_cus() * kLaneWavesPerCU;
    w.active = c.take<int>(static_cast<size_t>(w.nactive));
    w.acc = c.take<unsigned long long>(kAccWords);
    *bytes = c.bytes();
    return w;
}

int grid_for(long long items) {
    long long blocks = (items + kBlock - 1) / kBlock;
    const long long cap = static_cast<long long>(device_cus()) * 8;
    if (blocks > cap) blocks = cap;
    return static_cast<int>(blocks < 1 ? 1 : blocks);
}

}  // namespace
}  // namespace kc

using namespace kc;

extern "C" KC_API size_t kc_batch_workspace(const kc_batch* b, int32_t k) {
    (void)k;
    if (!b || b->ngraphs < 0 || b->n < 0 || b->nnz < 0) return 0;
    size_t bytes = 0;
    carve_batch(nullptr, b, &bytes);
    return bytes;
}

extern "C" KC_API int32_t kc_batch_count(const kc_batch* b, int32_t k, uint64_t* counts, void* ws, size_t ws_bytes,
                                         const kc_batch_plan* plan, void* stream) {
    if (!b || !counts || k < 1 || b->ngraphs < 1 || b->n < 1 || b->nnz < 0 || (b->nnz & 1)) return KC_EINVAL;
    if (!b->row_ptr || !b->voff || (b->nnz > 0 && !b->col)) return KC_EINVAL;
    if (b->max_degree < 0 || b->max_graph_edges < 0) return KC_EINVAL;
    // bound on every out-degree of the degree orientation, hence on |S|
    int out_bound = b->max_degree;
    if (b->max_graph_edges > 0) {
        const long long two_m = 2LL * b->max_graph_edges;
        long long t = static_cast<long long>(std::sqrt(static_cast<double>(two_m)));
        while (t * t > two_m) t--;
        while ((t + 1) * (t + 1) <= two_m) t++;
        if (t < out_bound) out_bound = static_cast<int>(t);
    }
    if (out_bound > KC_MAX_DMAX) return KC_EUNSUPPORTED;
    kc_batch_plan pl{};
    if (plan) {
        pl = *plan;
        if (pl.nbuckets < 1 || pl.nbuckets > KC_BATCH_MAX_BUCKETS) return KC_EINVAL;
        for (int j = 0; j < pl.nbuckets; j++) {
            if (pl.scheme[j] != KC_SCHEME_VC && pl.scheme[j] != KC_SCHEME_EC) return KC_EINVAL;
            const int wd = pl.width[j];
            if (wd < 0 || wd > 32 || (wd & (wd - 1)) != 0) return KC_EINVAL;
        }
    } else {
        pl.nbuckets = 1;
        pl.n_hi[0] = 0x7fffffff;
        pl.scheme[0] = KC_SCHEME_VC;
        pl.width[0] = 0;
    }
    size_t need = 0;
    BatchWs w = carve_batch(ws, b, &need);
    if (!ws || ws_bytes < need) return KC_ENOMEM;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int G = b->ngraphs;
    if (k <= 2) {
        k_small_k<<<grid_for(G), kBlock, 0, s>>>(G, k, b->voff, b->row_ptr, reinterpret_cast<unsigned long long*>(counts));
        KC_CHECK(hipGetLastError());
        return KC_OK;
    }
    k_fill_u64<<<grid_for(2LL * G), kBlock, 0, s>>>(reinterpret_cast<unsigned long long*>(counts), 0ull, 2LL * G);
    const int n = b->n, m = b->nnz / 2;
    int bits = 0;
    while (bits < 31 && (b->max_degree >> bits) != 0) bits++;
    int st = orient_degree_async(n, b->nnz, b->row_ptr, b->col, bits, w.dag_row_ptr, w.dag_col, w.dag_src, w.perm,
                                 w.orient_ws, s);
    if (st != KC_OK) return st;
    k_gid<<<grid_for(n), kBlock, 0, s>>>(n, w.perm, b->voff, G, w.gid);
    k_graph_bucket<<<grid_for(G), kBlock, 0, s>>>(G, b->voff, pl, w.bucket);
    k_fill_i32<<<grid_for(w.nactive), kBlock, 0, s>>>(w.active, -1, w.nactive);
    k_fill_u64<<<1, kBlock, 0, s>>>(w.acc, 0ull, kAccWords);
    KC_CHECK(hipGetLastError());
    if (m == 0) return KC_OK;

    int top = 0;
    while (top < kWidthLists - 1 && (32 << top) < out_bound) top++;
    // one pass per distinct (scheme, traversal) pair of the plan; passes run in
    // stream order, so alternate passes may reuse the same lists
    unsigned done_mask = 0;
    int pass = -1;
    for (int b0 = 0; b0 < pl.nbuckets; b0++) {
        if ((done_mask >> b0) & 1u) continue;
        const int width = pl.width[b0] <= 1 ? 0 : pl.width[b0];
        unsigned buckets = 0;
        for (int j = b0; j < pl.nbuckets; j++)
            if (pl.scheme[j] == pl.scheme[b0] && (pl.width[j] <= 1 ? 0 : pl.width[j]) == width) buckets |= 1u << j;
        done_mask |= buckets;
        pass = (pass + 1) & 1;
        const bool ec = pl.scheme[b0] == KC_SCHEME_EC;
        const int nroots = ec ? m : n;
        const int need_s = ec ? k - 2 : k - 1;
        const bool deep = k >= (ec ? 3 : 2) + 4;
        int* ctl = w.ctl[pass];
        k_fill_i32<<<1, kBlock, 0, s>>>(ctl, 0, CC_WORDS);
        if (deep) {
            k_fill_i32<<<grid_for(nroots), kBlock, 0, s>>>(w.task_ctr, 0, nroots);
            k_fill_i32<<<grid_for(nroots), kBlock, 0, s>>>(w.task_tot, 0, nroots);
        }
        if (ec) {
            k_classify_batch<true, false><<<grid_for(nroots), kBlock, 0, s>>>(
                nroots, need_s, w.dag_row_ptr, w.dag_col, w.dag_src, w.gid, w.bucket, buckets, w.lists[pass], ctl);
            k_classify_batch<true, true><<<grid_for(nroots), kBlock, 0, s>>>(
                nroots, need_s, w.dag_row_ptr, w.dag_col, w.dag_src, w.gid, w.bucket, buckets, w.lists[pass], ctl);
        } else {
            k_classify_batch<false, false><<<grid_for(nroots), kBlock, 0, s>>>(
                nroots, need_s, w.dag_row_ptr, w.dag_col, w.dag_src, w.gid, w.bucket, buckets, w.lists[pass], ctl);
            k_classify_batch<false, true><<<grid_for(nroots), kBlock, 0, s>>>(
                nroots, need_s, w.dag_row_ptr, w.dag_col, w.dag_src, w.gid, w.bucket, buckets, w.lists[pass], ctl);
        }
        KC_CHECK(hipGetLastError());
        if (width >= 2) {
            // sub-wavefront groups (Sec. 3.5), widest list first
            for (int lst = top; lst >= 0; lst--) {
                GoBatchLaunch B;
                B.k = k;
                B.ec = ec;
                B.list = lst;
                B.group = width;
                B.row_ptr = w.dag_row_ptr;
                B.col = w.dag_col;
                B.src = w.dag_src;
                B.lists = w.lists[pass];
                B.list_counts = ctl + CC_WN0;
                B.head = ctl + CC_WH0 + lst;
                B.acc = w.acc;
                B.flags = ctl + CC_FLAGS;
                B.gacc = reinterpret_cast<unsigned long long*>(counts);
                B.gid = w.gid;
                st = go_batch_launch(B, s);
                if (st != KC_OK) return st;
            }
            continue;
        }
        for (int lst = top; lst >= 0; lst--) {
            LaneLaunch L;
            L.k = k;
            L.ec = ec;
            L.pair = deep && lst >= 1;
            L.stats = false;
            L.maxw = 1 << lst;
            L.list = lst;
            L.row_ptr = w.dag_row_ptr;
            L.col = w.dag_col;
            L.src = w.dag_src;
            L.lists = w.lists[pass];
            L.counts = ctl + CC_WN0;
            L.head = ctl + CC_WH0 + lst;
            L.task_ctr = w.task_ctr;
            L.task_tot = w.task_tot;
            L.active = w.active;
            L.acc = w.acc;
            L.stats_ptr = w.acc + 2;
            L.iters_ptr = w.acc + 4;
            L.gacc = reinterpret_cast<unsigned long long*>(counts);
            L.gid = w.gid;
            st = lane_launch(L, s);
            if (st != KC_OK) return st;
        }
    }
    return KC_OK;
}
