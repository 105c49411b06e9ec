// Per-vertex k-clique counts ("local counts"): for every vertex v, the number
// of k-cliques that contain v.
//
// Graph orientation (Fig. 2): every k-clique is found exactly once, at the leaf
// of the tree of its lowest vertex (vertex roots) or lowest edge (edge roots).
// A tree node is a path P of |P| = k - 1 vertices and its candidate set I, the
// common out-neighbours of P; its |I| k-cliques are P + {w} for w in I, so every
// vertex of P gains |I| and every w in I gains 1.  One wavefront owns a root:
// S and the bitset rows B are extracted into its LDS (Sec. 2.4, 3.4), each lane
// walks the subtrees of the tasks it takes (task i = the branch through S[i])
// depth first with an explicit stack, and keeps the S-local indices of its path
// in LDS.  Counts of S's members accumulate in per-root LDS counters and go to
// the output (in input vertex ids) once the root is done.
//
// Listing (kc_list) is the same walk with another leaf: the |I| k-cliques of a
// leaf reserve consecutive rows of the caller's output with one atomic add per
// lane, and every row below the capacity receives the clique's vertices (input
// ids, ascending orientation rank: root vertices, path, member of I).
#include "kc_count_impl.h"
#include "kc_extract.h"

namespace kc {
namespace {

struct LocalParams {
    int k;
    int nroots;
    int need;                         // smallest |S| bound that can hold a k-clique
    int s_cap;
    int levels;                       // saved levels per lane
    const int* __restrict__ row_ptr;
    const int* __restrict__ col;
    const int* __restrict__ src;
    const int* __restrict__ perm;     // DAG id -> input id
    int* head;                        // root queue head (zero at launch)
    unsigned long long* local;        // [n], input ids (zero at launch)
    int* flags;                       // CC_FLAGS word
    const int* cancel;                // caller's cancel flag (null: none)
    int* list;                        // listing: [cap][k] input ids
    long long cap;                    // listing: rows of `list`
    unsigned long long* listed;       // listing: k-cliques found (zero at launch)
};

// Listing leaf: the cliques (root vertices r0[, r1], the path's S members
// path[0], path[64], ... (this lane's LDS column), one member w of R) for each w
// in R (MW words), into consecutive output rows; nr root vertices, np path
// entries.
template <int MW>
__device__ __forceinline__ void emit_rows(const LocalParams& P, int r0, int r1, int nr, const int* path, int np,
                                          const int* S, const unsigned int* R, int c) {
    const unsigned long long base = atomicAdd(P.listed, static_cast<unsigned long long>(c));
    if (base + static_cast<unsigned long long>(c) < base) atomicOr(P.flags, kFlagLocalOverflow);
    const unsigned long long cap = static_cast<unsigned long long>(P.cap);
    if (base >= cap) return;
    unsigned long long row = base;
#pragma unroll
    for (int t = 0; t < MW; t++) {
        unsigned int x = R[t];
        while (x && row < cap) {
            const int b = __ffs(x) - 1;
            x &= x - 1u;
            int* out = P.list + row * static_cast<unsigned long long>(P.k);
            out[0] = r0;
            if (nr == 2) out[1] = r1;
            for (int q = 0; q < np; q++) out[nr + q] = P.perm[S[path[q * 64]]];
            out[nr + np] = P.perm[S[32 * t + b]];
            row++;
        }
    }
}

__device__ __forceinline__ void add_local(unsigned long long* p, unsigned long long x, int* flags) {
    if (x == 0ull) return;
    const unsigned long long old = atomicAdd(p, x);
    if (old + x < old) atomicOr(flags, kFlagLocalOverflow);
}

// LDS words of one wavefront: control, S, rows, per-root counters (u64), path
// indices and saved levels.
__host__ __device__ constexpr int local_lds_words(int mw, int s_cap, int k, int levels) {
    return 16 + s_cap + s_cap * b_stride_of(mw) + ((s_cap * b_stride_of(mw)) & 1) + 2 * s_cap + k * 64 +
           levels * (mw + 1) * 64;
}

template <int MW, bool EC, bool LIST>
__global__ void __launch_bounds__(64) k_local(LocalParams P) {
    constexpr int STRIDE = b_stride_of(MW);
    constexpr int SLOT = MW + 1;                        // saved level: R words + p
    extern __shared__ __align__(16) unsigned int lds[];
    const int lane = threadIdx.x & 63;
    const int s_cap = P.s_cap;
    int* ctl = reinterpret_cast<int*>(lds);             // [1] |S|
    int* S = reinterpret_cast<int*>(lds + 16);
    unsigned int* B = lds + 16 + s_cap;
    const int bw = s_cap * STRIDE;
    unsigned long long* cnt = reinterpret_cast<unsigned long long*>(B + bw + (bw & 1));
    int* path = reinterpret_cast<int*>(cnt + s_cap);     // [position - (p0 - 1)][lane]
    unsigned int* stk = reinterpret_cast<unsigned int*>(path + P.k * 64);   // [level][slot word][lane]
    const int k = P.k;
    const int p0 = EC ? 3 : 2;                           // path length of a task's first node
    const unsigned long long lt = lanemask_lt();

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
        // the size bound of S decides before any extraction
        int bound;
        if (EC) {
            const int u = P.src[root], v = P.col[root];
            const int du = P.row_ptr[u + 1] - P.row_ptr[u], dv = P.row_ptr[v + 1] - P.row_ptr[v];
            bound = du - 1 < dv ? du - 1 : dv;
        } else {
            bound = P.row_ptr[root + 1] - P.row_ptr[root];
        }
        if (bound < P.need) continue;
        extract_set<1, EC>(root, P.row_ptr, P.col, P.src, lane, S, &ctl[1]);
        const int s = ctl[1];
        if (s < P.need) continue;
        if (!LIST)
            for (int j = lane; j < s; j += 64) cnt[j] = 0ull;
        unsigned long long rootacc = 0;                  // cliques through the root vertices
        // listing: the root vertices open every clique of this root
        int r0 = 0, r1 = 0;
        if (LIST) {
            r0 = P.perm[EC ? P.src[root] : root];
            if (EC) r1 = P.perm[P.col[root]];
        }
        if (EC && k == 3) {
            // the root edge's triangles: one per member of S
            if (LIST) {
                wave_sync_lds();
                const unsigned long long base = lane == 0 ? atomicAdd(P.listed, static_cast<unsigned long long>(s)) : 0ull;
                const unsigned long long b0 = __shfl(base, 0);
                for (int j = lane; j < s; j += 64) {
                    const unsigned long long row = b0 + static_cast<unsigned long long>(j);
                    if (row < static_cast<unsigned long long>(P.cap)) {
                        int* out = P.list + row * 3ull;
                        out[0] = r0;
                        out[1] = r1;
                        out[2] = P.perm[S[j]];
                    }
                }
            } else {
                for (int j = lane; j < s; j += 64) cnt[j] = 1ull;
                if (lane == 0) rootacc = static_cast<unsigned long long>(s);
            }
        } else {
            extract_rows<1, false>(s, P.row_ptr, P.col, lane, S, B, STRIDE);
            unsigned int R[MW];
#pragma unroll
            for (int t = 0; t < MW; t++) R[t] = 0u;
            int p = 0, depth = 0, next_task = 0;
            bool out = false;
            for (;;) {
                bool emp = true;
#pragma unroll
                for (int t = 0; t < MW; t++) emp &= R[t] == 0u;
                if (emp && depth > 0) {
                    depth--;
                    const unsigned int* f = stk + depth * SLOT * 64 + lane;
#pragma unroll
                    for (int t = 0; t < MW; t++) R[t] = f[t * 64];
                    p = static_cast<int>(f[MW * 64]);
                    emp = false;
                }
                // lanes without work take the next tasks in turn
                const unsigned long long needy = __ballot(emp && !out);
                if (needy) {
                    const int give = min(__popcll(needy), s - next_task > 0 ? s - next_task : 0);
                    const int rank = __popcll(needy & lt);
                    if (emp && !out) {
                        if (rank < give) {
                            const int i = next_task + rank;
#pragma unroll
                            for (int t = 0; t < MW; t++) R[t] = B[i * STRIDE + t];
                            p = p0;
                            path[lane] = i;
                        } else {
                            out = true;
                        }
                    }
                    next_task += give;
                }
                bool busy = !out || depth > 0;
#pragma unroll
                for (int t = 0; t < MW; t++) busy |= R[t] != 0u;
                if (__ballot(busy) == 0ull) break;
                int c = 0;
#pragma unroll
                for (int t = 0; t < MW; t++) c += __popc(R[t]);
                if (c == 0) continue;
                if (LIST && p + 1 == k) {
                    // leaf: list P + {w} for each w in R
                    emit_rows<MW>(P, r0, r1, p0 - 1, path + lane, p - p0 + 1, S, R, c);
#pragma unroll
                    for (int t = 0; t < MW; t++) R[t] = 0u;
                    continue;
                }
                if (p + 1 == k) {
                    // leaf: P + {w} for each w in R
                    rootacc += static_cast<unsigned long long>(c);
                    for (int q = 0; q <= p - p0; q++)
                        atomicAdd(&cnt[path[q * 64 + lane]], static_cast<unsigned long long>(c));
#pragma unroll
                    for (int t = 0; t < MW; t++) {
                        unsigned int x = R[t];
                        while (x) {
                            const int b = __ffs(x) - 1;
                            x &= x - 1u;
                            atomicAdd(&cnt[32 * t + b], 1ull);
                        }
                        R[t] = 0u;
                    }
                    continue;
                }
                if (c < k - p) {                      // too few candidates for a k-clique
#pragma unroll
                    for (int t = 0; t < MW; t++) R[t] = 0u;
                    continue;
                }
                // expand the lowest candidate v: child P + {v} with R cap B[v]
                int v = 0;
                bool got = false;
#pragma unroll
                for (int t = 0; t < MW; t++) {
                    if (!got && R[t] != 0u) {
                        v = 32 * t + __ffs(R[t]) - 1;
                        R[t] &= R[t] - 1u;
                        got = true;
                    }
                }
                unsigned int Y[MW];
                int cy = 0;
#pragma unroll
                for (int t = 0; t < MW; t++) {
                    Y[t] = R[t] & B[v * STRIDE + t];
                    cy += __popc(Y[t]);
                }
                if (c - 1 >= k - p && depth < P.levels) {
                    unsigned int* f = stk + depth * SLOT * 64 + lane;
#pragma unroll
                    for (int t = 0; t < MW; t++) f[t * 64] = R[t];
                    f[MW * 64] = static_cast<unsigned int>(p);
                    depth++;
                } else if (c - 1 >= k - p) {
                    // no free level (never taken: levels cover the deepest path)
                    atomicOr(P.flags, kFlagStalled);
                }
                path[(p - p0 + 1) * 64 + lane] = v;
                p++;
#pragma unroll
                for (int t = 0; t < MW; t++) R[t] = cy >= k - p ? Y[t] : 0u;
            }
        }
        // counts of this root: members of S, then the root vertices
        wave_sync_lds();
        if (LIST) continue;
        for (int j = lane; j < s; j += 64) add_local(&P.local[P.perm[S[j]]], cnt[j], P.flags);
        rootacc = wave_sum(rootacc);
        if (lane == 0) {
            if (EC) {
                add_local(&P.local[P.perm[P.src[root]]], rootacc, P.flags);
                add_local(&P.local[P.perm[P.col[root]]], rootacc, P.flags);
            } else {
                add_local(&P.local[P.perm[root]], rootacc, P.flags);
            }
        }
        wave_sync_lds();
    }
}

// k = 2: every edge adds 1 to both ends.
__global__ void k_local_edges(int m, const int* __restrict__ src, const int* __restrict__ col,
                              const int* __restrict__ perm, unsigned long long* local) {
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < m; e += gridDim.x * blockDim.x) {
        atomicAdd(&local[perm[src[e]]], 1ull);
        atomicAdd(&local[perm[col[e]]], 1ull);
    }
}

__global__ void k_fill_local(int n, unsigned long long* local, unsigned long long v) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) local[i] = v;
}

template <int MW, bool EC, bool LIST>
int launch_local_t(const LocalParams& base, hipStream_t s) {
    LocalParams P = base;
    P.s_cap = 32 * MW;
    const size_t lds_bytes = static_cast<size_t>(local_lds_words(MW, P.s_cap, P.k, P.levels)) * 4;
    if (lds_bytes > 160 * 1024) return KC_EUNSUPPORTED;
    auto kern = k_local<MW, EC, LIST>;
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

template <bool EC, bool LIST>
int launch_local(const LocalParams& P, int d_max, hipStream_t s) {
    if (d_max <= 32) return launch_local_t<1, EC, LIST>(P, s);
    if (d_max <= 64) return launch_local_t<2, EC, LIST>(P, s);
    if (d_max <= 128) return launch_local_t<4, EC, LIST>(P, s);
    if (d_max <= 256) return launch_local_t<8, EC, LIST>(P, s);
    if (d_max <= 512) return launch_local_t<16, EC, LIST>(P, s);
    return launch_local_t<32, EC, LIST>(P, s);
}

// Listing of k <= 2: vertices, or the DAG's edges (src < col in rank order).
__global__ void k_list_small(int k, int n, int m, const int* __restrict__ src, const int* __restrict__ col,
                             const int* __restrict__ perm, int* list, long long cap) {
    const long long items = k == 1 ? n : m;
    for (long long i = blockIdx.x * static_cast<long long>(blockDim.x) + threadIdx.x; i < items && i < cap;
         i += static_cast<long long>(gridDim.x) * blockDim.x) {
        if (k == 1) {
            list[i] = perm[i];
        } else {
            list[2 * i] = perm[src[i]];
            list[2 * i + 1] = perm[col[i]];
        }
    }
}

}  // namespace

int local_orient_launch(const kc_dag* d, int k, bool ec, unsigned long long* local, int* ctl, const int* cancel,
                        hipStream_t s) {
    const int n = d->n, m = d->m;
    const int grid = div_up(n > m ? n : m, 256) < device_cus() * 8 ? div_up(n > m ? n : m, 256) : device_cus() * 8;
    k_fill_local<<<grid > 0 ? grid : 1, 256, 0, s>>>(n, local, k == 1 ? 1ull : 0ull);
    KC_CHECK(hipGetLastError());
    if (k == 1 || m == 0 || k > d->d_max + 1) return KC_OK;
    if (k == 2) {
        k_local_edges<<<grid > 0 ? grid : 1, 256, 0, s>>>(m, d->src, d->col, d->perm, local);
        KC_CHECK(hipGetLastError());
        return KC_OK;
    }
    LocalParams P;
    P.k = k;
    P.nroots = ec ? m : n;
    P.need = ec ? k - 2 : k - 1;
    P.s_cap = 0;
    // saved levels: the path grows from p0 to k - 1, one level per path length
    const int p0 = ec ? 3 : 2;
    P.levels = k - p0 > 1 ? k - p0 : 1;
    P.row_ptr = d->row_ptr;
    P.col = d->col;
    P.src = d->src;
    P.perm = d->perm;
    P.head = ctl + CC_LIGHT_HEAD;
    P.local = local;
    P.flags = ctl + CC_FLAGS;
    P.cancel = cancel;
    P.list = nullptr;
    P.cap = 0;
    P.listed = nullptr;
    return ec ? launch_local<true, false>(P, d->d_max, s) : launch_local<false, false>(P, d->d_max, s);
}

int list_orient_launch(const kc_dag* d, int k, bool ec, int* list, long long cap, unsigned long long* listed,
                       int* ctl, const int* cancel, hipStream_t s) {
    const int n = d->n, m = d->m;
    if (k <= 2) {
        const long long items = k == 1 ? n : m;
        const long long todo = items < cap ? items : cap;
        if (todo > 0) {
            int grid = div_up(todo, 256);
            if (grid > device_cus() * 8) grid = device_cus() * 8;
            k_list_small<<<grid, 256, 0, s>>>(k, n, m, d->src, d->col, d->perm, list, cap);
            KC_CHECK(hipGetLastError());
        }
        return KC_OK;
    }
    if (m == 0 || k > d->d_max + 1) return KC_OK;
    LocalParams P;
    P.k = k;
    P.nroots = ec ? m : n;
    P.need = ec ? k - 2 : k - 1;
    P.s_cap = 0;
    const int p0 = ec ? 3 : 2;
    P.levels = k - p0 > 1 ? k - p0 : 1;
    P.row_ptr = d->row_ptr;
    P.col = d->col;
    P.src = d->src;
    P.perm = d->perm;
    P.head = ctl + CC_LIGHT_HEAD;
    P.local = nullptr;
    P.flags = ctl + CC_FLAGS;
    P.cancel = cancel;
    P.list = list;
    P.cap = cap;
    P.listed = listed;
    return ec ? launch_local<true, true>(P, d->d_max, s) : launch_local<false, true>(P, d->d_max, s);
}

}  // namespace kc
