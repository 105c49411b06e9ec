// Wide roots: roots whose first vertex u has more than KC_MAX_DMAX out-
// neighbours, so that the bitset rows of their candidate set S (|S| x
// ceil(|S|/32) words) do not fit on chip.  As in Sec. 3.3 and 3.6, the induced
// sub-graph and the explicit stack then live in pre-allocated global memory: one
// slab per resident wavefront, reused root after root.
//
// Wide roots are always vertex roots, S = N+(u), also when the call counts with
// edge roots: the edge roots (u, v) of one vertex u count, together, exactly the
// cliques whose lowest vertex is u, which is what the vertex root u counts (a
// dense graph has about d+(u) times fewer vertex roots than edge roots).
// One wavefront owns one root.  Lane l holds words l, l + 64, l + 128, ... of every
// set (WPL words per lane, rows of up to 64 * WPL words), so each set operation
// is one coalesced row read and WPL ANDs per lane.  All control flow is
// wave-uniform.
//
//   rows     row i = the members of S adjacent to S[i]: only out-neighbours
//            (j > i) for the orientation walk, the undirected adjacency for
//            the pivot walk (Sec. 3.4).  Each row word is filled by one ballot
//            of 64 binary searches in the DAG's sorted out-rows.
//   mode 0   Fig. 2: at a level with remaining candidates R, the lowest member
//            v is taken and cleared; Y = R & row[v] equals I cap Adj(v) because
//            rows are upper triangular.  When v completes a (k-1)-vertex path,
//            |Y| k-cliques are counted; otherwise Y becomes the next level if it
//            can still hold the missing vertices.
//   mode 1,2 Fig. 3 below the oriented root (root vertices are holds): at a node
//            with candidates I the pivot p maximises |I cap A[p]| (ties to the
//            lowest index), P = I - A[p], and each v of P in increasing order
//            spawns the child (I cap A[v]) with one more pivot (v == p) or hold,
//            after which v leaves I.  An empty I is a leaf with nh holds and np
//            pivots: mode 1 adds C(np, k - nh) (children with more than k holds,
//            or too few vertices left to reach k, are skipped); mode 2 adds
//            C(np, j) to counts[nh + j] for every j.  Binomials are formed exactly
//            on the fly in 128 bits; a larger one sets kFlagBigBinom.
#include <climits>

#include "kc_count_impl.h"

namespace kc {
namespace {

struct WideParams {
    int k;
    int need;                       // smallest candidate bound that can reach the target
    int s_cap;                      // candidate slots per slab
    int wcap;                       // row words per stack set (multiple of 4)
    size_t slab_words;
    const int* __restrict__ row_ptr;
    const int* __restrict__ col;
    const int* __restrict__ roots;
    const int* __restrict__ nroots;
    int* head;
    int* flags;
    const int* cancel;
    unsigned long long* acc;        // [lo, hi]
    unsigned long long* counts;     // mode 2: {lo, hi} per size
    int counts_len;
    unsigned int* slabs;
};

__device__ __forceinline__ unsigned int ld_coh(const unsigned int* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_coh(unsigned int* p, unsigned int v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// First index in the sorted range a[lo, hi) whose value is >= x.
__device__ __forceinline__ int lower_bound(const int* __restrict__ a, int lo, int hi, int x) {
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (a[mid] < x) lo = mid + 1; else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ bool in_row(const int* __restrict__ col, int lo, int hi, int x) {
    const int i = lower_bound(col, lo, hi, x);
    return i < hi && col[i] == x;
}

// Exclusive prefix sum of one int per lane over the wavefront.
__device__ __forceinline__ int wave_excl_scan(int v) {
    const int lane = __lane_id();
    int x = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int y = __shfl_up(x, off, kWave);
        if (lane >= off) x += y;
    }
    return x - v;
}

// (lo, hi) += (xlo, xhi); ovf set when the 128-bit sum wraps.
__device__ __forceinline__ void add128(unsigned long long& lo, unsigned long long& hi, unsigned long long xlo,
                                       unsigned long long xhi, int& ovf) {
    const unsigned long long s = lo + xlo;
    const unsigned long long c = s < lo ? 1ull : 0ull;
    const unsigned long long t = hi + xhi;
    const unsigned long long u = t + c;
    ovf |= (t < hi || u < t) ? 1 : 0;
    lo = s;
    hi = u;
}

__device__ __forceinline__ unsigned long long u4_lo(const U4& c) {
    return c.l[0] | (static_cast<unsigned long long>(c.l[1]) << 32);
}
__device__ __forceinline__ unsigned long long u4_hi(const U4& c) {
    return c.l[2] | (static_cast<unsigned long long>(c.l[3]) << 32);
}

// C(n, r) exactly; false when it needs more than 128 bits.
__device__ bool binom128(int n, int r, U4& c) {
    c = U4{{1u, 0u, 0u, 0u}};
    if (r < 0 || r > n) {
        c.l[0] = 0u;
        return true;
    }
    if (r > n - r) r = n - r;
    for (int i = 0; i < r; i++)
        if (!muldiv(c, static_cast<unsigned int>(n - i), static_cast<unsigned int>(i + 1))) return false;
    return true;
}

template <int WPL>
struct Set {
    unsigned int w[WPL];
};

// Lowest member of x (-1 when empty); it is cleared in x.
template <int WPL>
__device__ __forceinline__ int take_lowest(Set<WPL>& x) {
    const int lane = __lane_id();
#pragma unroll
    for (int j = 0; j < WPL; j++) {
        const unsigned long long m = __ballot(x.w[j] != 0u);
        if (m) {
            const int ln = __ffsll(static_cast<long long>(m)) - 1;
            const unsigned int word = static_cast<unsigned int>(__builtin_amdgcn_readlane(static_cast<int>(x.w[j]), ln));
            if (lane == ln) x.w[j] = word & (word - 1u);
            return ((j * 64 + ln) << 5) + __ffs(static_cast<int>(word)) - 1;
        }
    }
    return -1;
}

template <int WPL>
__device__ __forceinline__ int set_count(const Set<WPL>& x) {
    int c = 0;
#pragma unroll
    for (int j = 0; j < WPL; j++) c += __popc(x.w[j]);
    return wave_sum(c);
}

// A set saved in the slab keeps its first `wc` words (every later word is zero).
template <int WPL>
__device__ __forceinline__ void set_store(unsigned int* p, const Set<WPL>& x, int wc) {
    const int lane = __lane_id();
#pragma unroll
    for (int j = 0; j < WPL; j++)
        if (j * 64 + lane < wc) st_coh(p + j * 64 + lane, x.w[j]);
}

template <int WPL>
__device__ __forceinline__ void set_load(const unsigned int* p, Set<WPL>& x, int wc) {
    const int lane = __lane_id();
#pragma unroll
    for (int j = 0; j < WPL; j++) x.w[j] = j * 64 + lane < wc ? ld_coh(p + j * 64 + lane) : 0u;
}

// x & row (row of wr words; words past wr are zero).
template <int WPL>
__device__ __forceinline__ Set<WPL> set_and_row(const Set<WPL>& x, const unsigned int* row, int wr) {
    const int lane = __lane_id();
    Set<WPL> y;
#pragma unroll
    for (int j = 0; j < WPL; j++) {
        const int wi = j * 64 + lane;
        y.w[j] = wi < wr ? (x.w[j] & row[wi]) : 0u;
    }
    return y;
}

// Candidate set of vertex root u into sl[] (ascending DAG ids); returns |S|.
__device__ int gather_root(const WideParams& P, int u, int* sl) {
    const int lane = __lane_id();
    const int b = P.row_ptr[u], e = P.row_ptr[u + 1];
    int s = e - b;
    if (s > P.s_cap) s = P.s_cap;   // only a DAG whose rows exceed its d_max
    for (int i = lane; i < s; i += 64) sl[i] = P.col[b + i];
    return s;
}

// Rows of S into the slab, `wp` words per row (a multiple of 4; words past the
// last member zero).  Row i is assembled in the LDS stage from the members of
// N+(S[i]) found (binary search) in the sorted S, then written out.  UNDIRECTED
// also sets bit i of row j for each such member S[j] (a global atomic OR into the
// zeroed rows), so that rows hold the whole adjacency inside S.
template <bool UNDIRECTED>
__device__ void build_rows(const WideParams& P, const int* sl, int s, int wp, unsigned int* rows,
                           unsigned int* stage) {
    const int lane = __lane_id();
    const int last = sl[s - 1];
    if (UNDIRECTED) {
        const size_t tot = static_cast<size_t>(s) * wp;
        for (size_t t = lane; t < tot; t += 64) rows[t] = 0u;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");   // zeroes complete before the atomics
    }
    for (int w = lane; w < wp; w += 64) stage[w] = 0u;
    wave_sync_lds();
    for (int i = 0; i < s; i++) {
        const int x = sl[i];
        const int xb = P.row_ptr[x], xe = P.row_ptr[x + 1];
        // four entries per lane per round: their loads are independent
        for (int t0 = xb; t0 < xe; t0 += 256) {
            if (P.col[t0] > last) break;   // the rest of the sorted row lies past S
            int y[4];
#pragma unroll
            for (int c = 0; c < 4; c++) {
                const int t = t0 + 64 * c + lane;
                y[c] = t < xe ? P.col[t] : INT_MAX;
            }
#pragma unroll
            for (int c = 0; c < 4; c++) {
                if (y[c] > last) continue;
                const int q = lower_bound(sl, i + 1, s, y[c]);
                if (q < s && sl[q] == y[c]) {
                    atomicOr(&stage[q >> 5], 1u << (q & 31));
                    if (UNDIRECTED) atomicOr(&rows[static_cast<size_t>(q) * wp + (i >> 5)], 1u << (i & 31));
                }
            }
        }
        wave_sync_lds();
        unsigned int* row = rows + static_cast<size_t>(i) * wp;
        for (int w = lane; w < wp; w += 64) {
            const unsigned int b = stage[w];
            if (UNDIRECTED) {
                if (b) atomicOr(&row[w], b);
            } else {
                row[w] = b;
            }
            stage[w] = 0u;
        }
        wave_sync_lds();
    }
    // the rows are read back by other lanes (and the slab held another root
    // before): complete the writes and drop stale vector-cache lines
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}

template <int WPL>
__device__ __forceinline__ Set<WPL> first_bits(int s) {
    const int lane = __lane_id();
    Set<WPL> x;
#pragma unroll
    for (int j = 0; j < WPL; j++) {
        const int b = (j * 64 + lane) * 32;
        x.w[j] = s >= b + 32 ? 0xffffffffu : (s > b ? ((1u << (s - b)) - 1u) : 0u);
    }
    return x;
}

__device__ __forceinline__ bool poll_cancel(const WideParams& P, int& polls) {
    if (!P.cancel || ++polls < kCancelEvery) return false;
    polls = 0;
    int c = 0;
    if (__lane_id() == 0 && cancel_requested(P.cancel)) {
        atomicOr(P.flags, kFlagCanceled);
        c = 1;
    }
    return __shfl(c, 0) != 0;
}

// Pivot of the set x (|x| = c >= 1): the member u with the most neighbours in x,
// ties to the lowest index.  x is staged in LDS (xs, wp words) and its members
// listed in ml; each lane scores members against their rows.
template <int WPL>
__device__ int choose_pivot(const Set<WPL>& x, int c, const unsigned int* rows, int wp, unsigned int* xs, int* ml) {
    const int lane = __lane_id();
    int mine = 0;
#pragma unroll
    for (int j = 0; j < WPL; j++) {
        const int wi = j * 64 + lane;
        if (wi < wp) xs[wi] = x.w[j];
        mine += __popc(x.w[j]);
    }
    int at = wave_excl_scan(mine);
#pragma unroll
    for (int j = 0; j < WPL; j++) {
        unsigned int word = x.w[j];
        const int base = (j * 64 + lane) << 5;
        while (word) {
            const int b = __ffs(static_cast<int>(word)) - 1;
            word &= word - 1u;
            ml[at++] = base + b;
        }
    }
    wave_sync_lds();
    unsigned int best = 0u;
    const uint4* xv = reinterpret_cast<const uint4*>(xs);
    for (int t = lane; t < c; t += 64) {
        const int u = ml[t];
        const uint4* rv = reinterpret_cast<const uint4*>(rows + static_cast<size_t>(u) * wp);
        int sc = 0;
        const int nq = wp >> 2;
        int q = 0;
        for (; q + 4 <= nq; q += 4) {   // four independent row loads per round
            uint4 b[4];
#pragma unroll
            for (int c = 0; c < 4; c++) b[c] = rv[q + c];
#pragma unroll
            for (int c = 0; c < 4; c++) {
                const uint4 a = xv[q + c];
                sc += __popc(a.x & b[c].x) + __popc(a.y & b[c].y) + __popc(a.z & b[c].z) + __popc(a.w & b[c].w);
            }
        }
        for (; q < nq; q++) {
            const uint4 a = xv[q], b = rv[q];
            sc += __popc(a.x & b.x) + __popc(a.y & b.y) + __popc(a.z & b.z) + __popc(a.w & b.w);
        }
        const unsigned int key = (static_cast<unsigned int>(sc) << 13) | static_cast<unsigned int>(8191 - u);
        best = key > best ? key : best;
    }
    best = wave_max_dpp(best);
    wave_sync_lds();   // xs and ml are rewritten by the next call
    return 8191 - static_cast<int>(best & 8191u);
}

template <int MODE, int WPL>
__global__ void __launch_bounds__(64) k_wide(WideParams P) {
    extern __shared__ __align__(16) int lds_w[];
    int* sl = lds_w;                                                          // S, then member lists
    unsigned int* xs = reinterpret_cast<unsigned int*>(lds_w + P.s_cap);      // staged set (wcap words)
    unsigned int* stage = xs + P.wcap;                                        // row stage (wcap words)
    const int lane = threadIdx.x;
    unsigned int* slab = P.slabs + static_cast<size_t>(blockIdx.x) * P.slab_words;
    unsigned int* rows = slab;
    unsigned int* stk = slab + static_cast<size_t>(P.s_cap) * P.wcap;
    unsigned int* meta = stk + static_cast<size_t>(P.s_cap + 2) * 2 * P.wcap;
    if (ld_acquire(P.flags) & (kFlagStalled | kFlagCanceled)) return;
    const int nr = *P.nroots;
    const int k = P.k;
    const int p_root = 1;
    unsigned long long lane_cnt = 0;               // mode 0: this lane's counted cliques
    unsigned long long tot_lo = 0, tot_hi = 0;     // mode 1: wave-uniform 128-bit total
    int big = 0;
    int polls = 0;
    bool stop = false;
    while (!stop) {
        int r = 0;
        if (lane == 0) {
            r = atomicAdd(P.head, 1);
            if (P.cancel && r < nr && cancel_requested(P.cancel)) {
                atomicOr(P.flags, kFlagCanceled);
                r = nr;
            }
        }
        r = __shfl(r, 0);
        if (r >= nr) break;
        const int root = P.roots[r];
        const int s = gather_root(P, root, sl);
        wave_sync_lds();
        if (s < P.need) {
            wave_sync_lds();
            continue;
        }
        const int wr = (s + 31) >> 5;
        const int wp = (wr + 3) & ~3;
        build_rows<MODE != 0>(P, sl, s, wp, rows, stage);
        wave_sync_lds();   // sl is reused for member lists below
        if (MODE == 0) {
            // Fig. 2: levels L = 0, 1, ... hold the remaining candidates of a path
            // of p_root + L vertices; level L's set is saved in the slab while a
            // deeper level is open
            Set<WPL> R = first_bits<WPL>(s);
            int cnt = s;
            int L = 0;
            for (;;) {
                if (poll_cancel(P, polls)) {
                    stop = true;
                    break;
                }
                const int p = p_root + L;
                if (cnt < k - p) {   // too few candidates left for a k-clique
                    if (L == 0) break;
                    L--;
                    set_load<WPL>(stk + static_cast<size_t>(L) * P.wcap, R, P.wcap);
                    cnt = static_cast<int>(ld_coh(meta + 4 * L));
                    continue;
                }
                const int v = take_lowest<WPL>(R);
                if (v < 0) {   // cannot happen while cnt == |R|; closes the level if it did
                    cnt = 0;
                    continue;
                }
                cnt--;
                const Set<WPL> Y = set_and_row<WPL>(R, rows + static_cast<size_t>(v) * wp, wr);
                if (p + 2 == k) {   // the path with v has k - 1 vertices: each member of Y closes a k-clique
#pragma unroll
                    for (int j = 0; j < WPL; j++) lane_cnt += static_cast<unsigned long long>(__popc(Y.w[j]));
                    continue;
                }
                const int cy = set_count<WPL>(Y);
                if (cy >= k - p - 1) {
                    set_store<WPL>(stk + static_cast<size_t>(L) * P.wcap, R, P.wcap);
                    st_coh(meta + 4 * L, static_cast<unsigned int>(cnt));
                    L++;
                    R = Y;
                    cnt = cy;
                }
            }
        } else {
            // Fig. 3: frame d holds the candidate set I (members taken so far
            // removed), the branch set R (members of P not yet taken) and the
            // scalars nh, np, p; the top frame lives in registers
            Set<WPL> I, R, C = first_bits<WPL>(s);
            int nh = 0, np = 0, pv = 0;
            int cnh = p_root, cnp = 0, cc = s;   // pending child
            bool pending = true;
            int d = -1;
            for (;;) {
                if (poll_cancel(P, polls)) {
                    stop = true;
                    break;
                }
                if (pending) {
                    pending = false;
                    if (cc == 0) {
                        // leaf: cnh holds and cnp pivots
                        if (MODE == 1) {
                            U4 b;
                            if (!binom128(cnp, k - cnh, b)) big = 1;
                            else add128(tot_lo, tot_hi, u4_lo(b), u4_hi(b), big);
                        } else if (lane == 0) {
                            U4 b = U4{{1u, 0u, 0u, 0u}};
                            bool ok = true;
                            for (int j = 0; j <= cnp / 2; j++) {
                                if (j > 0 && ok) ok = muldiv(b, static_cast<unsigned int>(cnp - j + 1),
                                                             static_cast<unsigned int>(j));
                                if (!ok) {
                                    big = 1;
                                    break;
                                }
                                const int lo_i = cnh + j, hi_i = cnh + cnp - j;
                                if (lo_i < P.counts_len)
                                    big |= atomic_add_u128(P.counts + 2 * lo_i, P.counts + 2 * lo_i + 1, u4_lo(b),
                                                           u4_hi(b)) ? 1 : 0;
                                if (hi_i != lo_i && hi_i < P.counts_len)
                                    big |= atomic_add_u128(P.counts + 2 * hi_i, P.counts + 2 * hi_i + 1, u4_lo(b),
                                                           u4_hi(b)) ? 1 : 0;
                            }
                        }
                    } else if (!(MODE == 1 && cnh + cnp + cc < k)) {
                        const int p = choose_pivot<WPL>(C, cc, rows, wp, xs, sl);
                        // open the child's frame: save the parent's, then P = C - A[p]
                        if (d >= 0) {
                            unsigned int* f = stk + static_cast<size_t>(d) * 2 * P.wcap;
                            set_store<WPL>(f, I, P.wcap);
                            set_store<WPL>(f + P.wcap, R, P.wcap);
                            // every lane writes the scalars it reads back later
                            st_coh(meta + 4 * d, static_cast<unsigned int>(nh));
                            st_coh(meta + 4 * d + 1, static_cast<unsigned int>(np));
                            st_coh(meta + 4 * d + 2, static_cast<unsigned int>(pv));
                        }
                        d++;
                        const unsigned int* rp = rows + static_cast<size_t>(p) * wp;
#pragma unroll
                        for (int j = 0; j < WPL; j++) {
                            const int wi = j * 64 + lane;
                            I.w[j] = C.w[j];
                            R.w[j] = wi < wr ? (C.w[j] & ~rp[wi]) : 0u;
                        }
                        nh = cnh;
                        np = cnp;
                        pv = p;
                    }
                }
                if (d < 0) break;
                const int v = take_lowest<WPL>(R);
                if (v < 0) {   // frame done
                    d--;
                    if (d < 0) break;
                    const unsigned int* f = stk + static_cast<size_t>(d) * 2 * P.wcap;
                    set_load<WPL>(f, I, P.wcap);
                    set_load<WPL>(f + P.wcap, R, P.wcap);
                    nh = static_cast<int>(ld_coh(meta + 4 * d));
                    np = static_cast<int>(ld_coh(meta + 4 * d + 1));
                    pv = static_cast<int>(ld_coh(meta + 4 * d + 2));
                    continue;
                }
                C = set_and_row<WPL>(I, rows + static_cast<size_t>(v) * wp, wr);
#pragma unroll
                for (int j = 0; j < WPL; j++)
                    if (j == (v >> 11) && lane == ((v >> 5) & 63)) I.w[j] &= ~(1u << (v & 31));
                cnh = v == pv ? nh : nh + 1;
                cnp = v == pv ? np + 1 : np;
                if (MODE == 1 && cnh > k) continue;
                cc = set_count<WPL>(C);
                pending = true;
            }
        }
        wave_sync_lds();
    }
    if (MODE == 0) {
        unsigned long long lo = 0, hi = 0;
        wave_sum_u128(lane_cnt, lo, hi);
        if (lane == 0 && (lo | hi)) {
            if (atomic_add_u128(P.acc, P.acc + 1, lo, hi)) atomicOr(P.flags, kFlagBigBinom);
        }
    } else if (MODE == 1) {
        if (lane == 0 && (tot_lo | tot_hi)) big |= atomic_add_u128(P.acc, P.acc + 1, tot_lo, tot_hi) ? 1 : 0;
    }
    if (lane == 0 && big) atomicOr(P.flags, kFlagBigBinom);
}

// The vertices with more than KC_MAX_DMAX out-neighbours (at least `need`),
// appended to `list`; the count goes to ctl.
__global__ void __launch_bounds__(256) k_wide_roots(int n, int need, const int* __restrict__ row_ptr, int* list,
                                                   int* ctl) {
    const int lane = threadIdx.x & 63;
    for (int base = blockIdx.x * blockDim.x; base < n; base += gridDim.x * blockDim.x) {
        const int u = base + threadIdx.x;
        bool ok = false;
        if (u < n) {
            const int du = row_ptr[u + 1] - row_ptr[u];
            ok = du > KC_MAX_DMAX && du >= need;
        }
        const unsigned long long m = __ballot(ok);
        if (m == 0ull) continue;
        int b = 0;
        if (lane == 0) b = atomicAdd(&ctl[CC_WIDE_N], __popcll(m));
        b = __shfl(b, 0);
        if (ok) list[b + __popcll(m & lanemask_lt())] = u;
    }
}

template <int MODE, int WPL>
int launch_wide_t(const WideParams& P, int grid, hipStream_t s) {
    const size_t lds_bytes = (static_cast<size_t>(P.s_cap) + 2 * P.wcap) * sizeof(int);
    auto kern = k_wide<MODE, WPL>;
    if (lds_bytes > 64 * 1024)
        KC_CHECK(hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds_bytes)));
    kern<<<grid, 64, lds_bytes, s>>>(P);
    KC_CHECK(hipGetLastError());
    return KC_OK;
}

template <int MODE>
int launch_wide_m(const WideParams& P, int grid, hipStream_t s) {
    if (P.wcap <= 64) return launch_wide_t<MODE, 1>(P, grid, s);
    if (P.wcap <= 128) return launch_wide_t<MODE, 2>(P, grid, s);
    return launch_wide_t<MODE, 4>(P, grid, s);
}

}  // namespace

int wide_launch(const kc_dag* d, int k, int mode, const CountWs& w, const int* cancel, hipStream_t s) {
    if (d->d_max <= KC_MAX_DMAX) return KC_OK;
    if (d->d_max > KC_MAX_DMAX_WIDE || !w.wide || !w.wslabs) return KC_EUNSUPPORTED;
    // a vertex root needs k - 1 candidates (count-all: 2, the smallest size reported is 3)
    const int need = mode == 2 ? 2 : k - 1;
    int cblocks = div_up(d->n, 256);
    if (cblocks > device_cus() * 8) cblocks = device_cus() * 8;
    if (cblocks < 1) cblocks = 1;
    k_wide_roots<<<cblocks, 256, 0, s>>>(d->n, need, d->row_ptr, w.wide, w.ctl);
    KC_CHECK(hipGetLastError());
    WideParams P;
    P.k = k;
    P.need = need;
    P.s_cap = wide_s_cap(d->d_max);
    P.wcap = wide_wcap(d->d_max);
    P.slab_words = w.wslab_words;
    P.row_ptr = d->row_ptr;
    P.col = d->col;
    P.roots = w.wide;
    P.nroots = w.ctl + CC_WIDE_N;
    P.head = w.ctl + CC_WIDE_HEAD;
    P.flags = w.ctl + CC_FLAGS;
    P.cancel = cancel;
    P.acc = w.acc;
    P.counts = w.counts;
    P.counts_len = w.counts_len;
    P.slabs = w.wslabs;
    const int grid = w.nwslabs;
    switch (mode) {
        case 0: return launch_wide_m<0>(P, grid, s);
        case 1: return launch_wide_m<1>(P, grid, s);
        default: return launch_wide_m<2>(P, grid, s);
    }
}

}  // namespace kc
