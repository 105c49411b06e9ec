// Pivoting traversal (paper Sec. 2.3 Fig. 3, hybrid form of Sec. 2.3 / 2.4) for
// gfx950 wave64, and the exact binomial table its leaves use.
//
// Hybrid: the root level is oriented (a vertex root u with S = N+(u), or an edge
// root u->v with S = N+(u) cap N+(v)); below it the search pivots on the
// undirected sub-graph induced by S, encoded as bitset rows A[i] (Sec. 3.4).
// The root vertices are holds.
//
// One wavefront walks one root's tree depth-first (the paper keeps a whole block
// on one tree and splits the pivot search across groups, Sec. 3.2; here the
// wavefront is that block and its 64 lanes are groups of one lane).  At a node
// with candidate set I:
//   pivot   p = argmax over u in I of |I cap A[u]|, ties to the lowest index:
//           the members of I are compacted with a ballot, lanes score them in
//           parallel, a wave max-reduction picks the winner;
//   prune   P = I - A[p] (p stays in P);
//   branch  for each v in P in increasing order: a child with one more pivot
//           (v == p) or hold (v != p); with a target k a child with more than k
//           holds is skipped (the stopping criterion); the child's candidates are
//           I' = I cap A[v] minus the members of P before v;
//   leaf    I' empty: with nh holds and np pivots, count mode adds C(np, k - nh);
//           count-all mode adds C(np, j) to counts[nh + j] for j = 0..np.
// All control flow is wave-uniform; lane w holds word w of I, P and P-remaining.
// The explicit stack lives in LDS for light roots (|S| <= 64) and in a per-
// wavefront global-memory slab for heavy roots (its depth can reach |S|).
#include "kc_count_impl.h"
#include "kc_extract.h"

namespace kc {
namespace {

struct PivParams {
    int k;
    int s_cap;
    int binom_n;
    const int* __restrict__ row_ptr;
    const int* __restrict__ col;
    const int* __restrict__ src;
    const int* __restrict__ roots;
    const int* __restrict__ nroots;
    int* head;
    int* flags;
    unsigned long long* acc;                 // [lo, hi]
    unsigned long long* counts;              // count-all: {lo, hi} per size
    const unsigned long long* __restrict__ binom;
    const unsigned char* __restrict__ big;
    unsigned int* gstack;
    size_t slab_words;
    unsigned long long* stats;               // [nodes, words]
    bool steal;                              // hand saved frames to idle wavefronts
    int* qctl;                               // queue control words (zero at launch)
    int* qready;                             // ring slot sequence words (zero at launch)
    unsigned int* qitems;                    // kItemWords per ring slot
    const int* __restrict__ perm;            // local counts: DAG id -> input id
    unsigned long long* local;               // local counts: [n], input ids
    int steal_every;                         // tree nodes between looks at the frame queue
    int steal_after;                         // nodes of the current root or frame before it may hand over
    int max_waiters;                         // wavefronts that may wait for handed-over frames
    const int* cancel;                       // caller's cancel flag (null: none)
};

// ------------------------------------------------------------ binomials

// Row i of Pascal's triangle per thread: C(i, j) for j <= i / 2 from
// C(i, j + 1) = C(i, j) (i - j) / (j + 1), mirrored for j > i / 2.  Entries past
// 128 bits are flagged in big[] (and so is every later one on the rising half).
__global__ void k_binom(int N, unsigned long long* tab, unsigned char* big) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i > N) return;
    const size_t row = static_cast<size_t>(i) * (N + 1);
    U4 c = {{1u, 0u, 0u, 0u}};
    bool ok = true;
    for (int j = 0; j <= i / 2; j++) {
        const unsigned long long lo = c.l[0] | (static_cast<unsigned long long>(c.l[1]) << 32);
        const unsigned long long hi = c.l[2] | (static_cast<unsigned long long>(c.l[3]) << 32);
        for (int side = 0; side < 2; side++) {
            const int jj = side ? i - j : j;
            tab[2 * (row + jj)] = ok ? lo : ~0ull;
            tab[2 * (row + jj) + 1] = ok ? hi : ~0ull;
            big[row + jj] = ok ? 0 : 1;
        }
        if (ok && j + 1 <= i / 2) ok = muldiv(c, static_cast<unsigned int>(i - j), static_cast<unsigned int>(j + 1));
    }
    for (int j = i + 1; j <= N; j++) {
        tab[2 * (row + j)] = 0;
        tab[2 * (row + j) + 1] = 0;
        big[row + j] = 0;
    }
}

// ------------------------------------------------------------- traversal

__device__ __forceinline__ unsigned int rdlane(unsigned int v, int l) {
    return static_cast<unsigned int>(__builtin_amdgcn_readlane(static_cast<int>(v), l));
}

// (lo, hi) += (xlo, xhi); sets ovf when the sum wraps past 2^128.
__device__ __forceinline__ void add_u128(unsigned long long& lo, unsigned long long& hi, unsigned long long xlo,
                                         unsigned long long xhi, int& ovf) {
    const unsigned long long s = lo + xlo;
    const unsigned long long c = s < lo ? 1ull : 0ull;
    const unsigned long long t = hi + xhi;
    const unsigned long long u = t + c;
    ovf |= (t < hi || u < t) ? 1 : 0;
    hi = u;
    lo = s;
}

// Stack reload: a global-memory slab is read with device-coherent loads so that a
// line cached in the (non-coherent) vector L1 by an earlier pop of the same level
// cannot return stale words.
template <bool G>
__device__ __forceinline__ unsigned int st_load(const unsigned int* p) {
    if (G) return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return *p;
}

// MAXW: bitset words per row; EC: edge roots; MODE: 0 count size k, 1 count
// every size, 2 per-vertex counts of size k; GST: stack in global memory; WPB:
// wavefronts per block (each its own team).
template <int MAXW, bool EC, int MODE, bool GST, int WPB, bool STATS>
__global__ void __launch_bounds__(64 * WPB) k_piv(PivParams P) {
    constexpr bool ALL = MODE == 1;
    constexpr bool LOCAL = MODE == 2;
    constexpr int LV = 3 * MAXW + 4;
    extern __shared__ unsigned int lds[];
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int s_cap = P.s_cap;
    const int stride = b_stride_of(MAXW);
    const int cap = s_cap + 2;                        // largest clique size index
    const int extra = (ALL ? 4 * (cap + 1) : 0) + (LOCAL ? 4 * s_cap + 2 : 0);
    const int words = 8 + s_cap + s_cap * stride + extra + (GST ? 0 : (s_cap + 2) * LV);
    unsigned int* base = lds + wv * words;
    int* ctl = reinterpret_cast<int*>(base);
    int* S = reinterpret_cast<int*>(base + 8);        // candidate set, then member list
    unsigned int* A = base + 8 + s_cap;
    unsigned long long* cnt = reinterpret_cast<unsigned long long*>(A + s_cap * stride);
    // local counts: per-root counters of S's members, the path of the current
    // node (S index of each chosen vertex, top bit set for a pivot) and the
    // root's S in DAG ids (S itself is reused for member lists)
    unsigned long long* lcnt = cnt;
    unsigned int* pathv = A + s_cap * stride + 2 * s_cap;
    int* S_root = reinterpret_cast<int*>(pathv + s_cap + 2);
    unsigned int* stk = GST ? P.gstack + static_cast<size_t>(blockIdx.x * WPB + wv) * P.slab_words
                            : A + s_cap * stride + extra;
    const int k = P.k;
    const int N1 = P.binom_n + 1;
    const int nroots = *P.nroots;
    const int nh_root = EC ? 2 : 1;

    if (ALL)
        for (int i = lane; i < 2 * (cap + 1); i += 64) cnt[i] = 0ull;
    unsigned long long acc_lo = 0, acc_hi = 0, nodes = 0, words_done = 0;
    unsigned long long rootacc = 0;                   // local counts: cliques through the root vertices
    int ovf = 0, lovf = 0;

    // leaf with nh holds and np pivots; npath vertices below the root(s) on its path
    auto leaf = [&](int np, int nh, int npath) {
        if (LOCAL) {
            // Sec. 2.3: the leaf stands for C(np, k - nh) k-cliques; each hold is
            // in all of them, each pivot in the C(np - 1, k - nh - 1) that take it
            if (nh <= k && k - nh <= np) {
                const size_t ih = static_cast<size_t>(np) * N1 + (k - nh);
                const unsigned long long ph = P.binom[2 * ih];
                unsigned long long pp = 0;
                int big = P.big[ih] | (P.binom[2 * ih + 1] != 0ull);
                if (np >= 1 && k - nh - 1 >= 0) {
                    const size_t ip = static_cast<size_t>(np - 1) * N1 + (k - nh - 1);
                    pp = P.binom[2 * ip];
                    big |= P.big[ip] | (P.binom[2 * ip + 1] != 0ull);
                }
                lovf |= big;
                if (lane == 0) {
                    const unsigned long long r = rootacc + ph;
                    lovf |= r < rootacc;
                    rootacc = r;
                }
                for (int l = lane; l < npath; l += 64) {
                    const unsigned int e = pathv[l];
                    const unsigned long long x = (e & 0x80000000u) ? pp : ph;
                    if (x) {
                        const unsigned long long old = atomicAdd(&lcnt[e & 0x7fffffffu], x);
                        lovf |= old + x < old;
                    }
                }
            }
        } else if (!ALL) {
            if (lane == 0 && nh <= k && nh + np >= k) {
                const size_t ix = static_cast<size_t>(np) * N1 + (k - nh);
                ovf |= P.big[ix];
                add_u128(acc_lo, acc_hi, P.binom[2 * ix], P.binom[2 * ix + 1], ovf);
            }
        } else {
            for (int j = lane; j <= np; j += 64) {
                const size_t ix = static_cast<size_t>(np) * N1 + j;
                ovf |= P.big[ix];
                unsigned long long lo = cnt[2 * (nh + j)], hi = cnt[2 * (nh + j) + 1];
                add_u128(lo, hi, P.binom[2 * ix], P.binom[2 * ix + 1], ovf);
                cnt[2 * (nh + j)] = lo;
                cnt[2 * (nh + j) + 1] = hi;
            }
            wave_sync_lds();   // the next leaf may update these slots from other lanes
        }
    };

    // Work: the roots of this list, then frames that other wavefronts handed
    // over.  A busy wavefront that sees waiting wavefronts (and fewer queued
    // frames than waiters) hands over its shallowest saved frame that still has
    // children left: (root slot, I, P, rest of P, pivot, pivots, holds); it then
    // clears that frame's rest of P, so the children are walked exactly once.
    // Termination and the ring protocol are those of the lane walk's subtree
    // queue: a count of wavefronts in the root phase and a count of published,
    // unfinished frames, both read zero (root phase first) when all work is done.
    constexpr bool CAN_STEAL = 4 + 3 * MAXW <= kItemWords;
    const bool steal = CAN_STEAL && P.steal && !LOCAL;   // local counts keep each tree on one wavefront
    int* q = P.qctl;
    // an earlier launch of the call stalled or was canceled: give up at once
    if (ld_acquire(P.flags) & (kFlagStalled | kFlagCanceled)) return;
    if (P.cancel) {
        int c = 0;
        if (lane == 0 && cancel_requested(P.cancel)) {
            atomicOr(P.flags, kFlagCanceled);
            c = 1;
        }
        if (__shfl(c, 0)) return;
    }
    if (steal && lane == 0) atomicAdd(&q[Q_ROOTING], 1);
    bool roots_done = false, hungry = false, canceled = false;
    int cur = -1, chk = 0, cpoll = 0;                 // root whose S and rows are in LDS
    for (;;) {
        int slot = -1;
        bool from_item = false;
        unsigned int I = 0, Po = 0, Pr = 0;
        int np = 0, nh = nh_root, level = 0, p = 0;
        if (!roots_done) {
            int root = 0;
            if (lane == 0) root = atomicAdd(P.head, 1);
            root = __shfl(root, 0);
            if (root < nroots) {
                slot = root;
            } else {
                roots_done = true;
                if (!steal) break;
                if (lane == 0) __hip_atomic_fetch_add(&q[Q_ROOTING], -1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                int stay = 1;
                if (lane == 0 && atomicAdd(&q[Q_HUNGRY], 1) >= P.max_waiters) {
                    atomicAdd(&q[Q_HUNGRY], -1);
                    stay = 0;
                }
                stay = __shfl(stay, 0);
                if (!stay) break;
                hungry = true;
                continue;
            }
        } else {
            // wait for a queued frame, or for the end of all work
            int idx = -1, state = 0, backoff = 0;
            unsigned long long sig = ~0ull, t_sig = 0;
            for (;;) {
                if (lane == 0) {
                    const int h = ld_acquire(&q[Q_HEAD]);
                    const int t = ld_acquire(&q[Q_TAIL]);
                    if (h < t) {
                        if (atomicCAS(&q[Q_HEAD], h, h + 1) == h) idx = h;
                    } else {
                        const int rooting = __hip_atomic_load(&q[Q_ROOTING], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
                        const int pend = __hip_atomic_load(&q[Q_PENDING], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
                        const unsigned long long now = __builtin_amdgcn_s_memrealtime();
                        const unsigned long long sg = (static_cast<unsigned long long>(static_cast<unsigned int>(t)) << 40) ^
                                                      (static_cast<unsigned long long>(static_cast<unsigned int>(pend)) << 20) ^
                                                      static_cast<unsigned int>(rooting);
                        if (sg != sig) { sig = sg; t_sig = now; }
                        if ((rooting == 0 && pend == 0) || (ld_acquire(P.flags) & (kFlagStalled | kFlagCanceled))) state = 1;
                        else if (now - t_sig > kStallTicks) state = 2;
                    }
                }
                idx = __shfl(idx, 0);
                state = __shfl(state, 0);
                if (idx >= 0 || state != 0) break;
                if (backoff < 5) backoff++;
                for (int i = 0; i < (1 << backoff); i++) __builtin_amdgcn_s_sleep(127);
            }
            if (idx < 0) {
                if (state == 2 && lane == 0) atomicOr(P.flags, kFlagStalled);
                break;
            }
            if (hungry && lane == 0) atomicAdd(&q[Q_HUNGRY], -1);
            hungry = false;
            const int qs = idx & (kQueueCap - 1);
            const int gen = idx - qs;
            const unsigned int* it = P.qitems + static_cast<size_t>(qs) * kItemWords;
            int ok = 1;
            if (lane == 0) {
                int spins = 0;
                while (__hip_atomic_load(&P.qready[qs], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) != gen + 1) {
                    if (++spins > kReadySpins) { ok = 0; break; }
                    __builtin_amdgcn_s_sleep(2);
                }
            }
            ok = __shfl(ok, 0);
            if (!ok) {
                if (lane == 0) atomicOr(P.flags, kFlagStalled);
                break;
            }
            slot = static_cast<int>(ld_acquire(&it[0]));
            p = static_cast<int>(ld_acquire(&it[1]));
            np = static_cast<int>(ld_acquire(&it[2]));
            nh = static_cast<int>(ld_acquire(&it[3]));
            if (lane < MAXW) {
                I = ld_acquire(&it[4 + lane]);
                Po = ld_acquire(&it[4 + MAXW + lane]);
                Pr = ld_acquire(&it[4 + 2 * MAXW + lane]);
            }
            if (lane == 0)   // the wavefront's loads are done: the slot is free for the next generation
                __hip_atomic_store(&P.qready[qs], gen + kQueueCap, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            from_item = true;
        }
        // the root's S and rows (kept when the next frame is of the same root)
        if (slot != cur) {
            extract_set<1, EC>(P.roots[slot], P.row_ptr, P.col, P.src, lane, S, &ctl[1]);
            extract_rows<1, true>(ctl[1], P.row_ptr, P.col, lane, S, A, stride);
            cur = slot;
        }
        const int s = ctl[1];
        const int W = (s + 31) >> 5;
        if (!from_item && s == 0) {
            leaf(0, nh_root, 0);
            wave_sync_lds();
            continue;
        }
        if (LOCAL) {
            for (int j = lane; j < s; j += 64) {
                lcnt[j] = 0ull;
                S_root[j] = S[j];
            }
            rootacc = 0;
            wave_sync_lds();
        }

        // choose the pivot of the node with candidates I; sets p, Po, Pr
        auto enter = [&]() {
            int m = 0;
            for (int c = 0; 2 * c < W; c++) {
                const unsigned int lo = rdlane(I, 2 * c);
                const unsigned int hi = 2 * c + 1 < W ? rdlane(I, 2 * c + 1) : 0u;
                const bool mine = lane < 32 ? ((lo >> lane) & 1u) : ((hi >> (lane - 32)) & 1u);
                const unsigned long long b = __ballot(mine);
                if (mine) S[m + __popcll(b & lanemask_lt())] = 64 * c + lane;
                m += __popcll(b);
            }
            wave_sync_lds();
            unsigned int best = 0;
            for (int b0 = 0; b0 < m; b0 += 64) {
                if (b0 + lane < m) {
                    const int u = S[b0 + lane];
                    unsigned int sc = 0;
                    for (int w = 0; w < W; w++) sc += __popc(rdlane(I, w) & A[u * stride + w]);
                    const unsigned int key = (sc << 16) | (0xffffu - static_cast<unsigned int>(u));
                    best = key > best ? key : best;
                }
            }
            best = wave_max_dpp(best);
            p = static_cast<int>(0xffffu - (best & 0xffffu));
            Po = lane < W ? (I & ~A[p * stride + lane]) : 0u;
            Pr = Po;
            // scoring reads |I| rows of W words; P' one more
            if (STATS) words_done += static_cast<unsigned long long>(m + 1) * static_cast<unsigned long long>(W);
            wave_sync_lds();
        };

        if (!from_item) {
            if (lane < W) I = (lane < W - 1 || (s & 31) == 0) ? ~0u : ((1u << (s & 31)) - 1u);
            enter();
        }
        // only trees that have already run long hand work over: short ones would
        // cost a consumer more (a root extraction) than they save
        int run_nodes = 0;
        for (;;) {
            // cancellation: abandon the tree (the call's result is discarded)
            if (P.cancel && ++cpoll == kCancelEvery) {
                cpoll = 0;
                int c = 0;
                if (lane == 0 && (cancel_requested(P.cancel) || (ld_acquire(P.flags) & kFlagCanceled))) {
                    atomicOr(P.flags, kFlagCanceled);
                    c = 1;
                }
                if (__shfl(c, 0)) {
                    canceled = true;
                    break;
                }
            }
            if (steal && ++chk >= P.steal_every && (run_nodes += chk) >= P.steal_after) {
                chk = 0;
                int want = 0;
                if (lane == 0) {
                    want = ld_acquire(&q[Q_HUNGRY]);
                    if (want > 0) want -= ld_acquire(&q[Q_TAIL]) - ld_acquire(&q[Q_HEAD]);
                }
                want = __shfl(want, 0);
                int fl = -1;
                if (want > 0) {
                    // the shallowest saved frame with children left
                    for (int l = 0; l < level; l++) {
                        const unsigned int pr = lane < MAXW ? st_load<GST>(stk + static_cast<size_t>(l) * LV + 2 * MAXW + lane) : 0u;
                        if (__ballot(pr != 0u) != 0ull) { fl = l; break; }
                    }
                }
                if (fl >= 0) {
                    int t0 = -1;
                    if (lane == 0) {
                        const int h = ld_acquire(&q[Q_HEAD]);
                        int t = ld_acquire(&q[Q_TAIL]);
                        for (;;) {
                            if (t + 1 - h > kQueueCap) { t = -1; break; }
                            const int prev = atomicCAS(&q[Q_TAIL], t, t + 1);
                            if (prev == t) break;
                            t = prev;
                        }
                        if (t >= 0) atomicAdd(&q[Q_PENDING], 1);
                        t0 = t;
                    }
                    t0 = __shfl(t0, 0);
                    if (t0 >= 0) {
                        const int qs = t0 & (kQueueCap - 1);
                        const int gen = t0 - qs;
                        unsigned int* it = P.qitems + static_cast<size_t>(qs) * kItemWords;
                        int ok = 1;
                        if (lane == 0) {
                            int spins = 0;
                            while (__hip_atomic_load(&P.qready[qs], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) != gen) {
                                if (++spins > kReadySpins) { ok = 0; break; }
                                __builtin_amdgcn_s_sleep(2);
                            }
                        }
                        ok = __shfl(ok, 0);
                        if (!ok) {
                            if (lane == 0) atomicOr(P.flags, kFlagStalled);
                        } else {
                            unsigned int* f = stk + static_cast<size_t>(fl) * LV;
                            if (lane < MAXW) {
                                it[4 + lane] = st_load<GST>(f + lane);
                                it[4 + MAXW + lane] = st_load<GST>(f + MAXW + lane);
                                it[4 + 2 * MAXW + lane] = st_load<GST>(f + 2 * MAXW + lane);
                            }
                            if (lane == 0) {
                                it[0] = static_cast<unsigned int>(slot);
                                it[1] = st_load<GST>(f + 3 * MAXW);
                                it[2] = st_load<GST>(f + 3 * MAXW + 1);
                                it[3] = st_load<GST>(f + 3 * MAXW + 2);
                            }
                            // the frame's remaining children now belong to the item
                            if (lane < MAXW) f[2 * MAXW + lane] = 0u;
                            if (lane == 0)
                                __hip_atomic_store(&P.qready[qs], gen + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                        }
                    }
                }
            }
            if (chk >= P.steal_every) chk = 0;
            const unsigned long long bal = __ballot(Pr != 0u);
            if (bal == 0ull) {
                if (level == 0) break;
                level--;
                unsigned int* f = stk + static_cast<size_t>(level) * LV;
                if (lane < MAXW) {
                    I = st_load<GST>(f + lane);
                    Po = st_load<GST>(f + MAXW + lane);
                    Pr = st_load<GST>(f + 2 * MAXW + lane);
                }
                p = static_cast<int>(st_load<GST>(f + 3 * MAXW));
                np = static_cast<int>(st_load<GST>(f + 3 * MAXW + 1));
                nh = static_cast<int>(st_load<GST>(f + 3 * MAXW + 2));
                continue;
            }
            const int w0 = __ffsll(static_cast<long long>(bal)) - 1;
            const unsigned int word = rdlane(Pr, w0);
            const int v = 32 * w0 + __ffs(word) - 1;
            if (lane == w0) Pr &= Pr - 1u;
            const int np2 = np + (v == p ? 1 : 0);
            const int nh2 = nh + (v != p ? 1 : 0);
            if (!ALL && nh2 > k) continue;                  // stopping criterion: holds <= k
            if (LOCAL && lane == 0) pathv[level] = static_cast<unsigned int>(v) | (v == p ? 0x80000000u : 0u);
            const unsigned int Ip = lane < W ? (I & A[v * stride + lane] & ~(Po & ~Pr)) : 0u;
            if (STATS) {
                nodes += 1;
                words_done += static_cast<unsigned long long>(W);
            }
            if (__ballot(Ip != 0u) != 0ull) {
                unsigned int* f = stk + static_cast<size_t>(level) * LV;
                if (lane < MAXW) {
                    f[lane] = I;
                    f[MAXW + lane] = Po;
                    f[2 * MAXW + lane] = Pr;
                }
                if (lane == 0) {
                    f[3 * MAXW] = static_cast<unsigned int>(p);
                    f[3 * MAXW + 1] = static_cast<unsigned int>(np);
                    f[3 * MAXW + 2] = static_cast<unsigned int>(nh);
                }
                level++;
                I = Ip;
                np = np2;
                nh = nh2;
                enter();
            } else {
                if (LOCAL) wave_sync_lds();   // pathv[level] written by lane 0
                leaf(np2, nh2, level + 1);
            }
        }
        wave_sync_lds();
        if (canceled) break;   // waiting wavefronts leave on the flag
        if (LOCAL) {
            // this root's counts, in input vertex ids
            for (int j = lane; j < s; j += 64) {
                const unsigned long long x = lcnt[j];
                if (x) {
                    const unsigned long long old = atomicAdd(&P.local[P.perm[S_root[j]]], x);
                    lovf |= old + x < old;
                }
            }
            if (lane == 0 && rootacc) {
                const int r = P.roots[slot];
                const int u = EC ? P.src[r] : r;
                unsigned long long old = atomicAdd(&P.local[P.perm[u]], rootacc);
                lovf |= old + rootacc < old;
                if (EC) {
                    old = atomicAdd(&P.local[P.perm[P.col[r]]], rootacc);
                    lovf |= old + rootacc < old;
                }
            }
            wave_sync_lds();
        }
        if (from_item && lane == 0)
            __hip_atomic_fetch_add(&q[Q_PENDING], -1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        if (from_item) {
            // back to waiting for frames
            if (lane == 0) atomicAdd(&q[Q_HUNGRY], 1);
            hungry = true;
        }
    }
    if (hungry && lane == 0) atomicAdd(&q[Q_HUNGRY], -1);

    // flush
    if (!ALL) {
        if (lane == 0 && atomic_add_u128(P.acc, P.acc + 1, acc_lo, acc_hi)) ovf = 1;
    } else {
        wave_sync_lds();
        for (int i = lane; i <= cap; i += 64) {
            const unsigned long long lo = cnt[2 * i], hi = cnt[2 * i + 1];
            if ((lo | hi) && atomic_add_u128(P.counts + 2 * i, P.counts + 2 * i + 1, lo, hi)) ovf = 1;
        }
    }
    if (__ballot(ovf != 0) != 0ull && lane == 0) atomicOr(P.flags, kFlagBigBinom);
    if (LOCAL && __ballot(lovf != 0) != 0ull && lane == 0) atomicOr(P.flags, kFlagLocalOverflow);
    if (STATS && lane == 0) {
        atomicAdd(P.stats, nodes);
        atomicAdd(P.stats + 1, words_done);
    }
}

template <int MAXW, bool EC, int MODE, bool GST, int WPB>
int launch_piv_t(PivParams P, bool stats, int grid_cap_per_cu, hipStream_t s) {
    constexpr int LV = 3 * MAXW + 4;
    const int s_cap = P.s_cap;
    const int cap = s_cap + 2;
    const int words = 8 + s_cap + s_cap * b_stride_of(MAXW) + (MODE == 1 ? 4 * (cap + 1) : 0) +
                      (MODE == 2 ? 4 * s_cap + 2 : 0) + (GST ? 0 : (s_cap + 2) * LV);
    const size_t lds_bytes = static_cast<size_t>(words) * WPB * sizeof(unsigned int);
    if (lds_bytes > 160 * 1024) return KC_EUNSUPPORTED;
    auto kern = k_piv<MAXW, EC, MODE, GST, WPB, false>;
    if constexpr (MODE != 2) {   // no stats variant of the local-count kernels
        if (stats) kern = k_piv<MAXW, EC, MODE, GST, WPB, true>;
    }
    if (lds_bytes > 64 * 1024)
        KC_CHECK(hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds_bytes)));
    int occ = 0;
    KC_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, 64 * WPB, lds_bytes));
    if (occ < 1) return KC_EUNSUPPORTED;
    if (occ > grid_cap_per_cu) occ = grid_cap_per_cu;
    kern<<<device_cus() * occ, 64 * WPB, lds_bytes, s>>>(P);
    KC_CHECK(hipGetLastError());
    return KC_OK;
}

template <int MAXW, bool GST, int WPB, bool EC>
int launch_piv_e(const PivParams& P, int mode, bool stats, int cap, hipStream_t s) {
    switch (mode) {
        case 0: return launch_piv_t<MAXW, EC, 0, GST, WPB>(P, stats, cap, s);
        case 1: return launch_piv_t<MAXW, EC, 1, GST, WPB>(P, stats, cap, s);
        default: return launch_piv_t<MAXW, EC, 2, GST, WPB>(P, stats, cap, s);
    }
}

template <int MAXW, bool GST, int WPB>
int launch_piv_m(const PivParams& P, bool ec, int mode, bool stats, int cap, hipStream_t s) {
    return ec ? launch_piv_e<MAXW, GST, WPB, true>(P, mode, stats, cap, s)
              : launch_piv_e<MAXW, GST, WPB, false>(P, mode, stats, cap, s);
}

}  // namespace

int pivot_binom_table(const CountWs& w, hipStream_t s) {
    const int N = w.binom_n;
    k_binom<<<div_up(N + 1, 64), 64, 0, s>>>(N, w.binom, w.big);
    KC_CHECK(hipGetLastError());
    return KC_OK;
}

int pivot_launch(const PivLaunch& L, bool heavy, hipStream_t s) {
    PivParams P;
    P.k = L.k;
    P.binom_n = L.w.binom_n;
    P.row_ptr = L.row_ptr;
    P.col = L.col;
    P.src = L.src;
    P.flags = L.w.ctl + CC_FLAGS;
    P.acc = L.w.acc;
    P.counts = L.w.counts;
    P.binom = L.w.binom;
    P.big = L.w.big;
    P.gstack = L.w.gstack;
    P.slab_words = L.w.slab_words;
    P.steal = L.steal;
    P.qctl = L.w.qctl + kQueueCtlWords * (heavy ? 1 : 0);
    P.qready = L.w.qready + static_cast<size_t>(kQueueCap) * (heavy ? 1 : 0);
    P.qitems = L.w.qitems + static_cast<size_t>(kQueueCap) * kItemWords * (heavy ? 1 : 0);
    P.perm = L.perm;
    P.local = L.local;
    const int mode = L.local ? 2 : (L.all ? 1 : 0);
    P.steal_every = L.steal_every > 0 ? L.steal_every : kPivStealEvery;
    P.steal_after = L.steal_after > 0 ? L.steal_after : (L.ec && !heavy ? kPivStealAfterLightEC : kPivStealAfter);
    P.max_waiters = kPivWaitersPerCU * device_cus();
    P.cancel = L.cancel;
    if (!heavy) {
        P.s_cap = kLightCap;
        P.roots = L.w.light;
        P.nroots = L.w.ctl + CC_LIGHT_N;
        P.head = L.w.ctl + CC_LIGHT_HEAD;
        P.stats = L.w.acc + 2;
        return launch_piv_m<2, false, 4>(P, L.ec, mode, L.stats, 64, s);
    }
    P.s_cap = s_cap_for(L.d_max);
    P.roots = L.w.heavy;
    P.nroots = L.w.ctl + CC_HEAVY_N;
    P.head = L.w.ctl + CC_HEAVY_HEAD;
    P.stats = L.w.acc + 4;
    // the grid cap keeps every wavefront within the global stack slabs carved
    switch (maxw_for(L.d_max)) {
        case 4:
            // rows of at most 4 words: the frames fit in LDS beside the rows
            // (about 13.5 KB per wavefront at |S| = 128), so the stack stays on chip
            return launch_piv_m<4, false, 4>(P, L.ec, mode, L.stats, kPivBlocksPerCU, s);
        case 8: return launch_piv_m<8, true, 4>(P, L.ec, mode, L.stats, kPivBlocksPerCU, s);
        case 16: return launch_piv_m<16, true, 1>(P, L.ec, mode, L.stats, kPivBlocksPerCU, s);
        default: return launch_piv_m<32, true, 1>(P, L.ec, mode, L.stats, kPivBlocksPerCU, s);
    }
}

}  // namespace kc
