// Graph-orientation traversal (paper Fig. 2) with lane-private depth-first
// walks and in-wavefront work donation, for gfx950 wave64.  The kernel
// templates live here; kc_lane_w*.hip instantiate one row width each (so the
// widths compile in parallel) and kc_lane.hip dispatches to them.
//
// Each wavefront owns one root at a time: it extracts S and the bitset rows B
// into its own LDS (Sec. 2.4, 3.4), then every lane walks subtrees on its own:
// lane state is the current level's remaining candidate set R (MAXW words in
// registers), the path length p, and an explicit stack of saved levels in LDS
// (Sec. 3.3).  A step takes the lowest set bit v of R, clears it, and forms
// Y = R & B[v] (rows are upper triangular, so this is I cap Adj(v) of Fig. 2);
// at the last level it adds popcount(Y), otherwise it descends into Y, saving R
// only when R still holds candidates.
//
// Work sources, in order:
//   tasks      vertex tasks i (the branch through S[i]) from a per-wavefront
//              counter; for deep trees on wide roots, pair tasks (i, j) (the
//              branch through S[i], S[j]) from a global per-root counter, so that
//              other wavefronts can join a root that is still being counted;
//   donation   when some lanes have nothing left and others are deep in a
//              subtree, the r-th idle lane receives the shallowest saved level of
//              the r-th busy lane through an LDS mailbox (ballot ranks pair them;
//              no atomics are needed inside a wavefront);
//   helping    a wavefront whose root queue is empty joins a root whose pair tasks
//              are not all claimed (it extracts its own copy of that root).
#pragma once

#include "kc_count_impl.h"
#include "kc_extract.h"

namespace kc {
namespace lanewalk {

constexpr int kPairChunk = 64;    // pair tasks claimed per global atomic
constexpr int kRootChunk = 8;     // vertex-task roots claimed per global atomic
constexpr int kInner = 8;         // lane-local steps per wavefront-level round
constexpr int kStealMax = 8;      // subtrees handed over per look

struct LaneParams {
    int k;
    int s_cap;
    int levels;                     // saved levels per lane
    int list;                       // index of this root list
    const int* __restrict__ row_ptr;
    const int* __restrict__ col;
    const int* __restrict__ src;
    const int* __restrict__ lists;  // all root lists, back to back
    const int* __restrict__ counts; // root count of every list
    int* head;                      // this list's queue head
    int* task_ctr;                  // pair mode: per-root claimed-task counters
    int* task_tot;                  // pair mode: per-root task totals + 1 (0 = not published)
    int* active;                    // pair mode: root slot owned by each wavefront, -1 if none
    unsigned long long* acc;        // [lo, hi]
    unsigned long long* stats;      // [nodes, words]
    unsigned long long* iters;      // [traversal loop iterations per wavefront, lane expansions], summed
    unsigned long long* timing;     // [sum of wavefront busy ticks, min start, max end]
    unsigned long long* cwords;     // stats: sum over counted cliques of the root's bitset words
    unsigned long long* gacc;       // batched: per-graph {lo, hi}; null otherwise
    const int* __restrict__ gid;    // batched: graph of each DAG vertex
    bool steal;                     // pair mode: subtree queue between wavefronts
    bool helper;                    // joins a running launch: no roots of its own, no waiter cap
    int* qctl;                      // queue control words (zero at launch)
    int* qready;                    // per ring slot (zero at launch): g*cap free for the producer of
                                    // generation g, g*cap + 1 written, (g+1)*cap read
    unsigned int* qitems;           // kItemWords per item
    int* flags;                     // CC_FLAGS word: kFlagStalled, kFlagCanceled
    int steal_every;                // wavefront rounds (up to kInner lane steps each) between queue looks
    int steal_after;                // rounds on the current root or subtree before it may hand over
    const int* cancel;              // caller's cancel flag (null: none)
};

// Poll the caller's cancel flag (lane 0, broadcast); on a request, mark the
// call canceled.  Wave-uniform result.
__device__ __forceinline__ bool poll_cancel(const int* cancel, int* flags) {
    int c = 0;
    if (__lane_id() == 0 && cancel_requested(cancel)) {
        atomicOr(flags, kFlagCanceled);
        c = 1;
    }
    return __shfl(c, 0) != 0;
}

// Batched counts: the lanes' partial counts of one root belong to one graph; add
// them to that graph's 128-bit counter and restart from zero.
__device__ __forceinline__ void flush_root(const LaneParams& P, int g, unsigned long long& acc) {
    unsigned long long lo, hi;
    wave_sum_u128(acc, lo, hi);
    if (__lane_id() == 0 && (lo | hi)) atomic_add_u128(P.gacc + 2 * g, P.gacc + 2 * g + 1, lo, hi);
    acc = 0;
}

// Index of the r-th set bit (0-based) of x, r < popc(x).
__device__ __forceinline__ int select_bit(unsigned int x, int r) {
    int pos = 0;
    int c = __popc(x & 0xffffu);
    if (r >= c) { r -= c; x >>= 16; pos += 16; }
    c = __popc(x & 0xffu);
    if (r >= c) { r -= c; x >>= 8; pos += 8; }
    c = __popc(x & 0xfu);
    if (r >= c) { r -= c; x >>= 4; pos += 4; }
    c = __popc(x & 0x3u);
    if (r >= c) { r -= c; x >>= 2; pos += 2; }
    c = static_cast<int>(x & 1u);
    if (r >= c) { pos += 1; }
    return pos;
}

// Edges of the sub-graph induced by Y: sum over x in Y of |Y cap B[x]|.  Rows
// are upper triangular, so this counts every pair once in any visiting order,
// and row x (word t) can skip the words below t.  This is the whole last level
// of Fig. 2 under a node whose candidate set is Y, done in one tight loop.
template <int MW>
__device__ __forceinline__ unsigned int leaf_edges(const unsigned int (&Y)[MW], const unsigned int* B) {
    constexpr int STRIDE = lane_stride(MW);
    unsigned int c = 0;
#pragma unroll
    for (int t = 0; t < MW; t++) {
        unsigned int x = Y[t];
        while (x) {
            const int b = __ffs(x) - 1;
            x &= x - 1u;
            const unsigned int* row = B + (32 * t + b) * STRIDE;
            if constexpr (STRIDE % 4 != 0) {
#pragma unroll
                for (int w = t; w < MW; w++) c += __popc(Y[w] & row[w]);
            } else {
                // 128-bit reads from the quad holding word t on
#pragma unroll
                for (int q = t >> 2; q < (MW + 3) / 4; q++) {
                    const uint4 r4 = *reinterpret_cast<const uint4*>(row + 4 * q);
                    c += __popc(Y[4 * q] & r4.x);
                    if (4 * q + 1 < MW) c += __popc(Y[4 * q + 1] & r4.y);
                    if (4 * q + 2 < MW) c += __popc(Y[4 * q + 2] & r4.z);
                    if (4 * q + 3 < MW) c += __popc(Y[4 * q + 3] & r4.w);
                }
            }
        }
    }
    return c;
}

// Lowest set bit of R (R not empty): returns its index and clears it.  Words are
// taken in 64-bit pairs, which halves the select chain.
template <int MW>
__device__ __forceinline__ int pop_lowest(unsigned int (&R)[MW]) {
    int v = 0;
    bool got = false;
#pragma unroll
    for (int t = 0; t < MW; t += 2) {
        if (t + 1 < MW) {
            unsigned long long x = (static_cast<unsigned long long>(R[t + 1]) << 32) | R[t];
            if (!got && x != 0ull) {
                v = 32 * t + __ffsll(x) - 1;
                x &= x - 1ull;
                R[t] = static_cast<unsigned int>(x);
                R[t + 1] = static_cast<unsigned int>(x >> 32);
                got = true;
            }
        } else if (!got && R[t] != 0u) {
            v = 32 * t + __ffs(R[t]) - 1;
            R[t] &= R[t] - 1u;
            got = true;
        }
    }
    return v;
}

// Words [0, MW) of a bitset row at stride lane_stride(MW): 32-bit reads for odd
// strides, 128-bit reads when the stride is a multiple of 4 (16-byte aligned).
template <int MW>
__device__ __forceinline__ void load_row(const unsigned int* p, unsigned int (&x)[MW]) {
    if constexpr (lane_stride(MW) % 4 != 0) {
#pragma unroll
        for (int i = 0; i < MW; i++) x[i] = p[i];
    } else {
#pragma unroll
        for (int i = 0; i < (MW + 3) / 4; i++) {
            const uint4 q = *reinterpret_cast<const uint4*>(p + 4 * i);
            x[4 * i] = q.x;
            if (4 * i + 1 < MW) x[4 * i + 1] = q.y;
            if (4 * i + 2 < MW) x[4 * i + 2] = q.z;
            if (4 * i + 3 < MW) x[4 * i + 3] = q.w;
        }
    }
}

// One root's traversal with rows of MW words (MW >= the root's word count):
// bitset rows, pair-task prefix, then the lane walks until no lane holds work
// and no task is left.  acc / nodes / wsum / iters accumulate per lane.
template <int MW, bool EC, bool PAIR, bool STATS>
__device__ __forceinline__ void walk_root(const LaneParams& P, int k, int p0, int s, int slot, bool helping,
                                          const unsigned int* item, int item_p, bool fresh,
                                          const int* S, unsigned int* B, int* pre, unsigned int* mbox,
                                          unsigned int* stk, int* tctr, int* ttot, unsigned long long lt,
                                          unsigned long long& acc, unsigned long long& nodes,
                                          unsigned long long& wsum, unsigned long long& iters,
                                          unsigned long long& exps, unsigned long long& cw) {
    constexpr int STRIDE = lane_stride(MW);
    const unsigned long long acc_in = acc;
    constexpr int SLOT = MW + 1;                    // saved level: R words + p
    const int lane = __lane_id();
    if (fresh) extract_rows<1, false>(s, P.row_ptr, P.col, lane, S, B, STRIDE);
    const unsigned long long W = static_cast<unsigned long long>((s + 31) >> 5);

    int total = item ? 0 : s;                        // tasks of this root
    if (PAIR && !item) {
        // pre[i] = number of pair tasks before row i
        int run = 0;
        for (int b0 = 0; b0 < s; b0 += 64) {
            const int i = b0 + lane;
            int c = 0;
            if (i < s) {
                unsigned int row[MW];
                load_row<MW>(B + i * STRIDE, row);
#pragma unroll
                for (int t = 0; t < MW; t++) c += __popc(row[t]);
            }
            int inc = c;
#pragma unroll
            for (int off = 1; off < 64; off <<= 1) {
                const int y = __shfl_up(inc, off, 64);
                if (lane >= off) inc += y;
            }
            if (i < s) pre[i] = run + inc - c;
            run += __shfl(inc, 63);
        }
        if (lane == 0) pre[s] = run;
        wave_sync_lds();
        total = run;
        if (!helping && lane == 0) {
            __hip_atomic_store(&ttot[slot], run + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&P.active[blockIdx.x], slot, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        }
    }

    // ---------------------------------------------------- traversal
    unsigned int R[MW];
#pragma unroll
    for (int t = 0; t < MW; t++) R[t] = 0u;        // words >= Wr stay zero for this root
    int p = 0, depth = 0, sbase = 0;
    bool out = item != nullptr;                      // no task left for this lane
    if (item && lane == 0) {
        // a queued subtree: lane 0 starts from its candidate set, the others
        // receive work by donation
#pragma unroll
        for (int t = 0; t < MW; t++) R[t] = item[4 + t];
        p = item_p;
    }
    const bool steal = PAIR && P.steal && P.counts[P.list] < 2 * static_cast<int>(gridDim.x);
    int chk = 0, run_rounds = 0;   // only walks that have already run long hand work over
    int cpoll = 0;                 // rounds since the last look at the cancel flag
    int next_task = 0;                               // vertex tasks: wave counter
    int tq = 0, tq_end = 0;                          // pair tasks: claimed, unassigned range
    bool pq_done = false;                            // pair tasks: root counter exhausted

    for (;;) {
        if (STATS) iters += 1;
        bool emp = true;
#pragma unroll
        for (int t = 0; t < MW; t++) emp &= R[t] == 0u;
        // pop a saved level
        if (emp && depth > sbase) {
            depth--;
            const unsigned int* f = stk + depth * SLOT * 64 + lane;
#pragma unroll
            for (int t = 0; t < MW; t++) R[t] = f[t * 64];
            p = static_cast<int>(f[MW * 64]);
            emp = false;
        }
        // claim tasks for lanes that have nothing
        const unsigned long long needy = __ballot(emp && !out);
        if (needy) {
            const int nn = __popcll(needy);
            const int rank = __popcll(needy & lt);
            int t0 = 0, give = 0;
            bool exhausted = false;
            if (item) {
                exhausted = true;
            } else if (PAIR) {
                // pair tasks: claim whole chunks from the root's global counter
                // only when the wavefront-local range is empty, then hand them out
                if (tq == tq_end && !pq_done) {
                    int b = 0;
                    if (lane == 0) b = atomicAdd(&tctr[slot], kPairChunk);
                    b = __shfl(b, 0);
                    if (b < total) {
                        tq = b;
                        tq_end = b + kPairChunk < total ? b + kPairChunk : total;
                    } else {
                        pq_done = true;
                    }
                }
                t0 = tq;
                give = min(nn, tq_end - tq);
                tq += give;
                exhausted = pq_done && tq == tq_end;
            } else {
                t0 = next_task;
                give = min(nn, total - next_task > 0 ? total - next_task : 0);
                next_task += give;
                exhausted = next_task >= total;
            }
            if (emp && !out) {
                if (rank < give) {
                    const int t = t0 + rank;
                    sbase = depth = 0;
                    if (PAIR) {
                        // pair task t -> (i, j): row i by binary search of pre[],
                        // j the (t - pre[i])-th set bit of B[i]
                        int lo = 0, hi = s;                     // pre[lo] <= t < pre[hi]
                        while (hi - lo > 1) {
                            const int mid = (lo + hi) >> 1;
                            if (pre[mid] <= t) lo = mid; else hi = mid;
                        }
                        const int i = lo;
                        int r = t - pre[i], j = 0;
                        bool got = false;
#pragma unroll
                        for (int w = 0; w < MW; w++) {
                            const unsigned int x = B[i * STRIDE + w];
                            const int c = __popc(x);
                            if (!got && r < c) { j = 32 * w + select_bit(x, r); got = true; }
                            if (!got) r -= c;
                        }
                        unsigned int c2 = 0, ri[MW], rj[MW];
                        load_row<MW>(B + i * STRIDE, ri);
                        load_row<MW>(B + j * STRIDE, rj);
#pragma unroll
                        for (int w = 0; w < MW; w++) {
                            R[w] = ri[w] & rj[w];
                            c2 += __popc(R[w]);
                        }
                        p = p0 + 1;
                        if (STATS) { nodes += 1; wsum += W; }
                        if (p + 1 == k || p + 2 == k || static_cast<int>(c2) < k - p) {
                            // leaf levels counted at once; a set smaller than the
                            // k - p vertices still missing holds no k-clique
                            if (p + 1 == k) {
                                acc += c2;
                            } else if (p + 2 == k) {
                                if (c2 >= 2) acc += leaf_edges<MW>(R, B);
                                if (STATS) { nodes += c2; wsum += W * c2; }
                            }
#pragma unroll
                            for (int w = 0; w < MW; w++) R[w] = 0u;
                        }
                    } else {
                        unsigned int c2 = 0;
                        load_row<MW>(B + t * STRIDE, R);
#pragma unroll
                        for (int w = 0; w < MW; w++) c2 += __popc(R[w]);
                        p = p0;
                        if (p + 1 == k || p + 2 == k || static_cast<int>(c2) < k - p) {
                            // leaf levels counted at once; a set smaller than the
                            // k - p vertices still missing holds no k-clique
                            if (p + 1 == k) {
                                acc += c2;
                            } else if (p + 2 == k) {
                                if (c2 >= 2) acc += leaf_edges<MW>(R, B);
                                if (STATS) { nodes += c2; wsum += W * c2; }
                            }
#pragma unroll
                            for (int w = 0; w < MW; w++) R[w] = 0u;
                        }
                    }
                } else if (exhausted) {
                    out = true;
                }
            }
        }
        // donation: the r-th idle lane takes the shallowest saved level of the
        // r-th lane that has one
        bool idle = true;
#pragma unroll
        for (int t = 0; t < MW; t++) idle &= R[t] == 0u;
        idle = idle && depth <= sbase && out;
        const unsigned long long idle_m = __ballot(idle);
        const unsigned long long donor_m = __ballot(depth > sbase);
        if (idle_m != 0ull && donor_m != 0ull) {
            const int n = min(__popcll(idle_m), __popcll(donor_m));
            if (depth > sbase) {
                const int rd = __popcll(donor_m & lt);
                if (rd < n) {
                    const unsigned int* f = stk + sbase * SLOT * 64 + lane;
#pragma unroll
                    for (int t = 0; t <= MW; t++) mbox[rd * SLOT + t] = f[t * 64];
                    sbase++;
                }
            }
            wave_sync_lds();
            if (idle) {
                const int ri = __popcll(idle_m & lt);
                if (ri < n) {
#pragma unroll
                    for (int t = 0; t < MW; t++) R[t] = mbox[ri * SLOT + t];
                    p = static_cast<int>(mbox[ri * SLOT + MW]);
                    depth = sbase = 0;
                }
            }
            wave_sync_lds();
        }
        // cancellation: abandon the walk (the call's count is discarded)
        if (P.cancel && ++cpoll == kCancelEvery) {
            cpoll = 0;
            if (poll_cancel(P.cancel, P.flags)) return;
        }
        // subtree queue: when wavefronts wait for work (more than are queued),
        // hand over the shallowest saved levels of up to kStealMax lanes
        if (steal && ++chk >= P.steal_every && (run_rounds += chk) >= P.steal_after) {
            chk = 0;
            int want = 0;
            if (lane == 0) {
                want = ld_acquire(&P.qctl[Q_HUNGRY]);
                if (want > 0) want -= ld_acquire(&P.qctl[Q_TAIL]) - ld_acquire(&P.qctl[Q_HEAD]);
            }
            want = __shfl(want, 0);
            const unsigned long long dm = __ballot(depth > sbase);
            int n = min(min(want, __popcll(dm)), kStealMax);
            if (n > 0) {
                int t0 = -1;
                if (lane == 0) {
                    // reserve n consecutive items while the ring has room
                    // (items below head are claimed; their slots free up once read)
                    const int h = ld_acquire(&P.qctl[Q_HEAD]);
                    int t = ld_acquire(&P.qctl[Q_TAIL]);
                    for (;;) {
                        if (t + n - h > kQueueCap) { t = -1; break; }
                        const int prev = atomicCAS(&P.qctl[Q_TAIL], t, t + n);
                        if (prev == t) break;
                        t = prev;
                    }
                    if (t >= 0) atomicAdd(&P.qctl[Q_PENDING], n);
                    t0 = t;
                }
                t0 = __shfl(t0, 0);
                if (t0 >= 0 && depth > sbase) {
                    const int rd = __popcll(dm & lt);
                    if (rd < n) {
                        const int idx = t0 + rd;
                        const int qs = idx & (kQueueCap - 1);
                        const int gen = idx - qs;           // ring generation x capacity
                        unsigned int* it = P.qitems + static_cast<size_t>(qs) * kItemWords;
                        // wait until the slot's item of the previous generation has been read
                        int spins = 0;
                        while (__hip_atomic_load(&P.qready[qs], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) != gen &&
                               ++spins <= kReadySpins)
                            __builtin_amdgcn_s_sleep(2);
                        if (spins > kReadySpins) {
                            atomicOr(P.flags, kFlagStalled);
                        } else {
                            const unsigned int* f = stk + sbase * SLOT * 64 + lane;
                            it[0] = static_cast<unsigned int>(slot);
                            it[1] = f[MW * 64];
#pragma unroll
                            for (int t = 0; t < MW; t++) it[4 + t] = f[t * 64];
                            __hip_atomic_store(&P.qready[qs], gen + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                        }
                        sbase++;
                    }
                }
            }
        }
        if (chk >= P.steal_every) chk = 0;
        // done with this root when no lane holds work and no task is left
        bool busy = false;
#pragma unroll
        for (int t = 0; t < MW; t++) busy |= R[t] != 0u;
        busy = busy || depth > sbase;
        if (__ballot(busy || !out) == 0ull) break;
        // up to kInner steps of lane-local work (pop a saved level, expand one
        // node) between the wavefront-level checks above
        for (int st = 0; st < kInner; st++) {
            if (st > 0) {
                bool e2 = true;
#pragma unroll
                for (int t = 0; t < MW; t++) e2 &= R[t] == 0u;
                if (e2 && depth > sbase) {
                    depth--;
                    const unsigned int* f = stk + depth * SLOT * 64 + lane;
#pragma unroll
                    for (int t = 0; t < MW; t++) R[t] = f[t * 64];
                    p = static_cast<int>(f[MW * 64]);
                }
            }
            int cnt = 0;
#pragma unroll
            for (int t = 0; t < MW; t++) cnt += __popc(R[t]);
            // a level with fewer candidates than the k - p vertices still missing
            // holds no k-clique: drop it
            if (cnt != 0 && cnt < k - p) {
#pragma unroll
                for (int t = 0; t < MW; t++) R[t] = 0u;
                cnt = 0;
            }
            if (cnt != 0) {
                if (STATS) exps += 1;
                // expand the lowest candidate v
                const int v = pop_lowest<MW>(R);
                unsigned int Y[MW];
                load_row<MW>(B + v * STRIDE, Y);
#pragma unroll
                for (int t = 0; t < MW; t++) Y[t] &= R[t];
                int c = 0;
#pragma unroll
                for (int t = 0; t < MW; t++) c += __popc(Y[t]);
                if (STATS) { nodes += 1; wsum += W; }
                if (p + 2 == k) {
                    acc += static_cast<unsigned int>(c);
                } else if (p + 3 == k) {
                    // Y holds the (k-1)-th vertex candidates: count the last
                    // level under it at once instead of descending
                    if (c >= 2) acc += leaf_edges<MW>(Y, B);
                    if (STATS) { nodes += c; wsum += W * c; }
                } else if (c >= k - p - 1) {
                    // descend into Y; save the rest of this level only if it can
                    // still complete a k-clique
                    if (cnt - 1 >= k - p) {
                        unsigned int* f = stk + depth * SLOT * 64 + lane;
#pragma unroll
                        for (int t = 0; t < MW; t++) f[t * 64] = R[t];
                        f[MW * 64] = static_cast<unsigned int>(p);
                        depth++;
                    }
#pragma unroll
                    for (int t = 0; t < MW; t++) R[t] = Y[t];
                    p++;
                }
            }
            if (st + 1 < kInner) {
                bool more = depth > sbase;
#pragma unroll
                for (int t = 0; t < MW; t++) more |= R[t] != 0u;
                if (__ballot(more) == 0ull) break;
            }
        }
    }
    // cliques counted by this walk, weighted by the root's row words (stats only)
    if (STATS) cw += W * (acc - acc_in);
}

// Extract root `slot` of this list into LDS and walk it with rows of the
// smallest supported width that holds its S.  item: a queued subtree of this
// root (path length item_p) instead of the root's own tasks.
template <int MAXW, bool EC, bool PAIR, bool STATS>
__device__ __forceinline__ void run_root(const LaneParams& P, const int* roots, int k, int p0, int slot,
                                         bool helping, const unsigned int* item, int item_p, bool cached, int* ctl, int* S,
                                         unsigned int* B, int* pre, unsigned int* mbox, unsigned int* stk, int* tctr,
                                         int* ttot, unsigned long long lt, unsigned long long& acc,
                                         unsigned long long& nodes, unsigned long long& wsum,
                                         unsigned long long& iters, unsigned long long& exps,
                                         unsigned long long& cw) {
    // cached: S and the rows of this root are still in LDS from the previous walk
    if (!cached) extract_set<1, EC>(roots[slot], P.row_ptr, P.col, P.src, __lane_id(), S, &ctl[1]);
    const int s = ctl[1];
    if (EC && k == 3) {
        if (__lane_id() == 0 && !helping) {
            acc += static_cast<unsigned long long>(s);
            if (STATS) cw += static_cast<unsigned long long>((s + 31) >> 5) * static_cast<unsigned long long>(s);
        }
        return;
    }
#define KC_WALK(MW)                                                                                          \
    walk_root<MW, EC, PAIR, STATS>(P, k, p0, s, slot, helping, item, item_p, !cached, S, B, pre, mbox, stk, tctr, ttot, lt, \
                                   acc, nodes, wsum, iters, exps, cw)
    const int Wr = __builtin_amdgcn_readfirstlane((s + 31) >> 5);
    if constexpr (MAXW >= 32) {
        if (Wr > 16) { KC_WALK(32); return; }
    }
    if constexpr (MAXW >= 16) {
        if (Wr > 8) { KC_WALK(16); return; }
    }
    if constexpr (MAXW >= 8) {
        if (Wr > 6) { KC_WALK(8); return; }
        if (Wr > 4) { KC_WALK(6); return; }
    }
    if constexpr (MAXW >= 4) {
        if (Wr > 3) { KC_WALK(4); return; }
        if (Wr > 2) { KC_WALK(3); return; }
    }
    if constexpr (MAXW >= 2) {
        if (Wr > 1) { KC_WALK(2); return; }
    }
    KC_WALK(1);
#undef KC_WALK
}

// MAXW: bitset words per row of this root list; EC: edge roots; PAIR: pair
// tasks + helping (deep trees on wide roots); STATS: count expanded nodes.
template <int MAXW, bool EC, bool PAIR, bool STATS>
__global__ void __launch_bounds__(64) k_lane(LaneParams P) {
    constexpr int STRIDE = lane_stride(MAXW);
    constexpr int SLOT = MAXW + 1;                  // saved level: R words + p
    extern __shared__ __align__(16) unsigned int lds[];
    const int lane = threadIdx.x & 63;
    const int s_cap = P.s_cap;
    unsigned int* base = lds;
    int* ctl = reinterpret_cast<int*>(base);
    int* S = reinterpret_cast<int*>(base + 16);
    unsigned int* B = base + 16 + s_cap;
    int* pre = reinterpret_cast<int*>(B + s_cap * STRIDE);
    unsigned int* mbox = B + s_cap * STRIDE + (PAIR ? s_cap + 1 : 0);
    unsigned int* stk = mbox + 64 * SLOT;           // [level][slot word][lane]
    const int k = P.k;
    const int p0 = EC ? 3 : 2;
    int list_off = 0;
    for (int j = 0; j < P.list; j++) list_off += P.counts[j];
    const int* roots = P.lists + list_off;
    const int nroots = P.counts[P.list];
    int* tctr = P.task_ctr + list_off;
    int* ttot = P.task_tot + list_off;
    const int nwaves = gridDim.x;                   // one wavefront per block
    const unsigned long long lt = lanemask_lt();
    // hand subtrees between wavefronts only where roots are scarce (under two per
    // wavefront): with many roots the walks balance by themselves and handoff
    // latency would only lengthen the critical path
    const bool steal = PAIR && P.steal && nroots < 2 * nwaves;
    int* q = P.qctl;
    int cur = -1;                                   // root whose S and rows are in LDS

    // an earlier launch of the same call stalled or was canceled: give up at once
    if (P.flags && (ld_acquire(P.flags) & (kFlagStalled | kFlagCanceled))) return;
    if (P.cancel && poll_cancel(P.cancel, P.flags)) return;
    unsigned long long acc = 0, nodes = 0, wsum = 0, iters = 0, exps = 0, idle = 0, cw = 0;
    const unsigned long long t_begin = STATS ? __builtin_amdgcn_s_memrealtime() : 0ull;
    if (steal && lane == 0) atomicAdd(&q[Q_ROOTING], 1);    // in the root phase
    bool helping = steal && P.helper;               // helpers own no roots (and no registry entry)
    int rq = 0, rq_end = 0;                         // claimed, unprocessed root range
    int claims = 0;                                 // root claims since the last cancel poll
    constexpr int RC = PAIR ? 1 : kRootChunk;

    // ---------------------------------------------- root phase
    for (;;) {
        int slot = -1;
        if (!helping) {
            if (rq == rq_end) {
                int r = 0;
                if (lane == 0) r = atomicAdd(P.head, RC);
                r = __shfl(r, 0);
                rq = r < nroots ? r : nroots;
                rq_end = r + RC < nroots ? r + RC : nroots;
            }
            if (rq < rq_end) slot = rq++;
            else if (PAIR) helping = true;
            else break;
        }
        if (PAIR && helping) {
            // join the in-progress root with the most unclaimed pair tasks
            unsigned long long best = 0;
            for (int b0 = 0; b0 < nwaves; b0 += 64) {
                const int e = b0 + lane;
                if (e < nwaves) {
                    const int sl = ld_acquire(&P.active[e]);
                    if (sl >= 0) {
                        const int tot = ld_acquire(&ttot[sl]);
                        const int rem = tot - 1 - ld_acquire(&tctr[sl]);
                        if (tot > 0 && rem > 0) {
                            const unsigned long long key = (static_cast<unsigned long long>(rem) << 32) |
                                                           static_cast<unsigned int>(sl);
                            best = key > best ? key : best;
                        }
                    }
                }
            }
            best = wave_max(best);
            if (best == 0ull) break;
            slot = static_cast<int>(best & 0xffffffffu);
        }
        const int graph = P.gacc ? P.gid[EC ? P.src[roots[slot]] : roots[slot]] : 0;
        run_root<MAXW, EC, PAIR, STATS>(P, roots, k, p0, slot, helping, nullptr, 0, false, ctl, S, B, pre, mbox, stk,
                                        tctr, ttot, lt, acc, nodes, wsum, iters, exps, cw);
        cur = slot;
        if (PAIR && !helping && lane == 0)
            __hip_atomic_store(&P.active[blockIdx.x], -1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (P.gacc) flush_root(P, graph, acc);
        wave_sync_lds();
        if (P.cancel) {
            // a walk that saw the request has marked it; otherwise look at the
            // caller's flag every 64 roots
            int c = 0;
            if (lane == 0) {
                c = (ld_acquire(P.flags) & kFlagCanceled) != 0;
                if (!c && (++claims & 63) == 0 && cancel_requested(P.cancel)) {
                    atomicOr(P.flags, kFlagCanceled);
                    c = 1;
                }
            }
            if (__shfl(c, 0)) break;
        }
    }

    // ---------------------------------------------- queue phase
    // Subtrees that busy wavefronts handed over (see walk_root).  The launch is
    // finished when no wavefront is in the root phase and no queued subtree is
    // unfinished; `pending` counts subtrees from publication to completion, so
    // both reading zero (rooting first) means no work can appear any more.
    if (steal) {
        if (lane == 0) __hip_atomic_fetch_add(&q[Q_ROOTING], -1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        // at most kMaxWaiters wavefronts wait; the others end here and free their
        // compute unit slots for launches that run beside this one.  A waiter
        // leaves only at the end, so handed-over subtrees always find one.
        int stay = 1;
        if (lane == 0 && atomicAdd(&q[Q_HUNGRY], 1) >= kMaxWaiters && !P.helper) {
            atomicAdd(&q[Q_HUNGRY], -1);
            stay = 0;
        }
        stay = __shfl(stay, 0);
        bool hungry = stay != 0;
        unsigned long long sig = ~0ull, t_sig = 0, t_idle = 0;
        bool idling = false;
        int backoff = 0;                            // empty polls in a row (sleep grows with it)
        while (stay) {
            int idx = -1, state = 0;                // state 1: finished, 2: stalled
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
            if (STATS && idling && (idx >= 0 || state != 0)) {
                idle += __builtin_amdgcn_s_memrealtime() - t_idle;
                idling = false;
            }
            if (idx >= 0) {
                if (hungry && lane == 0) atomicAdd(&q[Q_HUNGRY], -1);
                hungry = false;
                backoff = 0;
                // the producer reserved this item and is writing it: wait for its flag
                // the slot reads gen + 1 once the producer of item idx has written it
                int ok = 1, slot = 0, ip = 0;
                const int qs = idx & (kQueueCap - 1);
                const int gen = idx - qs;
                const unsigned int* it = P.qitems + static_cast<size_t>(qs) * kItemWords;
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
                // copy the item into LDS (the pair-task prefix area, unused for a
                // queued subtree) and free the slot for its next producer
                unsigned int* ibuf = reinterpret_cast<unsigned int*>(pre);
                if (lane < 4 + MAXW) ibuf[lane] = ld_acquire(&it[lane]);
                wave_sync_lds();
                if (lane == 0)   // next generation's producer may write the slot
                    __hip_atomic_store(&P.qready[qs], gen + kQueueCap, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                slot = static_cast<int>(ibuf[0]);
                ip = static_cast<int>(ibuf[1]);
                run_root<MAXW, EC, PAIR, STATS>(P, roots, k, p0, slot, true, ibuf, ip, slot == cur, ctl, S, B, pre,
                                                mbox, stk, tctr, ttot, lt, acc, nodes, wsum, iters, exps, cw);
                cur = slot;
                wave_sync_lds();
                if (lane == 0) __hip_atomic_fetch_add(&q[Q_PENDING], -1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                continue;
            }
            if (state == 1) break;
            if (state == 2) {
                if (lane == 0) atomicOr(P.flags, kFlagStalled);
                break;
            }
            if (!hungry && lane == 0) atomicAdd(&q[Q_HUNGRY], 1);
            hungry = true;
            if (STATS && !idling) {
                t_idle = __builtin_amdgcn_s_memrealtime();
                idling = true;
            }
            // back off: 1, 2, 4, .. 32 sleeps of 127 x 64 clocks between polls,
            // so that waiting wavefronts do not crowd the queue words
            if (backoff < 5) backoff++;
            for (int i = 0; i < (1 << backoff); i++) __builtin_amdgcn_s_sleep(127);
        }
        if (hungry && lane == 0) atomicAdd(&q[Q_HUNGRY], -1);
    }

    unsigned long long lo, hi;
    wave_sum_u128(acc, lo, hi);
    if (lane == 0) atomic_add_u128(P.acc, P.acc + 1, lo, hi);
    if (STATS) {
        nodes = wave_sum(nodes);
        wsum = wave_sum(wsum);
        exps = wave_sum(exps);
        cw = wave_sum(cw);
        if (lane == 0) {
            atomicAdd(P.stats, nodes);
            atomicAdd(P.stats + 1, wsum);
            atomicAdd(P.iters, iters);
            atomicAdd(P.iters + 1, exps);
            if (P.cwords) atomicAdd(P.cwords, cw);
            // busy time of this wavefront (queue waits excluded) and the span of
            // the whole grid (100 MHz constant clock): [sum of busy, min start, max end]
            const unsigned long long t_end = __builtin_amdgcn_s_memrealtime();
            atomicAdd(P.timing, t_end - t_begin - idle);
            atomicMin(P.timing + 1, t_begin);
            atomicMax(P.timing + 2, t_end);
        }
    }
}

template <int MAXW, bool EC, bool PAIR>
int launch_lane_t(const LaneParams& base, bool stats, int* grid_out, hipStream_t s) {
    constexpr int SLOT = MAXW + 1;
    LaneParams P = base;
    P.s_cap = 32 * MAXW;
    const int words = 16 + P.s_cap + P.s_cap * lane_stride(MAXW) + (PAIR ? P.s_cap + 1 : 0) + 64 * SLOT +
                      P.levels * SLOT * 64;
    const size_t lds_bytes = static_cast<size_t>(words) * sizeof(unsigned int);
    (void)SLOT;
    if (lds_bytes > 160 * 1024) return KC_EUNSUPPORTED;
    auto kern = stats ? k_lane<MAXW, EC, PAIR, true> : k_lane<MAXW, EC, PAIR, false>;
    if (lds_bytes > 64 * 1024)
        KC_CHECK(hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds_bytes)));
    int occ = 0;
    KC_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, 64, lds_bytes));
    if (occ < 1) return KC_EUNSUPPORTED;
    if (occ > kLaneWavesPerCU) occ = kLaneWavesPerCU;   // the registry holds one entry per wavefront
    if (grid_out) *grid_out = device_cus() * occ;
    kern<<<device_cus() * occ, 64, lds_bytes, s>>>(P);
    KC_CHECK(hipGetLastError());
    return KC_OK;
}

template <int MAXW>
int launch_lane_m(const LaneParams& P, bool ec, bool pair, bool stats, int* g, hipStream_t s) {
    if (ec) return pair ? launch_lane_t<MAXW, true, true>(P, stats, g, s) : launch_lane_t<MAXW, true, false>(P, stats, g, s);
    return pair ? launch_lane_t<MAXW, false, true>(P, stats, g, s) : launch_lane_t<MAXW, false, false>(P, stats, g, s);
}

}  // namespace lanewalk

// Launch of one width list's lane-walk kernel, rows of MAXW words (one
// definition per kc_lane_w<MAXW>.hip).
int lane_launch_w1(const lanewalk::LaneParams& P, bool ec, bool pair, bool stats, int* grid, hipStream_t s);
int lane_launch_w2(const lanewalk::LaneParams& P, bool ec, bool pair, bool stats, int* grid, hipStream_t s);
int lane_launch_w4(const lanewalk::LaneParams& P, bool ec, bool pair, bool stats, int* grid, hipStream_t s);
int lane_launch_w8(const lanewalk::LaneParams& P, bool ec, bool pair, bool stats, int* grid, hipStream_t s);
int lane_launch_w16(const lanewalk::LaneParams& P, bool ec, bool pair, bool stats, int* grid, hipStream_t s);
int lane_launch_w32(const lanewalk::LaneParams& P, bool ec, bool pair, bool stats, int* grid, hipStream_t s);

}  // namespace kc
