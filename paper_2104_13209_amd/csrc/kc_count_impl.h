// Host-side layout shared by the counting sources (not part of the ABI).
#pragma once

#include "kc_internal.h"

namespace kc {

constexpr int kLightCap = 64;          // |S| bound of the light root list
constexpr int kPivBlocksPerCU = 8;     // grid cap of the heavy pivot kernel (sizes its stacks)
constexpr int kLaneWavesPerCU = 32;    // grid cap of the lane-walk kernel (sizes its registry)
constexpr int kWidthLists = 6;         // root lists by bitset words per row: 1, 2, 4, 8, 16, 32
constexpr int kQueueCap = 16384;        // lane walk: ring slots for subtrees handed between wavefronts (power of 2)
constexpr int kItemWords = 36;          // queue item: root slot, path length, 2 spare, 32 words of R
constexpr int kQueueCtlWords = 8;       // per width list: head, tail, pending, rooting, hungry
// subtree queue control words, and its bounds
constexpr int Q_HEAD = 0, Q_TAIL = 1, Q_PENDING = 2, Q_ROOTING = 3, Q_HUNGRY = 4;
constexpr int kMaxWaiters = 256;                            // wavefronts that wait for handed-over work
constexpr unsigned long long kStallTicks = 2000000000ull;   // 20 s at 100 MHz without queue progress
constexpr int kReadySpins = 1 << 22;                        // wait for a reserved item's sequence word
// bits of the CC_FLAGS control word
constexpr int kFlagBigBinom = 1;    // a binomial beyond 128 bits was used
constexpr int kFlagStalled = 2;     // a work queue stopped making progress (no valid count)
constexpr int kFlagCanceled = 4;    // the caller's cancel flag was seen (no valid count)
constexpr int kFlagLocalOverflow = 8;   // a per-vertex count passed 2^64
// handoff thresholds (defaults; kc_opts may lower them for tests)
constexpr int kLaneStealEvery = 16;    // lane walk: wavefront rounds between looks at the subtree queue
constexpr int kLaneStealAfter = 256;   // lane walk: rounds on the current root or subtree before it may hand over
// pivot: tree nodes between looks at the frame queue, and nodes of the current
// root or frame before it may hand over.  A consumer re-extracts the frame's
// root, so only long trees should give work away.  Edge roots with at most 64
// candidates (the light list) are very many short trees: their frames go only
// after 65536 nodes; vertex roots and heavy edge roots after 8192.
constexpr int kPivStealEvery = 64;
constexpr int kPivStealAfter = 8192;
constexpr int kPivStealAfterLightEC = 65536;
// Pivot walks are latency-bound (one wavefront per tree, chains of dependent LDS
// and global accesses), so more wavefronts may wait for handed-over frames than
// in the lane walk: 4 per CU.  Dense-core count-all with a 4096-node first
// handoff (VC / EC, ms): 1500 / 800 with 256 waiters in all, 1110 / 713 at 2 per
// CU, 930 / 665 at 4, 1240 / 775 at 8, 3000 / 1390 at 16 (handoffs and queue
// traffic then outweigh the overlap); 810 / 650 at 4 per CU with 8192.
constexpr int kPivWaitersPerCU = 4;
constexpr int kCancelEvery = 32;       // wavefront rounds (lane walk) or nodes (pivot) between cancel polls
// count lo/hi, light/heavy stats, per width list: nodes, words, iterations,
// expansions, busy, start, end; helper timing (3); per width list: counted
// cliques weighted by row words
constexpr int kAccWords = 9 + 8 * kWidthLists;
constexpr int kAccCwords = 9 + 7 * kWidthLists;

enum CountCtl {
    CC_LIGHT_N = 0,      // light root count
    CC_HEAVY_N = 1,      // heavy root count
    CC_LIGHT_HEAD = 2,   // light queue head
    CC_HEAVY_HEAD = 3,   // heavy queue head
    CC_FLAGS = 4,        // kFlag* bits
    CC_WIDE_N = 5,       // wide root count
    CC_WIDE_HEAD = 6,    // wide queue head
    CC_WN0 = 8,          // width lists: root counts (8..13)
    CC_WC0 = 16,         // width lists: fill cursors (16..21)
    CC_WH0 = 24,         // width lists: queue heads (24..29)
    CC_WORDS = 32
};

// Saved levels a depth-first walk starting at path length `first` may need:
// the last two levels of a path are counted in registers (a node one level
// above the leaves adds the edge count of its candidate set), so levels are
// saved only while the path is shorter than k - 3.
inline int k_levels(int k, int first) {
    const int lv = k - 3 - first;
    return lv < 1 ? 1 : lv;
}

__host__ __device__ constexpr int b_stride_of(int maxw) { return (maxw > 1 && (maxw % 2) == 0) ? maxw + 1 : maxw; }

// Row stride (words) of the lane walk's bitset rows.  Rows of up to 4 words keep
// an odd stride and 32-bit reads (row starts spread over all banks); wider rows
// are padded to a multiple of 4 words and read with 128-bit loads (6 -> 8).
__host__ __device__ constexpr int lane_stride(int w) { return w <= 4 ? b_stride_of(w) : ((w + 3) & ~3); }

// Bitset words per row used for a DAG of this d_max (rows of at most 32 * maxw bits).
inline int maxw_for(int d_max) {
    if (d_max <= 64) return 2;
    if (d_max <= 128) return 4;
    if (d_max <= 256) return 8;
    if (d_max <= 512) return 16;
    return 32;
}

// The on-chip kernels see at most KC_MAX_DMAX out-neighbours per root: longer
// out-rows make their roots wide (kc_wide.hip) and the others skip them.
inline int bit_dmax(int d_max) { return d_max < KC_MAX_DMAX ? d_max : KC_MAX_DMAX; }

// Wide roots: candidate slots and row words (padded to 4) of one wavefront's slab,
// and the slab's words: rows, then per stack level the candidate and branch sets,
// then 4 words of level scalars.
inline int wide_s_cap(int d_max) { return ((d_max + 31) / 32) * 32; }
inline int wide_wcap(int d_max) { return ((wide_s_cap(d_max) / 32) + 3) & ~3; }
inline size_t wide_slab_words(int d_max) {
    const size_t s = static_cast<size_t>(wide_s_cap(d_max)), w = static_cast<size_t>(wide_wcap(d_max));
    return s * w + (s + 2) * (2 * w + 4);
}
constexpr size_t kWideSlabBudget = static_cast<size_t>(2) << 30;   // bytes of wide slabs at most

inline int s_cap_for(int d_max) { return ((d_max + 31) / 32) * 32 > kLightCap ? ((d_max + 31) / 32) * 32 : kLightCap; }

// Words of one pivot stack level: I, P_orig, P_remaining (maxw each) + p, np, nh, pad.
inline int piv_level_words(int maxw) { return 3 * maxw + 4; }

struct CountWs {
    int* ctl;
    unsigned long long* acc;      // [lo, hi, light nodes, words, heavy nodes, words, then per width list nodes, words]
    int* light;
    int* heavy;
    unsigned long long* counts;   // count_all: (binom_n + 1) x {lo, hi}
    unsigned long long* binom;    // (binom_n + 1)^2 x {lo, hi}: C(i, j) at [i * (binom_n + 1) + j]
    unsigned char* big;           // same shape: 1 if C(i, j) needs more than 128 bits
    unsigned int* gstack;         // heavy pivot stacks, one slab per resident wavefront
    int* task_ctr;                // lane walk, pair tasks: claimed tasks per root
    int* task_tot;                // lane walk, pair tasks: total tasks + 1 per root (0 = unpublished)
    int* active;                  // lane walk: root slot owned by each wavefront (-1 = none), main + side
    int* qctl;                    // lane walk, subtree queue: kQueueCtlWords per width list
    int* qready;                  // lane walk, subtree queue: slot sequence words, kQueueCap per width list
    unsigned int* qitems;         // lane walk, subtree queue: kItemWords per slot, main + side
    int* wide;                    // wide roots (d_max > KC_MAX_DMAX only)
    unsigned int* wslabs;         // wide roots: one slab per wavefront
    size_t wslab_words;
    int nwslabs;
    int nactive;
    int binom_n;
    int counts_len;               // entries of counts (sizes 0 .. counts_len - 1)
    size_t slab_words;
    int slabs;
};

inline CountWs carve_count(void* ws, const kc_dag* d, bool pivot, size_t* bytes) {
    Carver c(ws);
    CountWs w{};
    const int nr = d->m > d->n ? d->m : d->n;
    w.ctl = c.take<int>(CC_WORDS);
    w.acc = c.take<unsigned long long>(kAccWords);
    w.light = c.take<int>(static_cast<size_t>(nr > 0 ? nr : 1));
    w.heavy = c.take<int>(static_cast<size_t>(nr > 0 ? nr : 1));
    w.task_ctr = c.take<int>(static_cast<size_t>(nr > 0 ? nr : 1));
    w.task_tot = c.take<int>(static_cast<size_t>(nr > 0 ? nr : 1));
    w.nactive = device_cus() * kLaneWavesPerCU;
    w.active = c.take<int>(2 * static_cast<size_t>(w.nactive));    // main and side stream
    w.qctl = c.take<int>(kQueueCtlWords * kWidthLists);
    w.qready = c.take<int>(static_cast<size_t>(kQueueCap) * kWidthLists);
    w.qitems = c.take<unsigned int>(2 * static_cast<size_t>(kQueueCap) * kItemWords);   // main and side stream
    const int dm = bit_dmax(d->d_max);
    if (pivot) {
        const int s_cap = s_cap_for(dm);
        w.binom_n = s_cap + 2;
        w.counts_len = w.binom_n + 1;
        if (d->d_max > KC_MAX_DMAX && d->d_max + 3 > w.counts_len) w.counts_len = d->d_max + 3;
        const size_t cells = static_cast<size_t>(w.binom_n + 1) * (w.binom_n + 1);
        w.counts = c.take<unsigned long long>(2 * static_cast<size_t>(w.counts_len));
        w.binom = c.take<unsigned long long>(2 * cells);
        w.big = c.take<unsigned char>(cells);
        if (dm > kLightCap) {
            const int maxw = maxw_for(dm);
            w.slab_words = static_cast<size_t>(s_cap + 2) * piv_level_words(maxw);
            w.slabs = device_cus() * kPivBlocksPerCU * 4;
            w.gstack = c.take<unsigned int>(w.slab_words * w.slabs);
        }
    }
    if (d->d_max > KC_MAX_DMAX && d->d_max <= KC_MAX_DMAX_WIDE) {
        w.wide = c.take<int>(static_cast<size_t>(d->n > 0 ? d->n : 1));
        w.wslab_words = wide_slab_words(d->d_max);
        size_t slabs = kWideSlabBudget / (4 * w.wslab_words);
        const size_t most = static_cast<size_t>(device_cus()) * 2;
        if (slabs > most) slabs = most;
        if (slabs < 1) slabs = 1;
        w.nwslabs = static_cast<int>(slabs);
        w.wslabs = c.take<unsigned int>(w.wslab_words * slabs);
    }
    *bytes = c.bytes();
    return w;
}

// Wide roots (kc_wide.hip): counts the cliques whose lowest vertex has more
// than KC_MAX_DMAX out-neighbours, one vertex root per such vertex (the other
// kernels skip these vertices' vertex and edge roots).  mode 0: graph
// orientation with target k (adds to w.acc); 1: pivoting with target k (w.acc);
// 2: pivoting, every size (w.counts).
int wide_launch(const kc_dag* d, int k, int mode, const CountWs& w, const int* cancel, hipStream_t s);

// Launch description for the pivot kernels (kc_pivot.hip).
struct PivLaunch {
    int k;                // clique size (ignored when all)
    bool all;             // count every size
    bool ec;              // edge roots
    bool stats;
    bool steal;           // hand saved frames to idle wavefronts (queue regions 0 and 1)
    int steal_every = 0;                   // 0: the default (kPivStealEvery)
    int steal_after = 0;                   // 0: the default of the root list and scheme
    const int* cancel = nullptr;   // caller's cancel flag (null: none)
    unsigned long long* local = nullptr;   // per-vertex counts of size k (input ids); null: totals
    const int* perm = nullptr;             // DAG id -> input id (local counts)
    int d_max;
    const int* row_ptr;
    const int* col;
    const int* src;
    CountWs w;
};

int pivot_binom_table(const CountWs& w, hipStream_t s);
int pivot_launch(const PivLaunch& L, bool heavy, hipStream_t s);

// Launch description for the lane-walk graph-orientation kernel (kc_lane.hip).
struct LaneLaunch {
    int k;
    bool ec;
    bool pair;            // pair tasks from a global per-root counter + helping
    bool stats;
    int maxw;             // bitset words per row of this list
    int list;             // list index (0..kWidthLists-1)
    const int* row_ptr;
    const int* col;
    const int* src;
    const int* lists;     // all width lists back to back
    const int* counts;    // ctl + CC_WN0
    int* head;            // ctl + CC_WH0 + list
    int* task_ctr;
    int* task_tot;
    int* active;
    bool steal = false;   // hand subtrees to idle wavefronts through a global queue (pair mode)
    bool helper = false;  // join a running launch of this list: help and take queued subtrees only
    int* qctl = nullptr;  // this list's queue control words (zero at launch)
    int* qready = nullptr;  // this list's ring slot sequence words (zero at launch)
    unsigned int* qitems = nullptr;
    int* flags = nullptr;   // CC_FLAGS word: kFlagStalled, kFlagCanceled
    int steal_every = kLaneStealEvery;
    int steal_after = kLaneStealAfter;
    const int* cancel = nullptr;   // caller's cancel flag (null: none)
    unsigned long long* acc;
    unsigned long long* stats_ptr;
    unsigned long long* iters_ptr = nullptr;
    unsigned long long* timing_ptr = nullptr;
    unsigned long long* cwords_ptr = nullptr;   // stats: counted cliques x root row words
    int* grid_out = nullptr;              // receives the launched grid (wavefronts)
    unsigned long long* gacc = nullptr;   // batched: per-graph counters
    const int* gid = nullptr;             // batched: graph of each DAG vertex
};

int lane_launch(const LaneLaunch& L, hipStream_t s);

// On-chip memory a kc_count call keeps resident while it runs (an estimate for
// admission): the LDS bytes of one wavefront of its dominant traversal kernel
// (the widest width list's lane walk, or the heavy pivot kernel) times the
// wavefronts that kernel launches (at most one per root), capped at the device's
// LDS (kc_count.hip).
size_t count_lds_demand(const kc_dag* d, int k, int pivot);
size_t device_lds_bytes();

// Sub-wavefront group walk (k_go, Sec. 3.5) over one width list of a batched
// call, adding each root's count to its graph's counter (kc_count.hip).
struct GoBatchLaunch {
    int k;
    bool ec;
    int list;                  // width list index (bitset words per row = 2^list)
    int group;                 // lanes per group (2 .. 32)
    const int* row_ptr;
    const int* col;
    const int* src;
    const int* lists;          // all width lists back to back
    const int* list_counts;    // ctl + CC_WN0
    int* head;                 // ctl + CC_WH0 + list
    unsigned long long* acc;   // scratch counters of the launch
    int* flags;                // CC_FLAGS word
    unsigned long long* gacc;  // per-graph {lo, hi}
    const int* gid;            // graph of each DAG vertex
};

int go_batch_launch(const GoBatchLaunch& B, hipStream_t s);

// Graph orientation over sorted candidate lists and binary-search
// intersections instead of bitsets (kc_lists.hip; KC_OPT_NO_BITSETS).
int lists_launch(const kc_dag* d, int k, bool ec, const CountWs& w, const int* cancel, hipStream_t s);

// Per-vertex counts by graph orientation (kc_local.hip): zeroes `local` (n
// entries, input ids) and adds every vertex's k-clique count; ctl is the
// count workspace's control block (zero at launch).
int local_orient_launch(const kc_dag* d, int k, bool ec, unsigned long long* local, int* ctl, const int* cancel,
                        hipStream_t s);

// k-clique listing by graph orientation (kc_local.hip): writes up to `cap` rows
// of k input ids into `list` and counts every k-clique into *listed (device,
// zero at launch); ctl is the count workspace's control block (zero at launch).
int list_orient_launch(const kc_dag* d, int k, bool ec, int* list, long long cap, unsigned long long* listed,
                       int* ctl, const int* cancel, hipStream_t s);

// Capture-safe degree orientation (kc_orient.hip).
size_t orient_async_workspace(int n, int nnz);
int orient_degree_async(int n, int nnz, const int* row_ptr, const int* col, int key_bits, int* out_row_ptr,
                        int* out_col, int* out_src, int* out_perm, void* ws, hipStream_t s);

// LDS bytes one lane-walk wavefront needs for a list of `maxw` words per row.
inline size_t lane_lds_bytes(int maxw, int k, bool ec, bool pair) {
    const int s_cap = 32 * maxw;
    const int slot = maxw + 1;
    const int first = (ec ? 3 : 2) + (pair ? 1 : 0);
    const int words = 16 + s_cap + s_cap * lane_stride(maxw) + (pair ? s_cap + 1 : 0) + 64 * slot +
                      k_levels(k, first) * slot * 64;
    return static_cast<size_t>(words) * 4;
}

}  // namespace kc
