// Orientation and CSR rebuild on the GPU (paper Sec. 3.1).
//
// Steps, all on one stream:
//   validate  (optional) sorted, simple, symmetric CSR check
//   key       degree order: key(v) = deg(v)
//             degeneracy order: key(v) = peeling round of v (k-core removal
//             order computed by level-synchronous peeling, one cooperative kernel)
//   sort      stable LSD radix sort of vertex ids by key: the position in the
//             sorted order is the new id, so (key, old id) order is the orientation
//   filter    per vertex, keep neighbours with a larger new id; out-degree
//             histogram, exclusive scan -> row_ptr (the paper's histogram + scan)
//   compact   gather each kept row, sort it by new id, write col and the COO src
#include <hip/hip_cooperative_groups.h>

#include <climits>

#include "kc_internal.h"

namespace cg = cooperative_groups;

namespace kc {
namespace {

constexpr int kBlock = 256;
constexpr int kItems = 8;                       // scan items per thread
constexpr int kTile = kBlock * kItems;          // 2048 elements per scan tile
constexpr int kRowCap = KC_MAX_DMAX;            // rows sorted in LDS up to this length

// Control words in the orientation workspace.
enum Ctl {
    CTL_ERR = 0,       // validation error flag
    CTL_MAXKEY = 1,    // largest sort key
    CTL_DMAX = 2,      // max out-degree
    CTL_DEGEN = 3,     // degeneracy (peel)
    CTL_ROUNDS = 4,    // peel rounds
    CTL_LONG = 5,      // a row longer than kRowCap exists
    CTL_ZEROS = 6,     // zero count of the current radix pass
    CTL_SIZE0 = 8,     // peel frontier sizes, ring of 3 (8, 9, 10)
    CTL_MIN = 11,      // peel level minimum
    CTL_HSIZE0 = 12,   // peel heavy-frontier sizes, ring of 3 (12, 13, 14)
    CTL_CL_SIZE0 = 8,  // colouring: light frontier sizes, ring of 3 (8, 9, 10; not used with the peel)
    CTL_CL_HSIZE0 = 12,// colouring: heavy frontier sizes, ring of 3 (12, 13, 14)
    CTL_AD_LIVE = 16,  // approximate degeneracy: vertices left
    CTL_AD_SUM = 18,   // approximate degeneracy: their degree sum (u64 over words 18, 19)
    CTL_WORDS = 20
};

// ------------------------------------------------------------ validation

// One wave per vertex.  Every index is clamped before use so that the check is
// memory-safe on any input.
__global__ void __launch_bounds__(kBlock) k_validate(int n, int nnz, const int* __restrict__ row_ptr,
                                                    const int* __restrict__ col, int* ctl) {
    const int lane = threadIdx.x & 63;
    const int wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int nwaves = (gridDim.x * blockDim.x) >> 6;
    int bad = 0;
    for (int v = wave; v < n; v += nwaves) {
        int b = row_ptr[v], e = row_ptr[v + 1];
        if (b < 0 || e < b || e > nnz) { bad = 1; continue; }
        if (v == 0 && b != 0) bad = 1;
        if (v == n - 1 && e != nnz) bad = 1;
        for (int j = b + lane; j < e; j += 64) {
            int w = col[j];
            if (w < 0 || w >= n || w == v) { bad = 1; continue; }
            if (j > b && col[j - 1] >= w) bad = 1;
            int lo = row_ptr[w], hi = row_ptr[w + 1];
            lo = lo < 0 ? 0 : (lo > nnz ? nnz : lo);
            hi = hi < lo ? lo : (hi > nnz ? nnz : hi);
            while (lo < hi) {
                int mid = lo + ((hi - lo) >> 1);
                if (col[mid] < v) lo = mid + 1; else hi = mid;
            }
            int ehi = row_ptr[w + 1];
            ehi = ehi > nnz ? nnz : ehi;
            if (lo >= ehi || col[lo] != v) bad = 1;
        }
    }
    if (__ballot(bad) && lane == 0) atomicOr(&ctl[CTL_ERR], 1);
}

// --------------------------------------------------------------- keys

__global__ void __launch_bounds__(kBlock) k_degree_key(int n, const int* __restrict__ row_ptr,
                                                      int* key, int* val, int* ctl) {
    int mx = 0;
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        int d = row_ptr[v + 1] - row_ptr[v];
        key[v] = d;
        val[v] = v;
        mx = d > mx ? d : mx;
    }
    mx = wave_max(mx);
    if ((threadIdx.x & 63) == 0) atomicMax(&ctl[CTL_MAXKEY], mx);
}

// Appends the flagged lanes' values to list[] with one atomic per wavefront.
__device__ __forceinline__ void append_wave(bool flag, int v, int* list, int* size, int lane) {
    const unsigned long long m = __ballot(flag);
    if (m == 0ull) return;
    int base = 0;
    if (lane == 0) base = atomicAdd(size, __popcll(m));
    base = __shfl(base, 0);
    if (flag) list[base + __popcll(m & lanemask_lt())] = v;
}

// Frontier of one peeling round, split by row length: light vertices (rows of
// at most kHeavyRow entries) are walked by one wavefront each, the rows of heavy
// vertices are cut into 64-entry chunks that all wavefronts share.
constexpr int kHeavyRow = 128;
struct Frontier {
    int* light;
    int* heavy;
    int* nlight;
    int* nheavy;
};

// Appends flagged vertices to the light or heavy list by row length.
__device__ __forceinline__ void append_split(bool flag, int v, const int* __restrict__ row_ptr, const Frontier& f,
                                             int lane) {
    bool heavy = false;
    if (flag) heavy = row_ptr[v + 1] - row_ptr[v] > kHeavyRow;
    append_wave(flag && !heavy, v, f.light, f.nlight, lane);
    append_wave(flag && heavy, v, f.heavy, f.nheavy, lane);
}

// One entry of the row being peeled: a live neighbour loses one degree and joins
// the next frontier when it drops to the level c.  A stale read of a vertex
// removed earlier only decrements a dead degree, which never equals c + 1.
__device__ __forceinline__ void peel_entry(int j, int e, int c, const int* __restrict__ row_ptr,
                                           const int* __restrict__ col, int* deg, const int* rnd,
                                           const Frontier& nx, int lane) {
    bool hit = false;
    int w = 0;
    if (j < e) {
        w = col[j];
        if (ld_acquire(&rnd[w]) < 0) hit = atomicSub(&deg[w], 1) == c + 1;
    }
    append_split(hit, w, row_ptr, nx, lane);
}

// One peeling round: the frontier's vertices get round r and their live
// neighbours lose one degree each.  Light vertices: wavefront `wave` of nwaves
// takes entries wave, wave + nwaves, ...  Heavy vertices, 64 at a time: every
// wavefront reads their row lengths, numbers the 64-entry chunks of all their
// rows, and takes chunks wave, wave + nwaves, ...
__device__ __forceinline__ void peel_round(int r, int c, const int* cur, int fsize, const int* hcur, int hsize,
                                           const Frontier& nx, const int* __restrict__ row_ptr,
                                           const int* __restrict__ col, int* deg, int* rnd, int wave, int nwaves,
                                           int lane) {
    for (int fi = wave; fi < fsize; fi += nwaves) {
        const int v = ld_acquire(&cur[fi]);
        if (lane == 0) rnd[v] = r;
        const int b = row_ptr[v], e = row_ptr[v + 1];
        for (int j0 = b; j0 < e; j0 += 64) peel_entry(j0 + lane, e, c, row_ptr, col, deg, rnd, nx, lane);
    }
    for (int h0 = 0; h0 < hsize; h0 += 64) {
        const int hi = h0 + lane;
        int v = 0, b = 0, e = 0, nch = 0;
        if (hi < hsize) {
            v = ld_acquire(&hcur[hi]);
            b = row_ptr[v];
            e = row_ptr[v + 1];
            nch = (e - b + 63) >> 6;
            if (wave == 0) rnd[v] = r;
        }
        int incl = nch;                          // inclusive prefix of chunk counts
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int y = __shfl_up(incl, off, 64);
            if (lane >= off) incl += y;
        }
        const int excl = incl - nch;
        const int total = __shfl(incl, 63);
        for (int q = wave; q < total; q += nwaves) {
            // owner: the last lane whose exclusive prefix is <= q
            const int owner = __popcll(__ballot(hi < hsize && excl <= q)) - 1;
            const int ob = __shfl(b, owner), oe = __shfl(e, owner), ox = __shfl(excl, owner);
            peel_entry(ob + (q - ox) * 64 + lane, oe, c, row_ptr, col, deg, rnd, nx, lane);
        }
    }
}

// Degeneracy order by level-synchronous peeling (the paper only states that its
// k-core decomposition runs on the GPU; this schedule is ours).
//
// Level c starts when no live vertex has degree <= c - 1; its first frontier is
// every live vertex of degree <= c.  Each round removes the whole frontier
// (rnd[v] = round), decrements live neighbours, and a neighbour whose degree
// falls from c + 1 to c joins the next frontier.  When a round leaves an empty
// frontier the next level is the minimum live degree.  A vertex removed in round
// r at level c had at most c live neighbours at the start of round r, and its
// out-neighbours under the (round, id) order are among them, so the out-degree
// is bounded by the degeneracy (the largest level).
//
// One pass collects both the vertices of degree <= c + 1 and the minimum live
// degree, since the next level is almost always c + 1; a second pass runs only
// when no live vertex has that degree.  Frontier appends take one atomic per
// wavefront.
__global__ void __launch_bounds__(kBlock) k_peel(int n, const int* __restrict__ row_ptr,
                                                const int* __restrict__ col, int* deg, int* rnd,
                                                int* fr0, int* fr1, int* hf0, int* hf1, int* val, int* ctl) {
    cg::grid_group grid = cg::this_grid();
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    const int nth = gridDim.x * blockDim.x;
    const int lane = threadIdx.x & 63;
    const int wave = tid >> 6;
    const int nwaves = nth >> 6;

    for (int v = tid; v < n; v += nth) {
        deg[v] = row_ptr[v + 1] - row_ptr[v];
        rnd[v] = -1;
        val[v] = v;
    }
    if (tid == 0) {
        ctl[CTL_SIZE0] = ctl[CTL_SIZE0 + 1] = ctl[CTL_SIZE0 + 2] = 0;
        ctl[CTL_HSIZE0] = ctl[CTL_HSIZE0 + 1] = ctl[CTL_HSIZE0 + 2] = 0;
        ctl[CTL_MIN] = INT_MAX;
    }
    grid.sync();

    int removed = 0, r = 0, c = -1, degen = 0;
    while (removed < n) {
        const int* cur = (r & 1) ? fr1 : fr0;
        const int* hcur = (r & 1) ? hf1 : hf0;
        const Frontier nx{(r & 1) ? fr0 : fr1, (r & 1) ? hf0 : hf1, &ctl[CTL_SIZE0 + (r + 1) % 3],
                          &ctl[CTL_HSIZE0 + (r + 1) % 3]};
        const int fsize = ld_acquire(&ctl[CTL_SIZE0 + r % 3]);
        const int hsize = ld_acquire(&ctl[CTL_HSIZE0 + r % 3]);
        if (fsize + hsize == 0) {
            // Level change, as an empty round r: the next frontier is collected
            // into the next lists (no block reads those while others may still be
            // reading csize above), then round r + 1 peels it.  One pass takes
            // the live vertices of degree <= c + 1 and the minimum live degree.
            if (tid == 0) ctl[CTL_SIZE0 + (r + 2) % 3] = ctl[CTL_HSIZE0 + (r + 2) % 3] = 0;
            int mn = INT_MAX;
            for (int b0 = tid - lane; b0 < n; b0 += nth) {
                const int v = b0 + lane;
                bool in = false;
                if (v < n && ld_acquire(&rnd[v]) < 0) {
                    const int d = ld_acquire(&deg[v]);
                    mn = d < mn ? d : mn;
                    in = d <= c + 1;
                }
                append_split(in, v, row_ptr, nx, lane);
            }
            mn = wave_min(mn);
            if (lane == 0 && mn != INT_MAX) atomicMin(&ctl[CTL_MIN], mn);
            grid.sync();
            if (ld_acquire(nx.nlight) + ld_acquire(nx.nheavy) > 0) {
                c = c + 1;          // the minimum live degree is c + 1
            } else {
                c = ld_acquire(&ctl[CTL_MIN]);
                for (int b0 = tid - lane; b0 < n; b0 += nth) {
                    const int v = b0 + lane;
                    const bool in = v < n && ld_acquire(&rnd[v]) < 0 && ld_acquire(&deg[v]) <= c;
                    append_split(in, v, row_ptr, nx, lane);
                }
                grid.sync();
            }
            if (tid == 0) ctl[CTL_MIN] = INT_MAX;   // every read of it is behind the last barrier
            degen = c > degen ? c : degen;
            r++;
            continue;
        }
        if (tid == 0) ctl[CTL_SIZE0 + (r + 2) % 3] = ctl[CTL_HSIZE0 + (r + 2) % 3] = 0;
        peel_round(r, c, cur, fsize, hcur, hsize, nx, row_ptr, col, deg, rnd, wave, nwaves, lane);
        removed += fsize + hsize;
        r++;
        grid.sync();
    }
    if (tid == 0) {
        ctl[CTL_DEGEN] = degen;
        ctl[CTL_ROUNDS] = r;
        ctl[CTL_MAXKEY] = r > 0 ? r - 1 : 0;
    }
}

// ------------------------------------------------------- block-level scan

// Exclusive scan of one int per thread across the block; returns the block total
// through *total.  All threads of the block must call it.
__device__ int block_exclusive_scan(int x, int* total, int* sh /* >= kBlock/64 + 1 */) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int inc = x;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        int y = __shfl_up(inc, off, 64);
        if (lane >= off) inc += y;
    }
    if (lane == 63) sh[w] = inc;
    __syncthreads();
    if (threadIdx.x == 0) {
        int run = 0;
        for (int i = 0; i < kBlock / 64; i++) {
            int t = sh[i];
            sh[i] = run;
            run += t;
        }
        sh[kBlock / 64] = run;
    }
    __syncthreads();
    int res = inc - x + sh[w];
    *total = sh[kBlock / 64];
    __syncthreads();
    return res;
}

// --------------------------------------------------------- exclusive scan

// Pass 1: per-tile sums.  mode 0: sum of in[]; mode 1: count of radix zeros.
// ------------------------------------------- approximate degeneracy order

// A relaxation of k-core peeling (an orientation criterion named in Sec. 2;
// the approximate peeling of ARB-COUNT with eps = 1/10): in rounds r = 0, 1,
// ..., with L vertices left of total current degree D, every remaining vertex
// of degree at most 1.1 D / L (10 deg L <= 11 D, exact in integers) leaves in
// round r; afterwards its remaining neighbours lose one degree each.  The round
// is the sort key, ties by id.  Rounds end when no vertex is left (each removes
// at least one: the smallest degree is at most the average).

__global__ void __launch_bounds__(kBlock) k_ad_init(int n, const int* __restrict__ row_ptr, int* deg, int* rnd,
                                                   int* val) {
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        deg[v] = row_ptr[v + 1] - row_ptr[v];
        rnd[v] = -1;
        val[v] = v;
    }
}

// L and D of the vertices still present.
__global__ void __launch_bounds__(kBlock) k_ad_sum(int n, const int* __restrict__ deg, const int* __restrict__ rnd,
                                                  int* ctl) {
    const int lane = threadIdx.x & 63;
    int live = 0;
    unsigned long long dsum = 0;
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        if (rnd[v] < 0) {
            live++;
            dsum += static_cast<unsigned long long>(deg[v]);
        }
    }
    live = wave_sum(live);
    dsum = wave_sum(dsum);
    if (lane == 0 && live) {
        atomicAdd(&ctl[CTL_AD_LIVE], live);
        atomicAdd(reinterpret_cast<unsigned long long*>(ctl + CTL_AD_SUM), dsum);
    }
}

__global__ void __launch_bounds__(kBlock) k_ad_mark(int n, int r, const int* __restrict__ deg, int* rnd,
                                                   const int* __restrict__ ctl) {
    const long long L = ctl[CTL_AD_LIVE];
    const long long D = static_cast<long long>(*reinterpret_cast<const unsigned long long*>(ctl + CTL_AD_SUM));
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x)
        if (rnd[v] < 0 && 10 * static_cast<long long>(deg[v]) * L <= 11 * D) rnd[v] = r;
}

// One wavefront per vertex that left in round r: its remaining neighbours lose
// one degree each.
__global__ void __launch_bounds__(kBlock) k_ad_dec(int n, int r, const int* __restrict__ row_ptr,
                                                  const int* __restrict__ col, int* deg,
                                                  const int* __restrict__ rnd) {
    const int lane = threadIdx.x & 63;
    const int wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int nwaves = (gridDim.x * blockDim.x) >> 6;
    for (int v = wave; v < n; v += nwaves) {
        if (rnd[v] != r) continue;
        for (int j = row_ptr[v] + lane; j < row_ptr[v + 1]; j += 64) {
            const int w = col[j];
            if (rnd[w] < 0) atomicSub(&deg[w], 1);
        }
    }
}

// ---------------------------------------------------------- colouring order

// Graph colouring as an orientation criterion (Sec. 2 names it): vertices get
// the greedy first-fit colour in decreasing order of a pseudo-random priority
// (SplitMix64's output for the vertex id; the output function is a bijection, so
// priorities never tie), and the order is (colour, id); adjacent vertices differ
// in colour, so every edge goes from its lower colour to its higher one.
//
// The sequential greedy colouring is reproduced in Jones-Plassmann rounds kept
// as a countdown: hp[v] counts v's neighbours of higher priority that are not
// coloured yet, a vertex is coloured in the round after its count reaches zero
// (the first round for counts that start at zero), and then decrements its
// lower-priority neighbours.  Each vertex's colour depends only on its
// higher-priority neighbours, all coloured in earlier rounds, so the result is
// the greedy one and the total work is O(m) over however many rounds (the
// longest decreasing-priority path: 943 on the 1M-vertex power-law graph).

__device__ __forceinline__ unsigned long long colour_priority(int v) {
    unsigned long long z = static_cast<unsigned long long>(v) + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Frontiers are split by degree: a light vertex (degree <= kClHeavy) is coloured
// by one wavefront, a heavy one by a whole block, because the rounds are serial
// and almost every one of them holds a hub of thousands of neighbours.
constexpr int kClHeavy = 512;

struct ClFront {
    int* light;        // this round's light vertices
    int* heavy;        // and heavy ones
    int* next_light;   // the next round's
    int* next_heavy;
};

__device__ __forceinline__ void cl_append(int u, const int* row_ptr, const ClFront& f, int* ctl, int r) {
    if (row_ptr[u + 1] - row_ptr[u] > kClHeavy)
        f.next_heavy[atomicAdd(&ctl[CTL_CL_HSIZE0 + (r + 1) % 3], 1)] = u;
    else
        f.next_light[atomicAdd(&ctl[CTL_CL_SIZE0 + (r + 1) % 3], 1)] = u;
}

// One wavefront per vertex: hp[v] = higher-priority neighbours; the vertices
// with none form round 0's frontier (sizes in ring slot 0).
__global__ void __launch_bounds__(kBlock) k_cl_init(int n, const int* __restrict__ row_ptr,
                                                   const int* __restrict__ col, int* hp, int* val, ClFront f,
                                                   int* ctl) {
    const int lane = threadIdx.x & 63;
    const int wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int nwaves = (gridDim.x * blockDim.x) >> 6;
    for (int v = wave; v < n; v += nwaves) {
        const unsigned long long pv = colour_priority(v);
        int c = 0;
        for (int j = row_ptr[v] + lane; j < row_ptr[v + 1]; j += 64)
            c += colour_priority(col[j]) > pv;
        c = wave_sum(c);
        if (lane == 0) {
            hp[v] = c;
            val[v] = v;
            if (c == 0) cl_append(v, row_ptr, f, ctl, -1);
        }
    }
}

// Colour v with the T threads of a wavefront (T = 64, sync = wave_sync_lds) or a
// block (T = kBlock, sync = __syncthreads), t = the thread's index among them:
// first fit over the colours of v's higher-priority neighbours in windows of
// 1024 (an LDS bitmap; every wavefront reads the whole bitmap, so all of them
// find the same colour), then count down the lower-priority neighbours.  The
// neighbour loops keep four loads in flight per thread.
template <int T, typename Sync>
__device__ __forceinline__ int cl_colour_vertex(int v, int t, unsigned int* used, const int* __restrict__ row_ptr,
                                                const int* __restrict__ col, int* hp, int* colour, const ClFront& f,
                                                int* ctl, int r, Sync sync) {
    constexpr int U = 4;
    const int lane = threadIdx.x & 63;
    const unsigned long long pv = colour_priority(v);
    const int b = row_ptr[v], e = row_ptr[v + 1];
    int c = -1;
    for (int base = 0; c < 0; base += 1024) {
        if (t < 32) used[t] = 0u;
        sync();
        for (int j0 = b + t; j0 < e; j0 += U * T) {
            int u[U];
#pragma unroll
            for (int q = 0; q < U; q++) u[q] = j0 + q * T < e ? col[j0 + q * T] : -1;
            int cu[U];
#pragma unroll
            for (int q = 0; q < U; q++) cu[q] = u[q] >= 0 && colour_priority(u[q]) > pv ? colour[u[q]] - base : -1;
#pragma unroll
            for (int q = 0; q < U; q++)
                if (cu[q] >= 0 && cu[q] < 1024) atomicOr(&used[cu[q] >> 5], 1u << (cu[q] & 31));
        }
        sync();
        const unsigned int free_bits = lane < 32 ? ~used[lane] : 0u;
        const unsigned long long m = __ballot(free_bits != 0u);
        if (m) {
            const int w = __ffsll(static_cast<long long>(m)) - 1;
            const unsigned int fw =
                static_cast<unsigned int>(__builtin_amdgcn_readlane(static_cast<int>(free_bits), w));
            c = base + 32 * w + __ffs(static_cast<int>(fw)) - 1;
        }
        sync();
    }
    if (t == 0) colour[v] = c;
    for (int j0 = b + t; j0 < e; j0 += U * T) {
        int u[U];
#pragma unroll
        for (int q = 0; q < U; q++) u[q] = j0 + q * T < e ? col[j0 + q * T] : -1;
        bool z[U];
#pragma unroll
        for (int q = 0; q < U; q++) z[q] = u[q] >= 0 && colour_priority(u[q]) < pv && atomicSub(&hp[u[q]], 1) == 1;
#pragma unroll
        for (int q = 0; q < U; q++)
            if (z[q]) cl_append(u[q], row_ptr, f, ctl, r);
    }
    return c;
}

// Round r: colour this round's frontier and build the next one.  Sizes live in
// rings of three slots (light: CTL_CL_SIZE0, heavy: CTL_CL_HSIZE0): this round
// reads slot r % 3, appends to slot (r + 1) % 3 (cleared by round r - 1) and
// clears slot (r + 2) % 3, which only the finished round r - 1 read.  A fixed
// grid strides over the frontier (blocks over the heavy list, then wavefronts
// over the light one), so the host launches rounds without reading sizes back.
__global__ void __launch_bounds__(kBlock) k_cl_round(int r, ClFront f, const int* __restrict__ row_ptr,
                                                    const int* __restrict__ col, int* hp, int* colour, int* ctl) {
    __shared__ unsigned int used_all[kBlock / 64][32];
    const int lane = threadIdx.x & 63;
    const int count = ctl[CTL_CL_SIZE0 + r % 3];
    const int hcount = ctl[CTL_CL_HSIZE0 + r % 3];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        ctl[CTL_CL_SIZE0 + (r + 2) % 3] = ctl[CTL_CL_HSIZE0 + (r + 2) % 3] = 0;
        if (count + hcount > 0) atomicMax(&ctl[CTL_ROUNDS], r + 1);
    }
    int mx = 0;
    for (int h = blockIdx.x; h < hcount; h += gridDim.x) {
        const int c = cl_colour_vertex<kBlock>(f.heavy[h], threadIdx.x, used_all[0], row_ptr, col, hp, colour, f,
                                               ctl, r, [] { __syncthreads(); });
        mx = c > mx ? c : mx;
    }
    const int wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int nwaves = (gridDim.x * blockDim.x) >> 6;
    for (int i = wave; i < count; i += nwaves) {
        const int c = cl_colour_vertex<64>(f.light[i], lane, used_all[threadIdx.x >> 6], row_ptr, col, hp, colour, f,
                                           ctl, r, [] { wave_sync_lds(); });
        mx = c > mx ? c : mx;
    }
    if (lane == 0 && mx > 0) atomicMax(&ctl[CTL_MAXKEY], mx);
}

__global__ void __launch_bounds__(kBlock) k_tile_sum(int count, const int* __restrict__ in, int bit,
                                                    int mode, int* tile_sum) {
    __shared__ int sh[kBlock / 64 + 1];
    const int base = blockIdx.x * kTile + threadIdx.x * kItems;
    int s = 0;
#pragma unroll
    for (int i = 0; i < kItems; i++) {
        int idx = base + i;
        if (idx < count) s += mode == 0 ? in[idx] : (((in[idx] >> bit) & 1) == 0);
    }
    int tot;
    block_exclusive_scan(s, &tot, sh);
    if (threadIdx.x == 0) tile_sum[blockIdx.x] = tot;
}

// Pass 2: exclusive scan of the tile sums by one block; total into *total.
__global__ void __launch_bounds__(kBlock) k_scan_tiles(int ntiles, int* tile_sum, int* total) {
    __shared__ int sh[kBlock / 64 + 1];
    int carry = 0;
    for (int base = 0; base < ntiles; base += kBlock) {
        int idx = base + threadIdx.x;
        int x = idx < ntiles ? tile_sum[idx] : 0;
        int tot;
        int ex = block_exclusive_scan(x, &tot, sh);
        if (idx < ntiles) tile_sum[idx] = ex + carry;
        carry += tot;
    }
    if (threadIdx.x == 0) *total = carry;
}

// Pass 3 (mode 0): out[i] = exclusive prefix of in[] (+ tile offset); out[count]
// = total.
__global__ void __launch_bounds__(kBlock) k_scan_apply(int count, const int* __restrict__ in,
                                                      const int* __restrict__ tile_off,
                                                      const int* __restrict__ total, int* out) {
    __shared__ int sh[kBlock / 64 + 1];
    const int base = blockIdx.x * kTile + threadIdx.x * kItems;
    int v[kItems];
    int s = 0;
#pragma unroll
    for (int i = 0; i < kItems; i++) {
        int idx = base + i;
        v[i] = idx < count ? in[idx] : 0;
        s += v[i];
    }
    int tot;
    int run = block_exclusive_scan(s, &tot, sh) + tile_off[blockIdx.x];
#pragma unroll
    for (int i = 0; i < kItems; i++) {
        int idx = base + i;
        if (idx < count) out[idx] = run;
        run += v[i];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) out[count] = *total;
}

// Pass 3 (radix): stable split on `bit`: zeros keep their order at the front,
// ones keep their order after all zeros.
__global__ void __launch_bounds__(kBlock) k_radix_scatter(int count, int bit, const int* __restrict__ kin,
                                                         const int* __restrict__ vin,
                                                         const int* __restrict__ tile_off,
                                                         const int* __restrict__ zeros, int* kout,
                                                         int* vout) {
    __shared__ int sh[kBlock / 64 + 1];
    const int base = blockIdx.x * kTile + threadIdx.x * kItems;
    int k[kItems];
    int s = 0;
#pragma unroll
    for (int i = 0; i < kItems; i++) {
        int idx = base + i;
        k[i] = idx < count ? kin[idx] : 0;
        s += idx < count ? (((k[i] >> bit) & 1) == 0) : 0;
    }
    int tot;
    int zb = block_exclusive_scan(s, &tot, sh) + tile_off[blockIdx.x];
    const int nz = *zeros;
#pragma unroll
    for (int i = 0; i < kItems; i++) {
        int idx = base + i;
        if (idx < count) {
            int one = (k[i] >> bit) & 1;
            int pos = one ? nz + (idx - zb) : zb;
            kout[pos] = k[i];
            vout[pos] = vin[idx];
            zb += one ? 0 : 1;
        }
    }
}

// --------------------------------------------------------- filter, compact

__global__ void __launch_bounds__(kBlock) k_rank(int n, const int* __restrict__ perm, int* rank) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        rank[perm[i]] = i;
}

// Out-degree of new vertex i: neighbours of perm[i] with a larger new id.
__global__ void __launch_bounds__(kBlock) k_outdeg(int n, const int* __restrict__ row_ptr,
                                                  const int* __restrict__ col, const int* __restrict__ perm,
                                                  const int* __restrict__ rank, int* outdeg, int* ctl) {
    const int lane = threadIdx.x & 63;
    const int wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int nwaves = (gridDim.x * blockDim.x) >> 6;
    int mx = 0;
    for (int i = wave; i < n; i += nwaves) {
        int v = perm[i];
        int b = row_ptr[v], e = row_ptr[v + 1];
        int cnt = 0;
        for (int j = b + lane; j < e; j += 64) cnt += rank[col[j]] > i;
        cnt = wave_sum(cnt);
        if (lane == 0) outdeg[i] = cnt;
        mx = cnt > mx ? cnt : mx;
    }
    if (lane == 0) atomicMax(&ctl[CTL_DMAX], mx);
}

// Gather row i's kept neighbours (as new ids) into LDS, then place each at its
// rank within the row (count of smaller entries): col[] rows come out sorted.
// Rows longer than kRowCap go to tmp[] unsorted and are finished by
// k_sort_long_rows.
__global__ void __launch_bounds__(kBlock) k_fill(int n, const int* __restrict__ row_ptr,
                                                const int* __restrict__ col, const int* __restrict__ perm,
                                                const int* __restrict__ rank,
                                                const int* __restrict__ dag_ptr, int* dag_col, int* dag_src,
                                                int* tmp, int* ctl) {
    __shared__ int rows[kBlock / 64][kRowCap];
    const int lane = threadIdx.x & 63;
    const int wslot = threadIdx.x >> 6;
    const int wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int nwaves = (gridDim.x * blockDim.x) >> 6;
    int* row = rows[wslot];
    for (int i = wave; i < n; i += nwaves) {
        const int base = dag_ptr[i];
        const int len = dag_ptr[i + 1] - base;
        if (len == 0) continue;
        const bool in_lds = len <= kRowCap;
        int* dst = in_lds ? row : tmp + base;
        int v = perm[i];
        int b = row_ptr[v], e = row_ptr[v + 1];
        int pos = 0;
        for (int j0 = b; j0 < e; j0 += 64) {
            int j = j0 + lane;
            int r = j < e ? rank[col[j]] : -1;
            bool keep = r > i;
            unsigned long long mask = __ballot(keep);
            if (keep) dst[pos + __popcll(mask & lanemask_lt())] = r;
            pos += __popcll(mask);
        }
        if (in_lds) {
            wave_sync_lds();
            for (int t = lane; t < len; t += 64) {
                int x = row[t];
                int below = 0;
                for (int q = 0; q < len; q++) below += row[q] < x;
                dag_col[base + below] = x;
                dag_src[base + below] = i;
            }
            wave_sync_lds();
        } else if (lane == 0) {
            atomicOr(&ctl[CTL_LONG], 1);
        }
    }
}

// One block per row longer than kRowCap: rows up to kLongSortCap entries are
// bitonic-sorted in LDS (entries are distinct new ids; the padding is INT_MAX);
// longer ones place each entry at its rank, counted over the row in global memory.
constexpr int kLongSortCap = 8192;

__global__ void __launch_bounds__(kBlock) k_sort_long_rows(int n, const int* __restrict__ dag_ptr,
                                                          const int* __restrict__ tmp, int* dag_col,
                                                          int* dag_src) {
    __shared__ int buf[kLongSortCap];
    for (int i = blockIdx.x; i < n; i += gridDim.x) {
        const int base = dag_ptr[i];
        const int len = dag_ptr[i + 1] - base;
        if (len <= kRowCap) continue;
        const int* row = tmp + base;
        if (len <= kLongSortCap) {
            int p = 1;
            while (p < len) p <<= 1;
            for (int t = threadIdx.x; t < p; t += kBlock) buf[t] = t < len ? row[t] : INT_MAX;
            __syncthreads();
            for (int k = 2; k <= p; k <<= 1) {
                for (int j = k >> 1; j > 0; j >>= 1) {
                    for (int t = threadIdx.x; t < p; t += kBlock) {
                        const int o = t ^ j;
                        if (o > t) {
                            const int x = buf[t], y = buf[o];
                            if ((x > y) == ((t & k) == 0)) {
                                buf[t] = y;
                                buf[o] = x;
                            }
                        }
                    }
                    __syncthreads();
                }
            }
            for (int t = threadIdx.x; t < len; t += kBlock) {
                dag_col[base + t] = buf[t];
                dag_src[base + t] = i;
            }
            __syncthreads();
        } else {
            for (int t = threadIdx.x; t < len; t += kBlock) {
                const int x = row[t];
                int below = 0;
                for (int q = 0; q < len; q++) below += row[q] < x;
                dag_col[base + below] = x;
                dag_src[base + below] = i;
            }
        }
    }
}

struct OrientWs {
    int *ctl, *key_a, *val_a, *key_b, *val_b, *rank, *outdeg, *tiles, *rnd, *fr0, *fr1, *hf0, *hf1, *tmp;
};

OrientWs carve(void* ws, int n, int nnz, size_t* bytes) {
    Carver c(ws);
    OrientWs w;
    size_t nn = static_cast<size_t>(n > 0 ? n : 1);
    size_t m = static_cast<size_t>(nnz / 2 > 0 ? nnz / 2 : 1);
    int ntiles = div_up(static_cast<long long>(n) + 1, kTile) + 1;
    w.ctl = c.take<int>(CTL_WORDS);
    w.key_a = c.take<int>(nn);
    w.val_a = c.take<int>(nn);
    w.key_b = c.take<int>(nn);
    w.val_b = c.take<int>(nn);
    w.rank = c.take<int>(nn);
    w.outdeg = c.take<int>(nn + 1);
    w.tiles = c.take<int>(static_cast<size_t>(ntiles));
    w.rnd = c.take<int>(nn);
    w.fr0 = c.take<int>(nn);
    w.fr1 = c.take<int>(nn);
    w.hf0 = c.take<int>(nn);
    w.hf1 = c.take<int>(nn);
    w.tmp = c.take<int>(m);
    *bytes = c.bytes();
    return w;
}

int grid_for_waves(long long items_per_wave_units) {
    long long blocks = (items_per_wave_units + (kBlock / 64) - 1) / (kBlock / 64);
    long long cap = static_cast<long long>(device_cus()) * 16;
    if (blocks > cap) blocks = cap;
    return static_cast<int>(blocks < 1 ? 1 : blocks);
}

int grid_for_threads(long long n) {
    long long blocks = (n + kBlock - 1) / kBlock;
    long long cap = static_cast<long long>(device_cus()) * 16;
    if (blocks > cap) blocks = cap;
    return static_cast<int>(blocks < 1 ? 1 : blocks);
}

// out[0..count] = exclusive prefix sums of in[0..count) with out[count] = total.
int exclusive_scan(int count, const int* in, int* out, int* tiles, int* total, hipStream_t s) {
    int ntiles = div_up(count, kTile);
    if (ntiles < 1) ntiles = 1;
    k_tile_sum<<<ntiles, kBlock, 0, s>>>(count, in, 0, 0, tiles);
    k_scan_tiles<<<1, kBlock, 0, s>>>(ntiles, tiles, total);
    k_scan_apply<<<ntiles, kBlock, 0, s>>>(count, in, tiles, total, out);
    KC_CHECK(hipGetLastError());
    return KC_OK;
}

__global__ void __launch_bounds__(kBlock) k_zero(int* p, int count) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) p[i] = 0;
}

__global__ void __launch_bounds__(kBlock) k_copy(int* dst, const int* src, int count) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) dst[i] = src[i];
}

}  // namespace

size_t orient_async_workspace(int n, int nnz) {
    size_t bytes = 0;
    carve(nullptr, n, nnz, &bytes);
    return bytes;
}

// Degree-order orientation with no host synchronisation (every launch size is
// known on the host: `key_bits` bounds the bit length of the largest degree), so
// it can be captured in a HIP graph.  Writes row_ptr, col, src, perm; the max
// out-degree stays on the device (ws control word), unread.
int orient_degree_async(int n, int nnz, const int* row_ptr, const int* col, int key_bits, int* out_row_ptr,
                        int* out_col, int* out_src, int* out_perm, void* ws, hipStream_t s) {
    size_t need = 0;
    OrientWs w = carve(ws, n, nnz, &need);
    if (n <= 0) return KC_EINVAL;
    k_zero<<<1, kBlock, 0, s>>>(w.ctl, CTL_WORDS);
    k_degree_key<<<grid_for_threads(n), kBlock, 0, s>>>(n, row_ptr, w.key_a, w.val_a, w.ctl);
    const int ntiles = div_up(n, kTile);
    int *kin = w.key_a, *vin = w.val_a, *kout = w.key_b, *vout = w.val_b;
    for (int bit = 0; bit < key_bits; bit++) {
        k_tile_sum<<<ntiles, kBlock, 0, s>>>(n, kin, bit, 1, w.tiles);
        k_scan_tiles<<<1, kBlock, 0, s>>>(ntiles, w.tiles, w.ctl + CTL_ZEROS);
        k_radix_scatter<<<ntiles, kBlock, 0, s>>>(n, bit, kin, vin, w.tiles, w.ctl + CTL_ZEROS, kout, vout);
        int* t = kin; kin = kout; kout = t;
        t = vin; vin = vout; vout = t;
    }
    k_copy<<<grid_for_threads(n), kBlock, 0, s>>>(out_perm, vin, n);
    k_rank<<<grid_for_threads(n), kBlock, 0, s>>>(n, out_perm, w.rank);
    k_outdeg<<<grid_for_waves(n), kBlock, 0, s>>>(n, row_ptr, col, out_perm, w.rank, w.outdeg, w.ctl);
    KC_CHECK(hipGetLastError());
    int st = exclusive_scan(n, w.outdeg, out_row_ptr, w.tiles, w.ctl + CTL_ZEROS, s);
    if (st != KC_OK) return st;
    if (nnz > 0) {
        k_fill<<<grid_for_waves(n), kBlock, 0, s>>>(n, row_ptr, col, out_perm, w.rank, out_row_ptr, out_col,
                                                   out_src, w.tmp, w.ctl);
        k_sort_long_rows<<<grid_for_threads(n), kBlock, 0, s>>>(n, out_row_ptr, w.tmp, out_col, out_src);
        KC_CHECK(hipGetLastError());
    }
    return KC_OK;
}

}  // namespace kc

using namespace kc;

extern "C" KC_API size_t kc_orient_workspace(int32_t n, int32_t nnz, int32_t order) {
    (void)order;
    if (n < 0 || nnz < 0) return 0;
    size_t bytes = 0;
    carve(nullptr, n, nnz, &bytes);
    return bytes;
}

extern "C" KC_API int32_t kc_orient(const kc_csr* g, int32_t order, kc_dag* out, void* ws,
                                    size_t ws_bytes, int32_t validate, void* stream) {
    if (!g || !out) return KC_EINVAL;
    if (order != KC_ORDER_DEGREE && order != KC_ORDER_DEGENERACY && order != KC_ORDER_APPROX_DEGENERACY &&
        order != KC_ORDER_COLOR)
        return KC_EINVAL;
    const int n = g->n, nnz = g->nnz;
    if (n < 0 || nnz < 0 || (nnz & 1)) return KC_EINVAL;
    if (!g->row_ptr || !out->row_ptr || (n > 0 && !out->perm)) return KC_EINVAL;
    if (nnz > 0 && (!g->col || !out->col || !out->src)) return KC_EINVAL;
    size_t need = 0;
    OrientWs w = carve(ws, n, nnz, &need);
    if (!ws || ws_bytes < need) return KC_ENOMEM;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int m = nnz / 2;

    out->n = n;
    out->m = m;
    out->order = order;
    out->d_max = 0;
    out->degeneracy = order == KC_ORDER_DEGENERACY ? 0 : -1;
    KC_CHECK(hipMemsetAsync(w.ctl, 0, CTL_WORDS * sizeof(int), s));
    if (n == 0) {
        if (nnz != 0) return KC_EINVAL;
        KC_CHECK(hipMemsetAsync(out->row_ptr, 0, sizeof(int), s));
        KC_CHECK(hipStreamSynchronize(s));
        return KC_OK;
    }

    if (validate) {
        k_validate<<<grid_for_waves(n), kBlock, 0, s>>>(n, nnz, g->row_ptr, g->col, w.ctl);
        KC_CHECK(hipGetLastError());
        int err = 0;
        KC_CHECK(hipMemcpyAsync(&err, w.ctl + CTL_ERR, sizeof(int), hipMemcpyDeviceToHost, s));
        KC_CHECK(hipStreamSynchronize(s));
        if (err) return KC_EINVAL;
    }

    // 1. sort keys
    if (order == KC_ORDER_DEGREE) {
        k_degree_key<<<grid_for_threads(n), kBlock, 0, s>>>(n, g->row_ptr, w.key_a, w.val_a, w.ctl);
        KC_CHECK(hipGetLastError());
    } else if (order == KC_ORDER_COLOR) {
        // the colours go straight into the sort keys; rounds are launched in
        // batches of 4, 8, ... 64, and the host reads the frontier size after each
        k_cl_init<<<grid_for_waves(n), kBlock, 0, s>>>(n, g->row_ptr, g->col, w.rnd, w.val_a,
                                                       ClFront{nullptr, nullptr, w.fr0, w.hf0}, w.ctl);
        KC_CHECK(hipGetLastError());
        const int grid = device_cus() * 4;
        int r = 0;
        for (int batch = 4;; batch = batch < 64 ? 2 * batch : 64) {
            for (int i = 0; i < batch; i++, r++) {
                const ClFront f = (r & 1) ? ClFront{w.fr1, w.hf1, w.fr0, w.hf0} : ClFront{w.fr0, w.hf0, w.fr1, w.hf1};
                k_cl_round<<<grid, kBlock, 0, s>>>(r, f, g->row_ptr, g->col, w.rnd, w.key_a, w.ctl);
            }
            KC_CHECK(hipGetLastError());
            int left[2] = {0, 0};
            KC_CHECK(hipMemcpyAsync(&left[0], w.ctl + CTL_CL_SIZE0 + r % 3, sizeof(int), hipMemcpyDeviceToHost, s));
            KC_CHECK(hipMemcpyAsync(&left[1], w.ctl + CTL_CL_HSIZE0 + r % 3, sizeof(int), hipMemcpyDeviceToHost, s));
            KC_CHECK(hipStreamSynchronize(s));
            if (left[0] + left[1] == 0) break;
            if (r > n) return KC_EDEVICE;   // cannot happen: every round colours at least one vertex
        }
    } else if (order == KC_ORDER_APPROX_DEGENERACY) {
        // host-driven rounds: the live count decides when to stop
        int* deg = w.key_b;   // scratch until the sort
        k_ad_init<<<grid_for_threads(n), kBlock, 0, s>>>(n, g->row_ptr, deg, w.rnd, w.val_a);
        KC_CHECK(hipGetLastError());
        int r = 0;
        for (;; r++) {
            KC_CHECK(hipMemsetAsync(w.ctl + CTL_AD_LIVE, 0, 4 * sizeof(int), s));
            k_ad_sum<<<grid_for_threads(n), kBlock, 0, s>>>(n, deg, w.rnd, w.ctl);
            KC_CHECK(hipGetLastError());
            int live = 0;
            KC_CHECK(hipMemcpyAsync(&live, w.ctl + CTL_AD_LIVE, sizeof(int), hipMemcpyDeviceToHost, s));
            KC_CHECK(hipStreamSynchronize(s));
            if (live == 0) break;
            k_ad_mark<<<grid_for_threads(n), kBlock, 0, s>>>(n, r, deg, w.rnd, w.ctl);
            k_ad_dec<<<grid_for_waves(n), kBlock, 0, s>>>(n, r, g->row_ptr, g->col, deg, w.rnd);
            KC_CHECK(hipGetLastError());
        }
        const int maxkey = r > 0 ? r - 1 : 0;
        KC_CHECK(hipMemcpyAsync(w.ctl + CTL_MAXKEY, &maxkey, sizeof(int), hipMemcpyHostToDevice, s));
        KC_CHECK(hipMemcpyAsync(w.ctl + CTL_ROUNDS, &r, sizeof(int), hipMemcpyHostToDevice, s));
        KC_CHECK(hipMemcpyAsync(w.key_a, w.rnd, sizeof(int) * n, hipMemcpyDeviceToDevice, s));
    } else {
        int occ = 0;
        KC_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_peel, kBlock, 0));
        if (occ < 1) return KC_EDEVICE;
        // Most rounds are small and end in a grid barrier whose cost grows with
        // the number of blocks: one block per 16k vertices, between 32 and one
        // per CU (64 blocks peeled the 1M-vertex power-law graph in 37 ms, 256 in 61).
        int blocks = n / 16384;
        if (blocks > device_cus()) blocks = device_cus();
        if (blocks < 32) blocks = 32;
        if (blocks > occ * device_cus()) blocks = occ * device_cus();   // all blocks co-resident
        int n_ = n;
        const int* rp = g->row_ptr;
        const int* cl = g->col;
        int* deg = w.key_b;   // scratch until the sort
        void* args[] = {&n_, &rp, &cl, &deg, &w.rnd, &w.fr0, &w.fr1, &w.hf0, &w.hf1, &w.val_a, &w.ctl};
        KC_CHECK(hipLaunchCooperativeKernel(reinterpret_cast<void*>(k_peel), dim3(blocks), dim3(kBlock),
                                            args, 0, s));
        KC_CHECK(hipMemcpyAsync(w.key_a, w.rnd, sizeof(int) * n, hipMemcpyDeviceToDevice, s));
    }
    int hctl[CTL_WORDS];
    KC_CHECK(hipMemcpyAsync(hctl, w.ctl, sizeof(hctl), hipMemcpyDeviceToHost, s));
    KC_CHECK(hipStreamSynchronize(s));
    int bits = 0;
    while (bits < 31 && (hctl[CTL_MAXKEY] >> bits) != 0) bits++;

    // 2. stable radix sort (key, id) -> position = new id
    int ntiles = div_up(n, kTile);
    int *kin = w.key_a, *vin = w.val_a, *kout = w.key_b, *vout = w.val_b;
    for (int bit = 0; bit < bits; bit++) {
        k_tile_sum<<<ntiles, kBlock, 0, s>>>(n, kin, bit, 1, w.tiles);
        k_scan_tiles<<<1, kBlock, 0, s>>>(ntiles, w.tiles, w.ctl + CTL_ZEROS);
        k_radix_scatter<<<ntiles, kBlock, 0, s>>>(n, bit, kin, vin, w.tiles, w.ctl + CTL_ZEROS, kout, vout);
        KC_CHECK(hipGetLastError());
        int* t = kin; kin = kout; kout = t;
        t = vin; vin = vout; vout = t;
    }
    KC_CHECK(hipMemcpyAsync(out->perm, vin, sizeof(int) * n, hipMemcpyDeviceToDevice, s));
    k_rank<<<grid_for_threads(n), kBlock, 0, s>>>(n, out->perm, w.rank);
    KC_CHECK(hipGetLastError());

    // 3. filter: out-degree histogram + exclusive scan -> row_ptr
    k_outdeg<<<grid_for_waves(n), kBlock, 0, s>>>(n, g->row_ptr, g->col, out->perm, w.rank, w.outdeg, w.ctl);
    KC_CHECK(hipGetLastError());
    int st = exclusive_scan(n, w.outdeg, out->row_ptr, w.tiles, w.ctl + CTL_ZEROS, s);
    if (st != KC_OK) return st;

    // 4. compact + per-row sort
    if (m > 0) {
        k_fill<<<grid_for_waves(n), kBlock, 0, s>>>(n, g->row_ptr, g->col, out->perm, w.rank, out->row_ptr,
                                                   out->col, out->src, w.tmp, w.ctl);
        KC_CHECK(hipGetLastError());
    }
    KC_CHECK(hipMemcpyAsync(hctl, w.ctl, sizeof(hctl), hipMemcpyDeviceToHost, s));
    int total = 0;
    KC_CHECK(hipMemcpyAsync(&total, out->row_ptr + n, sizeof(int), hipMemcpyDeviceToHost, s));
    KC_CHECK(hipStreamSynchronize(s));
    if (hctl[CTL_LONG]) {
        k_sort_long_rows<<<grid_for_threads(n), kBlock, 0, s>>>(n, out->row_ptr, w.tmp, out->col, out->src);
        KC_CHECK(hipGetLastError());
        KC_CHECK(hipStreamSynchronize(s));
    }
    if (total != m) return KC_EINVAL;   // not symmetric (only possible without validation)
    out->d_max = hctl[CTL_DMAX];
    out->degeneracy = order == KC_ORDER_DEGENERACY ? hctl[CTL_DEGEN] : -1;
    return KC_OK;
}
