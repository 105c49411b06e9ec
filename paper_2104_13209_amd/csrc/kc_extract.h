// Induced sub-graph extraction into LDS bitsets (paper Sec. 2.4, 3.4), shared by
// the graph-orientation and pivoting traversals.
#pragma once

#include "kc_internal.h"

namespace kc {

// A team is TEAM_LANES consecutive threads (one wavefront or a whole workgroup)
// that extracts one root's sub-graph together; tl is the thread's index in it.
template <int TW>
__device__ __forceinline__ void team_sync() {
    if (TW == 1) wave_sync_lds();
    else __syncthreads();
}

// Candidate set S of a root, sorted ascending, into S[]; returns |S| through
// ctl_s (written by team lane 0) after a team sync.
//   VC root u:    S = N+(u)
//   EC root u->v: S = N+(u) cap N+(v)   (one wavefront: binary search of each
//                 element of N+(v) in N+(u), compacted in order with a ballot)
template <int TW, bool EC>
__device__ __forceinline__ void extract_set(int rid, const int* __restrict__ row_ptr, const int* __restrict__ col,
                                            const int* __restrict__ src, int tl, int* S, int* ctl_s) {
    constexpr int TEAM_LANES = 64 * TW;
    if (!EC) {
        const int b = row_ptr[rid], e = row_ptr[rid + 1];
        for (int j = tl; j < e - b; j += TEAM_LANES) S[j] = col[b + j];
        if (tl == 0) *ctl_s = e - b;
    } else if (tl < 64) {
        const int lane = tl;
        const int u = src[rid], v = col[rid];
        const int ub = row_ptr[u], ue = row_ptr[u + 1];
        const int vb = row_ptr[v], ve = row_ptr[v + 1];
        int cnt = 0;
        for (int j0 = vb; j0 < ve; j0 += 64) {
            const int j = j0 + lane;
            bool hit = false;
            int x = 0;
            if (j < ve) {
                x = col[j];
                int lo = ub, hi = ue;
                while (lo < hi) {
                    int mid = (lo + hi) >> 1;
                    if (col[mid] < x) lo = mid + 1; else hi = mid;
                }
                hit = lo < ue && col[lo] == x;
            }
            const unsigned long long mk = __ballot(hit);
            if (hit) S[cnt + __popcll(mk & lanemask_lt())] = x;
            cnt += __popcll(mk);
        }
        if (lane == 0) *ctl_s = cnt;
    }
    team_sync<TW>();
}

// Bitset rows over S (row stride `stride` words, rows 0..s-1 zeroed first):
//   directed (UND = false): bit j of row i  <=>  S[j] in N+(S[i])  (j > i only)
//   undirected (UND = true): additionally bit i of row j for every such pair.
// Bits come from binary searches of each out-neighbour of S[i] in S[i+1..s),
// 16 lanes per row; rows are sorted, so the scan of N+(S[i]) stops past max S.
template <int TW, bool UND>
__device__ __forceinline__ void extract_rows(int s, const int* __restrict__ row_ptr, const int* __restrict__ col,
                                             int tl, const int* S, unsigned int* B, int stride) {
    constexpr int TEAM_LANES = 64 * TW;
    constexpr int XG = 16;
    for (int w = tl; w < s * stride; w += TEAM_LANES) B[w] = 0u;
    team_sync<TW>();
    const int smax = s > 0 ? S[s - 1] : 0;
    for (int i = tl / XG; i < s; i += TEAM_LANES / XG) {
        const int w = S[i];
        const int b = row_ptr[w], e = row_ptr[w + 1];
        for (int j = b + (tl % XG); j < e; j += XG) {
            const int x = col[j];
            if (x > smax) break;
            int lo = i + 1, hi = s;
            while (lo < hi) {
                int mid = (lo + hi) >> 1;
                if (S[mid] < x) lo = mid + 1; else hi = mid;
            }
            if (lo < s && S[lo] == x) {
                atomicOr(&B[i * stride + (lo >> 5)], 1u << (lo & 31));
                if (UND) atomicOr(&B[lo * stride + (i >> 5)], 1u << (i & 31));
            }
        }
    }
    team_sync<TW>();
}

}  // namespace kc
