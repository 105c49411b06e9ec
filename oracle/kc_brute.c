/*
 * Brute-force clique enumeration -- TEST INFRASTRUCTURE ONLY.
 *
 * Independent of the oracle's recursions: no orientation, no pivoting, no
 * induced sub-graphs.  For graphs of at most 64 vertices it lists every clique
 * exactly once by extending it only with larger vertex ids (adjacency as 64-bit
 * masks) and tallies the cliques by size.  counts[0] = 1 is the empty clique.
 */
#include <stdint.h>
#include <string.h>

typedef unsigned __int128 u128;

static void extend(const uint64_t* adj, uint64_t cand, int32_t size, u128* cnt, int32_t cap) {
    if (size <= cap) cnt[size] += 1;
    while (cand) {
        int32_t v = __builtin_ctzll(cand);
        cand &= cand - 1;
        /* candidates after v that are adjacent to v */
        uint64_t higher = (v == 63) ? 0 : (~0ULL << (v + 1));
        extend(adj, cand & adj[v] & higher, size + 1, cnt, cap);
    }
}

int kco_brute_counts(int32_t n, const int32_t* row_ptr, const int32_t* col, int32_t cap,
                     uint64_t* counts) {
    if (n < 0 || n > 64 || cap < 0) return -1;
    uint64_t adj[64];
    u128 cnt[65];
    memset(adj, 0, sizeof adj);
    memset(cnt, 0, sizeof cnt);
    for (int32_t v = 0; v < n; v++)
        for (int32_t e = row_ptr[v]; e < row_ptr[v + 1]; e++) adj[v] |= 1ULL << col[e];
    uint64_t all = (n == 64) ? ~0ULL : ((1ULL << n) - 1);
    extend(adj, all, 0, cnt, cap > 64 ? 64 : cap);
    for (int32_t j = 0; j <= cap; j++) {
        u128 x = j <= 64 ? cnt[j] : 0;
        counts[2 * j] = (uint64_t)x;
        counts[2 * j + 1] = (uint64_t)(x >> 64);
    }
    return 0;
}
