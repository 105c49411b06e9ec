// Lane-walk launches (Fig. 2): builds the kernel parameters of one width list
// and dispatches to the instantiation of its row width (kc_lane_w*.hip).
#include "kc_lane_impl.h"

namespace kc {

int lane_launch(const LaneLaunch& L, hipStream_t s) {
    if (L.pair && L.maxw < 2) return KC_EINVAL;    // pair mode keeps queued items in the prefix area
    lanewalk::LaneParams P;
    P.k = L.k;
    P.row_ptr = L.row_ptr;
    P.col = L.col;
    P.src = L.src;
    P.list = L.list;
    P.lists = L.lists;
    P.counts = L.counts;
    P.head = L.head;
    P.task_ctr = L.task_ctr;
    P.task_tot = L.task_tot;
    P.active = L.active;
    P.acc = L.acc;
    P.stats = L.stats_ptr;
    P.iters = L.iters_ptr;
    P.timing = L.timing_ptr;
    P.cwords = L.cwords_ptr;
    P.gacc = L.gacc;
    P.gid = L.gid;
    P.steal = L.pair && L.steal;
    P.helper = L.helper && P.steal;
    P.qctl = L.qctl;
    P.qready = L.qready;
    P.qitems = L.qitems;
    P.flags = L.flags;
    P.steal_every = L.steal_every > 0 ? L.steal_every : kLaneStealEvery;
    P.steal_after = L.steal_after > 0 ? L.steal_after : kLaneStealAfter;
    P.cancel = L.flags ? L.cancel : nullptr;   // a cancel request is recorded in the flags word
    const int p0 = L.ec ? 3 : 2;
    // pair tasks start at path length p0 + 1; vertex tasks at p0.  Saved levels
    // are needed for path lengths below k - 2.
    const int first = L.pair ? p0 + 1 : p0;
    P.levels = k_levels(L.k, first);
    P.s_cap = 0;
    switch (L.maxw) {
        case 1: return lane_launch_w1(P, L.ec, L.pair, L.stats, L.grid_out, s);
        case 2: return lane_launch_w2(P, L.ec, L.pair, L.stats, L.grid_out, s);
        case 4: return lane_launch_w4(P, L.ec, L.pair, L.stats, L.grid_out, s);
        case 8: return lane_launch_w8(P, L.ec, L.pair, L.stats, L.grid_out, s);
        case 16: return lane_launch_w16(P, L.ec, L.pair, L.stats, L.grid_out, s);
        case 32: return lane_launch_w32(P, L.ec, L.pair, L.stats, L.grid_out, s);
        default: return KC_EINVAL;
    }
}

}  // namespace kc
