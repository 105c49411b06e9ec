// Lane-walk kernels with bitset rows of up to 1 words (see kc_lane_impl.h).
#include "kc_lane_impl.h"

namespace kc {

int lane_launch_w1(const lanewalk::LaneParams& P, bool ec, bool pair, bool stats, int* grid, hipStream_t s) {
    return lanewalk::launch_lane_m<1>(P, ec, pair, stats, grid, s);
}

}  // namespace kc
