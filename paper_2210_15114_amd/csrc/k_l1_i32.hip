// k_l1_i32.hip - the l1 coordinate pass for integer points with int32 right-hand sides.
#include "l1_pass.h"

namespace dm {

hipError_t launch_l1_pass_i32(const L1PassArgs& a, int32_t b, int variant, hipStream_t s) {
    return launch_pass_p<IntPath<int32_t>>(a, b, variant, s);
}

int l1_tile_ranks_i32(int32_t b, int variant) { return tile_ranks_p<IntPath<int32_t>>(b, variant); }

}  // namespace dm
