// k_l1_i64.hip - the l1 coordinate pass for integer points with int64 right-hand sides.
#include "l1_pass.h"

namespace dm {

hipError_t launch_l1_pass_i64(const L1PassArgs& a, int32_t b, int variant, hipStream_t s) {
    return launch_pass_p<IntPath<int64_t>>(a, b, variant, s);
}

int l1_tile_ranks_i64(int32_t b, int variant) { return tile_ranks_p<IntPath<int64_t>>(b, variant); }

}  // namespace dm
