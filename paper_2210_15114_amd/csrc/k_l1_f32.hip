// k_l1_f32.hip - the l1 coordinate pass for float data (FP32 points and right-hand sides).
#include "l1_pass.h"

namespace dm {

hipError_t launch_l1_pass_f32(const L1PassArgs& a, int32_t b, int variant, hipStream_t s) {
    return launch_pass_p<FloatPath>(a, b, variant, s);
}

int l1_tile_ranks_f32(int32_t b, int variant) { return tile_ranks_p<FloatPath>(b, variant); }

}  // namespace dm
