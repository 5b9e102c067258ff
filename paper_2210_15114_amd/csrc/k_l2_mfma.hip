// k_l2_mfma.hip - matrix-core path of the l2-squared query (placeholder until
// the MFMA kernels land: reports that it did not run, so the vector path in
// k_l2.hip serves every call).
#include "dm_device.h"
#include "dm_internal.h"

namespace dm {

hipError_t launch_l2sq_mfma(const float* Xc, const double* nrm, int64_t n, int32_t d, const float* Z, int32_t b,
                            float* Out, void* scratch, const TotalsOut& tot, hipStream_t s, bool* used)
{
    (void)Xc; (void)nrm; (void)n; (void)d; (void)Z; (void)b; (void)Out; (void)scratch; (void)tot; (void)s;
    *used = false;
    return hipSuccess;
}

}  // namespace dm
