// Explicit instantiation of the per-stage minimum and sd-matrix kernels for 3 footprint slots.
#include "psdf_kernels.hpp"

namespace psdf {
template hipError_t launch_main_mf<3>(int, const LaunchShape&, const FpConst&, const float*, int,
                                       const psdf_edges&, uint64_t*, hipStream_t, hipEvent_t,
                                       hipEvent_t);
template hipError_t launch_sdmat_mf<3>(int, const FpConst&, const float*, int,
                                        const psdf_edges&, float*, hipStream_t);
}  // namespace psdf
