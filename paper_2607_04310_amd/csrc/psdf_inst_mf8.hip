// Explicit instantiation of the plain-path kernels for 8 footprint slots.
#include "psdf_kernels.hpp"

namespace psdf {
template hipError_t launch_main_mf<8>(int, const LaunchShape&, const FpConst&, const float*, int,
                                        const psdf_edges&, uint64_t*, hipStream_t);
template hipError_t launch_epi_mf<8>(int, const FpConst&, const float*, int, const psdf_edges&,
                                       const uint64_t*, const float*, int, float*, int*, int*,
                                       float*, hipStream_t);
}  // namespace psdf
