// Explicit instantiation of the screening kernels for 3 footprint slots.
#include "psdf_screen.hpp"

namespace psdf {
template hipError_t launch_screen_mf<3>(int, int, const ScreenArgs&, hipStream_t);
template hipError_t launch_screen_bound_mf<3>(int, int, const ScreenArgs&, hipStream_t);
template hipError_t launch_fallback_mf<3>(int, int, int, const ScreenArgs&, hipStream_t);
}  // namespace psdf
