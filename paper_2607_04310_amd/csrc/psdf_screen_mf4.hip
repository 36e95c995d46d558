// Explicit instantiation of the screening kernels for 4 footprint slots.
#include "psdf_screen.hpp"

namespace psdf {
template hipError_t launch_screen_mf<4>(int, int, const ScreenArgs&, hipStream_t);
template hipError_t launch_screen_bound_mf<4>(int, int, const ScreenArgs&, hipStream_t);
template hipError_t launch_fallback_mf<4>(int, int, int, const ScreenArgs&, hipStream_t);
}  // namespace psdf
