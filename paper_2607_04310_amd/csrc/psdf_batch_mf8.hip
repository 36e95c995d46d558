// Explicit instantiation of the persistent batch and screening kernels for 8 footprint slots.
#include "psdf_batch.hpp"
#include "psdf_screen.hpp"

namespace psdf {
template hipError_t launch_batch_mf<8>(int, int, int, const BatchArgs&, hipStream_t, hipEvent_t,
                                          hipEvent_t);
template hipError_t batch_occupancy_mf<8>(int, int, int*);
template hipError_t launch_screen_mf<8>(int, int, const ScreenArgs&, hipStream_t);
template hipError_t launch_screen_bound_mf<8>(int, int, const ScreenArgs&, hipStream_t);
template hipError_t launch_fallback_mf<8>(int, int, int, const ScreenArgs&, hipStream_t);
}  // namespace psdf
