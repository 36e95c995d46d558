// Explicit instantiation of the persistent batch kernel for 16 footprint slots.
#include "psdf_batch.hpp"

namespace psdf {
template hipError_t launch_batch_mf<16>(int, int, int, const BatchArgs&, hipStream_t, hipEvent_t,
                                          hipEvent_t);
template hipError_t batch_occupancy_mf<16>(int, int, int*);
}  // namespace psdf
