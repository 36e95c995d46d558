// Host-side helpers shared by the C-ABI entry points.
#pragma once

#include <hip/hip_runtime.h>

#include "psdf.h"
#include "psdf_device.hpp"

namespace psdf {

constexpr int kMaxStageBlock = 64;   // stages per work-group in the plain kernel

struct LaunchShape {
  int blk;  // lanes (obstacles) per work-group: 64 or 256
  int sb;   // stages per work-group, 1..kMaxStageBlock
};

const char* last_error();
void clear_error();
int set_error(int code, const char* fmt, ...);
int hip_status(hipError_t err);

// Validate the footprint (m in [3, 16], strictly convex, no zero-length edge),
// orient it counter-clockwise and derive its constants in double precision.
int prepare_footprint(const float* xy, int m, const psdf_params* params, FpConst* out);

// Validate the host-side description of an edge set.
int check_edges(const psdf_edges* in, psdf_edges* out);

// Register class of the per-obstacle edge arrays for a bound mbar.
inline int obst_class(int mbar) { return mbar <= 4 ? 4 : (mbar <= 8 ? 8 : 16); }

// Kernel timer: bracket one launch of the dominant kernel with events.
void timer_begin(hipStream_t st);
void timer_end(hipStream_t st);
// Or take an event pair for a launch that records them itself (the
// dispatch's own start and end, hipExtLaunchKernel); false when the timer is
// off or full.
bool timer_kernel_events(hipEvent_t* start, hipEvent_t* stop);

// Default launch shape of the plain kernel for N stages and M obstacles.
LaunchShape choose_shape(int N, int M);

// Launch shape for a problem: an explicit override (psdf_set_launch_shape),
// else choose_shape.
LaunchShape tuned_shape(int m, int mbar, int N, int M);

hipError_t launch_plain(const FpConst& F, const float* poses, int N, const psdf_edges& e,
                        uint64_t* partial, const LaunchShape& ls, hipStream_t st);
hipError_t launch_epilogue(const FpConst& F, const float* poses, int N, const psdf_edges& e,
                           const uint64_t* partial, int gx, uint64_t* keys, const float* gout,
                           int mode, float dmin, float* d, int* edge, int* obst, float* grad,
                           float* hj, hipStream_t st);
int partial_columns(int M, const LaunchShape& ls);

}  // namespace psdf
