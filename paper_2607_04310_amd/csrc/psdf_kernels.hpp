// Per-stage minimum kernel of the plain path, templated on the footprint slot
// count MF, the obstacle edge class MI and the work-group width BLK;
// instantiated per MF in psdf_inst_mf*.hip.
//
// Lane <-> obstacle: a lane loads its obstacle's edges once into registers
// and evaluates sd for every stage of the work-group's stage block.  Per
// stage the wave takes the minimum of the orderable sd, the lowest lane
// holding it names the obstacle (lowest index on ties), and the work-group
// writes one 16-byte partial per stage to partial[stage][blockIdx.x]: the key
// (orderable(sd) << 32 | obstacle) and the winner's (first edge << 32 | edge
// count).  The epilogue reduces the partial keys of a stage; no atomics and
// no initialisation pass are needed.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "psdf.h"
#include "psdf_device.hpp"
#include "psdf_host.hpp"
#include "psdf_staged.hpp"
#include "psdf_winner.hpp"

namespace psdf {

template <int MF, int MI, int BLK>
__global__ __launch_bounds__(BLK) void main_kernel(FpConst F, const float* __restrict__ poses,
                                                    int N, int SB, const float* __restrict__ ax,
                                                    const float* __restrict__ ay,
                                                    const float* __restrict__ bx,
                                                    const float* __restrict__ by,
                                                    const int* __restrict__ off, int E, int M,
                                                    ulonglong2* __restrict__ partial) {
  constexpr int NW = BLK / 64;
  __shared__ float4 st[kMaxStageBlock];
  __shared__ float4 rft[kMaxStageBlock * MF];
  __shared__ uint64_t wk[NW][kMaxStageBlock];
  __shared__ uint64_t wa[NW][kMaxStageBlock];
  const int s0 = blockIdx.y * SB;
  const int ns = min(SB, N - s0);
  const int gx = gridDim.x;
  const int w = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int wave_base = blockIdx.x * BLK + w * 64;

  const int i = wave_base + lane;
  const bool active = i < M;
  int e0 = 0, mi = 0;
  if (active) { e0 = off[i]; mi = off[i + 1] - e0; }

  fill_stage_table<MF>(F, poses, s0, ns, st, rft, BLK);
  __syncthreads();

  if (wave_base < M) {
    auto emit = [&](int t, uint64_t key, uint64_t a) {
      if (lane == 0) {
        if (NW == 1) {
          partial[(size_t)(s0 + t) * gx + blockIdx.x] = make_ulonglong2(key, a);
        } else {
          wk[w][t] = key;
          wa[w][t] = a;
        }
      }
    };
    // lazy own-axis intervals: a wave meets its obstacles at one or a few
    // stages here, and far obstacles never need them
    wave_stages<MF, MI, decltype(emit), true>(F, ax, ay, bx, by, e0, mi, E, active, false,
                                              wave_base, ns, st, rft, emit);
  } else if (NW > 1 && lane == 0) {
    for (int t = 0; t < ns; ++t) { wk[w][t] = kEmptyKey; wa[w][t] = 0; }
  }
  if (NW > 1) {
    __syncthreads();
    for (int t = threadIdx.x; t < ns; t += BLK) {
      uint64_t k = wk[0][t], a = wa[0][t];
#pragma unroll
      for (int v = 1; v < NW; ++v)
        if (wk[v][t] < k) { k = wk[v][t]; a = wa[v][t]; }
      partial[(size_t)(s0 + t) * gx + blockIdx.x] = make_ulonglong2(k, a);
    }
  }
}

// main_kernel on a staged edge set (psdf_staged.hpp): the lane's obstacle
// row (its slots, intervals and flags) comes from coalesced table loads,
// issued before the stage table is built, instead of from the offsets and
// edges plus the per-lane setup.  Same stage loop, same partials, bit for
// bit.
template <int MF, int MI, int BLK>
__global__ __launch_bounds__(BLK) void main_staged_kernel(FpConst F, const float* __restrict__ poses,
                                                           int N, int SB, StagedView v, int M,
                                                           ulonglong2* __restrict__ partial) {
  constexpr int NW = BLK / 64;
  __shared__ float4 st[kMaxStageBlock];
  __shared__ float4 rft[kMaxStageBlock * MF];
  __shared__ uint64_t wk[NW][kMaxStageBlock];
  __shared__ uint64_t wa[NW][kMaxStageBlock];
  const int s0 = blockIdx.y * SB;
  const int ns = min(SB, N - s0);
  const int gx = gridDim.x;
  const int w = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int wave_base = blockIdx.x * BLK + w * 64;

  const int i = wave_base + lane;
  const bool active = i < M;
  int4 meta = make_int4(0, 0, 0, 0);
  float4 r0[MI], r1[MI];
#pragma unroll
  for (int j = 0; j < MI; ++j) {
    r0[j] = make_float4(0.f, 0.f, 0.f, 0.f);
    r1[j] = make_float4(0.f, 0.f, 0.f, 0.f);
  }
  if (active) {
    meta = v.meta[i];
#pragma unroll
    for (int j = 0; j < MI; ++j) {
      r0[j] = v.rec0[(size_t)j * v.Mp + i];
      r1[j] = v.rec1[(size_t)j * v.Mp + i];
    }
  }

  fill_stage_table<MF>(F, poses, s0, ns, st, rft, BLK);
  __syncthreads();

  if (wave_base < M) {
    auto emit = [&](int t, uint64_t key, uint64_t a) {
      if (lane == 0) {
        if (NW == 1) {
          partial[(size_t)(s0 + t) * gx + blockIdx.x] = make_ulonglong2(key, a);
        } else {
          wk[w][t] = key;
          wa[w][t] = a;
        }
      }
    };
    const int e0 = meta.x, mi = meta.y;
    const bool segments = __ballot(active && mi > 1) == 0;
    if (MI > 1 && segments) {
      Obst<1> o;
      staged_obstacle<1, MI>(o, v, i, active, r0, r1, mi, meta.z);
      wave_stage_loop<MF, 1>(F, o, e0, mi, active, wave_base, ns, st, rft, emit);
    } else {
      Obst<MI> o;
      staged_obstacle<MI, MI>(o, v, i, active, r0, r1, mi, meta.z);
      wave_stage_loop<MF, MI>(F, o, e0, mi, active, wave_base, ns, st, rft, emit);
    }
  } else if (NW > 1 && lane == 0) {
    for (int t = 0; t < ns; ++t) { wk[w][t] = kEmptyKey; wa[w][t] = 0; }
  }
  if (NW > 1) {
    __syncthreads();
    for (int t = threadIdx.x; t < ns; t += BLK) {
      uint64_t k = wk[0][t], a = wa[0][t];
#pragma unroll
      for (int u = 1; u < NW; ++u)
        if (wk[u][t] < k) { k = wk[u][t]; a = wa[u][t]; }
      partial[(size_t)(s0 + t) * gx + blockIdx.x] = make_ulonglong2(k, a);
    }
  }
}

// ev0 / ev1 (may be null): events that the dispatch itself records at its
// start and end (kernel timer).  A staged table (e.staged) selects
// main_staged_kernel.
template <int MF, int MI>
hipError_t launch_main_t(const LaunchShape& ls, const FpConst& F, const float* poses, int N,
                         const psdf_edges& e, uint64_t* partial, hipStream_t st, hipEvent_t ev0,
                         hipEvent_t ev1) {
  dim3 grid((e.M + ls.blk - 1) / ls.blk, (N + ls.sb - 1) / ls.sb);
  ulonglong2* pk = reinterpret_cast<ulonglong2*>(partial);
  if (e.staged) {
    const StagedView v = staged_view(e.staged->table, e.M, MI);
    if (ls.blk == 64)
      hipExtLaunchKernelGGL(main_staged_kernel<MF, MI, 64>, grid, dim3(64), 0, st, ev0, ev1, 0,
                            F, poses, N, ls.sb, v, e.M, pk);
    else
      hipExtLaunchKernelGGL(main_staged_kernel<MF, MI, 256>, grid, dim3(256), 0, st, ev0, ev1, 0,
                            F, poses, N, ls.sb, v, e.M, pk);
    return hipGetLastError();
  }
  if (ls.blk == 64)
    hipExtLaunchKernelGGL(main_kernel<MF, MI, 64>, grid, dim3(64), 0, st, ev0, ev1, 0, F, poses,
                          N, ls.sb, e.ax, e.ay, e.bx, e.by, e.obst_off, e.E, e.M, pk);
  else
    hipExtLaunchKernelGGL(main_kernel<MF, MI, 256>, grid, dim3(256), 0, st, ev0, ev1, 0, F,
                          poses, N, ls.sb, e.ax, e.ay, e.bx, e.by, e.obst_off, e.E, e.M, pk);
  return hipGetLastError();
}

template <int MF>
hipError_t launch_main_mf(int mi_class, const LaunchShape& ls, const FpConst& F,
                          const float* poses, int N, const psdf_edges& e, uint64_t* partial,
                          hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
  if (mi_class == 4) return launch_main_t<MF, 4>(ls, F, poses, N, e, partial, st, ev0, ev1);
  if (mi_class == 8) return launch_main_t<MF, 8>(ls, F, poses, N, e, partial, st, ev0, ev1);
  return launch_main_t<MF, 16>(ls, F, poses, N, e, partial, st, ev0, ev1);
}

// Every obstacle's sd per stage, before the minimum over obstacles: lane <->
// obstacle as in main_kernel, sd[s][i] (stage-major, written coalesced along
// obstacles); +inf for an empty obstacle, NaN for a non-finite pose or an
// invalid obstacle.  Same obstacle_sd as main_kernel, so the row minimum is
// the per-stage minimum bit for bit.
constexpr int kSdmatStageBlock = 4;

template <int MF, int MI>
__global__ __launch_bounds__(256) void sdmat_kernel(FpConst F, const float* __restrict__ poses,
                                                     int N, int SB, const float* __restrict__ ax,
                                                     const float* __restrict__ ay,
                                                     const float* __restrict__ bx,
                                                     const float* __restrict__ by,
                                                     const int* __restrict__ off, int E, int M,
                                                     float* __restrict__ sd) {
  __shared__ float4 st[kSdmatStageBlock];
  __shared__ float4 rft[kSdmatStageBlock * MF];
  const int s0 = blockIdx.y * SB;
  const int ns = min(SB, N - s0);
  const int i = blockIdx.x * 256 + threadIdx.x;
  const bool active = i < M;
  int e0 = 0, mi = 0;
  if (active) { e0 = off[i]; mi = off[i + 1] - e0; }
  fill_stage_table<MF>(F, poses, s0, ns, st, rft, 256);
  __syncthreads();
  if (!active) return;
  Obst<MI> o;
  load_obstacle<MI>(o, ax, ay, bx, by, e0, mi, E, F.eps);
  for (int t = 0; t < ns; ++t) {
    const float4 q = st[t];
    const bool pose_ok = isfinite(q.x) && isfinite(q.y) && isfinite(q.z) && isfinite(q.w);
    float v = __builtin_huge_valf();
    if (mi != 0) v = pose_ok ? obstacle_sd<MF, MI>(F, o, rft + t * MF, q.z, q.w) : __builtin_nanf("");
    sd[(size_t)(s0 + t) * M + i] = v;
  }
}

template <int MF>
hipError_t launch_sdmat_mf(int mi_class, const FpConst& F, const float* poses, int N,
                           const psdf_edges& e, float* sd, hipStream_t st) {
  dim3 grid((e.M + 255) / 256, (N + kSdmatStageBlock - 1) / kSdmatStageBlock);
#define PSDF_SDMAT(MI)                                                                        \
  sdmat_kernel<MF, MI><<<grid, 256, 0, st>>>(F, poses, N, kSdmatStageBlock, e.ax, e.ay, e.bx, \
                                             e.by, e.obst_off, e.E, e.M, sd)
  if (mi_class == 4) PSDF_SDMAT(4);
  else if (mi_class == 8) PSDF_SDMAT(8);
  else PSDF_SDMAT(16);
#undef PSDF_SDMAT
  return hipGetLastError();
}

#define PSDF_EXTERN_MF(MF)                                                                  \
  extern template hipError_t launch_main_mf<MF>(int, const LaunchShape&, const FpConst&,    \
                                                const float*, int, const psdf_edges&,       \
                                                uint64_t*, hipStream_t, hipEvent_t,         \
                                                hipEvent_t);                                \
  extern template hipError_t launch_sdmat_mf<MF>(int, const FpConst&, const float*, int,    \
                                                 const psdf_edges&, float*, hipStream_t);
PSDF_EXTERN_MF(3)
PSDF_EXTERN_MF(4)
PSDF_EXTERN_MF(5)
PSDF_EXTERN_MF(6)
PSDF_EXTERN_MF(7)
PSDF_EXTERN_MF(8)
PSDF_EXTERN_MF(16)

}  // namespace psdf
