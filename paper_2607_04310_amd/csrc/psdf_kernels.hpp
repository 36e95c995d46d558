// Plain-path kernels, templated on the footprint slot count MF and the
// obstacle edge class MI; instantiated per MF in psdf_inst_mf*.hip.
//
//   main_kernel      lane <-> obstacle; a work-group owns BLK obstacles and a
//                    block of stages; per stage: sd of the lane's obstacle,
//                    wave min on the orderable sd, lowest lane of the minimum
//                    -> one 64-bit atomicMin of (sd, obstacle) per wave and stage
//   epilogue_kernel  one lane per stage: decode the winner, recompute its
//                    obstacle with the reverse-mode adjoint, write d, edge,
//                    obst and the gradient
#pragma once

#include <hip/hip_runtime.h>

#include "psdf.h"
#include "psdf_device.hpp"
#include "psdf_host.hpp"

namespace psdf {

// ------------------------------------------------------------------ kernels

// Wave-wide minimum of a 32-bit unsigned value.
__device__ __forceinline__ uint32_t wave_min_u32(uint32_t x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x = min(x, (uint32_t)__shfl_xor((int)x, o));
  return x;
}

template <int MF, int MI, int BLK>
__global__ __launch_bounds__(BLK) void main_kernel(FpConst F, const float* __restrict__ poses,
                                                    int N, int SB, const float* __restrict__ ax,
                                                    const float* __restrict__ ay,
                                                    const float* __restrict__ bx,
                                                    const float* __restrict__ by,
                                                    const int* __restrict__ off, int E, int M,
                                                    uint64_t* __restrict__ keys) {
  __shared__ float4 st[kMaxStageBlock];
  const int s0 = blockIdx.y * SB;
  const int ns = min(SB, N - s0);
  for (int t = threadIdx.x; t < ns; t += BLK) {
    const float* p = poses + 3 * (s0 + t);
    float sn, cs;
    sincosf(p[2], &sn, &cs);
    st[t] = make_float4(cs, sn, p[0], p[1]);
  }
  __syncthreads();

  const int wave_base = blockIdx.x * BLK + (threadIdx.x & ~63);
  if (wave_base >= M) return;
  const int i = blockIdx.x * BLK + threadIdx.x;
  const bool active = i < M;
  int e0 = 0, mi = 0;
  if (active) { e0 = off[i]; mi = off[i + 1] - e0; }
  Obst<MI> o;
  load_obstacle<MI>(o, ax, ay, bx, by, e0, mi, E, F.eps);
  const bool contributes = active && (mi != 0);
  const int lane = threadIdx.x & 63;

  for (int t = 0; t < ns; ++t) {
    const float4 q = st[t];
    // a non-finite pose makes every obstacle's sd NaN (min / max in the
    // pipeline would otherwise drop the NaN operands)
    const bool pose_ok = isfinite(q.x) && isfinite(q.y) && isfinite(q.z) && isfinite(q.w);
    uint32_t k = 0xffffffffu;
    if (contributes) k = pose_ok ? orderable(obstacle_sd<MF, MI>(F, o, q.x, q.y, q.z, q.w)) : 0u;
    const uint32_t kmin = wave_min_u32(k);
    if (kmin != 0xffffffffu) {
      const uint64_t hit = __ballot(k == kmin);
      const int first = __ffsll((unsigned long long)hit) - 1;
      if (lane == 0)
        atomicMin((unsigned long long*)&keys[s0 + t],
                  ((unsigned long long)kmin << 32) | (unsigned)(wave_base + first));
    }
  }
}

// One lane per stage.  mode 0: value only; 1: value + gradient; 2: bwd
// (gradient scaled by gout, written to grad only).
template <int MF, int MI>
__global__ __launch_bounds__(64) void epilogue_kernel(FpConst F, const float* __restrict__ poses,
                                                      int N, const float* __restrict__ ax,
                                                      const float* __restrict__ ay,
                                                      const float* __restrict__ bx,
                                                      const float* __restrict__ by,
                                                      const int* __restrict__ off, int E, int M,
                                                      const uint64_t* __restrict__ keys,
                                                      const float* __restrict__ gout, int mode,
                                                      float* __restrict__ d,
                                                      int* __restrict__ edge,
                                                      int* __restrict__ obst,
                                                      float* __restrict__ grad) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= N) return;
  const uint64_t key = keys[s];
  const float nan = __builtin_nanf("");
  float dv, g[3] = {0.f, 0.f, 0.f};
  int ev = -1, ov = -1;
  if (key == kEmptyKey) {
    dv = __builtin_huge_valf();
  } else if ((key >> 32) == 0 || (key & 0xffffffffu) >= (uint64_t)M) {
    // NaN result, or a key that names no obstacle of this edge set
    dv = nan;
    g[0] = g[1] = g[2] = nan;
  } else {
    const int i = (int)(key & 0xffffffffu);
    const int e0 = off[i], mi = off[i + 1] - e0;
    Obst<MI> o;
    load_obstacle<MI>(o, ax, ay, bx, by, e0, mi, E, F.eps);
    const float* p = poses + 3 * s;
    float sn, cs;
    sincosf(p[2], &sn, &cs);
    const float scale = mode == 2 ? gout[s] : 1.0f;
    int jstar = 0;
    obstacle_adjoint<MF, MI>(F, o, cs, sn, p[0], p[1], scale, jstar, g);
    dv = from_orderable((uint32_t)(key >> 32));
    ov = i;
    ev = e0 + jstar;
  }
  if (mode == 2) {
    if (key == kEmptyKey) { g[0] = g[1] = g[2] = 0.f * gout[s]; }
    grad[3 * s + 0] = g[0];
    grad[3 * s + 1] = g[1];
    grad[3 * s + 2] = g[2];
    return;
  }
  d[s] = dv;
  edge[s] = ev;
  obst[s] = ov;
  if (mode == 1) {
    grad[3 * s + 0] = g[0];
    grad[3 * s + 1] = g[1];
    grad[3 * s + 2] = g[2];
  }
}

// ------------------------------------------------------------------ dispatch

template <int MF, int MI>
hipError_t launch_main_t(const LaunchShape& ls, const FpConst& F, const float* poses, int N,
                                const psdf_edges& e, uint64_t* keys, hipStream_t st) {
  dim3 grid((e.M + ls.blk - 1) / ls.blk, (N + ls.sb - 1) / ls.sb);
  if (ls.blk == 64)
    main_kernel<MF, MI, 64><<<grid, 64, 0, st>>>(F, poses, N, ls.sb, e.ax, e.ay, e.bx, e.by,
                                                  e.obst_off, e.E, e.M, keys);
  else
    main_kernel<MF, MI, 256><<<grid, 256, 0, st>>>(F, poses, N, ls.sb, e.ax, e.ay, e.bx, e.by,
                                                    e.obst_off, e.E, e.M, keys);
  return hipGetLastError();
}

template <int MF, int MI>
hipError_t launch_epi_t(const FpConst& F, const float* poses, int N, const psdf_edges& e,
                               const uint64_t* keys, const float* gout, int mode, float* d,
                               int* edge, int* obst, float* grad, hipStream_t st) {
  epilogue_kernel<MF, MI><<<(N + 63) / 64, 64, 0, st>>>(F, poses, N, e.ax, e.ay, e.bx, e.by,
                                                         e.obst_off, e.E, e.M, keys, gout, mode, d,
                                                         edge, obst, grad);
  return hipGetLastError();
}

template <int MF>
hipError_t launch_main_mf(int mi_class, const LaunchShape& ls, const FpConst& F,
                          const float* poses, int N, const psdf_edges& e, uint64_t* keys,
                          hipStream_t st) {
  if (mi_class == 4) return launch_main_t<MF, 4>(ls, F, poses, N, e, keys, st);
  if (mi_class == 8) return launch_main_t<MF, 8>(ls, F, poses, N, e, keys, st);
  return launch_main_t<MF, 16>(ls, F, poses, N, e, keys, st);
}

template <int MF>
hipError_t launch_epi_mf(int mi_class, const FpConst& F, const float* poses, int N,
                         const psdf_edges& e, const uint64_t* keys, const float* gout, int mode,
                         float* d, int* edge, int* obst, float* grad, hipStream_t st) {
  if (mi_class == 4) return launch_epi_t<MF, 4>(F, poses, N, e, keys, gout, mode, d, edge, obst, grad, st);
  if (mi_class == 8) return launch_epi_t<MF, 8>(F, poses, N, e, keys, gout, mode, d, edge, obst, grad, st);
  return launch_epi_t<MF, 16>(F, poses, N, e, keys, gout, mode, d, edge, obst, grad, st);
}

#define PSDF_EXTERN_MF(MF)                                                                     \
  extern template hipError_t launch_main_mf<MF>(int, const LaunchShape&, const FpConst&,       \
                                                const float*, int, const psdf_edges&,          \
                                                uint64_t*, hipStream_t);                       \
  extern template hipError_t launch_epi_mf<MF>(int, const FpConst&, const float*, int,         \
                                               const psdf_edges&, const uint64_t*, const float*, \
                                               int, float*, int*, int*, float*, hipStream_t);
PSDF_EXTERN_MF(3)
PSDF_EXTERN_MF(4)
PSDF_EXTERN_MF(5)
PSDF_EXTERN_MF(6)
PSDF_EXTERN_MF(7)
PSDF_EXTERN_MF(8)
PSDF_EXTERN_MF(16)

}  // namespace psdf
