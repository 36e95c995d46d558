// Persistent kernel of psdf_batch.
//
// Work items (instance, stage block, obstacle tile) are grouped by footprint
// size; one persistent launch per group pulls its items from a device
// counter, largest first.  For an item, lane <-> obstacle of the tile (edges
// in registers), the work-group loops over the stage block exactly as the
// plain per-stage minimum kernel does and writes one partial key and aux word
// per stage.  A second kernel (batch_finish_kernel, one wave per stage)
// reduces each stage's partial row, runs the winner adjoint and writes the
// outputs, and clears the item counters for the next launch: the kernel
// boundary orders the partials before their readers, which costs less on
// this chip than a device-scope release per item (each one writes back the
// L2 of the issuing XCD).  No work-group ever waits for another.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "psdf_device.hpp"
#include "psdf_host.hpp"
#include "psdf_winner.hpp"

namespace psdf {

struct BatchInst {
  int pose_off, N, edge_off, E, obst_off, M;
  int part_off;   // first partial slot: partial[part_off + s * nt + tile]
  int nt;         // obstacle tiles
  int m;          // footprint vertices
  int circ_off;   // first bounding circle of this instance's obstacles (screening)
};

// What the finish kernel needs of a stage's instance, one record per stage,
// so that its first loads (record, pose, key) do not wait on an instance
// lookup.  row = part_off + (stage - pose_off) * nt: the stage's partial row
// (depends on the tile width, so it is rewritten with the shape).
struct FinStage {
  int inst, row, nt, obst_off, M, edge_off, E, pad;
};

struct BatchItem {
  int inst, s0, ns, o0, no, tile;
};

struct BatchArgs {
  const FpConst* fps;
  const BatchInst* insts;
  const BatchItem* items;   // this launch's items (one footprint-size group)
  int n_items;
  int sb;
  int direct;               // 1: one item per work-group (item = blockIdx.x), no counter
  const float* poses;
  const float* ax;
  const float* ay;
  const float* bx;
  const float* by;
  const int* off;
  uint64_t* partial;
  uint64_t* aux;
  unsigned* ctrl;   // this launch's [0] next item
  float* d;
  int* edge;
  int* obst;
  float* grad;
  uint64_t* keys;
};

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Instance inst's footprint constants read through the constant address
// space: the table is written before a launch and never during it, so the
// compiler may keep its uniform fields in scalar registers or reload them
// with scalar loads instead of vector loads (same values).
__device__ __forceinline__ const FpConst& fp_const(const FpConst* fps, int inst) {
  typedef const __attribute__((address_space(4))) FpConst FpC;
  return *(const FpConst*)((FpC*)fps + inst);
}

// The winner's global edge range [e0, e0 + mi) from a final key whose low
// word is the obstacle's index local to its instance (the screened forms):
// false for the empty key, a NaN-free key that names no obstacle of the
// instance, or an offset pair outside the instance's edges.
__device__ __forceinline__ bool key_range(uint64_t key, const int* __restrict__ off, int obst_off,
                                          int M, int edge_off, int E, int& e0, int& mi) {
  const int i = (int)(key & 0xffffffffu);
  e0 = 0;
  mi = 0;
  if (key == kEmptyKey || (key >> 32) == 0 || (uint64_t)i >= (uint64_t)M) return false;
  e0 = off[obst_off + i];
  mi = off[obst_off + i + 1] - e0;
  e0 += edge_off;
  return mi >= 1 && mi <= kMaxObst && e0 >= edge_off && e0 <= edge_off + E - mi;
}

// Stage g's outputs from its final key (Sec. IV-D: the winner adjoint of
// the winning obstacle, edges [e0, e0 + mi) global): an empty key gives the
// empty-set result (d = +inf, no winner, zero gradient); a key that names
// no usable obstacle (valid false) gives NaN.  One whole wave with uniform
// arguments; fl must hold F (stage_footprint) and be visible to the wave.
// Every kernel that ends a stage goes through here, so a stage's outputs do
// not depend on which kernel finished it.
__device__ __forceinline__ void write_stage(const FpConst& F, const FpLds& fl, WinnerLds& wl,
                                            const float* __restrict__ ax,
                                            const float* __restrict__ ay,
                                            const float* __restrict__ bx,
                                            const float* __restrict__ by, uint64_t key,
                                            bool valid, int e0, int mi, int edge_off, float cs,
                                            float sn, float px, float py, int g,
                                            uint64_t* __restrict__ keys, float* __restrict__ d,
                                            int* __restrict__ edge, int* __restrict__ obst,
                                            float* __restrict__ grad) {
  float dv = __builtin_huge_valf(), gv[3] = {0.f, 0.f, 0.f};
  int ev = -1, ov = -1;
  if (key != kEmptyKey && !valid) {
    dv = __builtin_nanf("");
    gv[0] = gv[1] = gv[2] = dv;
  } else if (valid) {
    int jstar = 0;
    winner_adjoint(F, fl, wl, ax, ay, bx, by, e0, mi, cs, sn, px, py, true, jstar, gv);
    dv = from_orderable((uint32_t)(key >> 32));
    ov = (int)(key & 0xffffffffu);
    ev = e0 - edge_off + jstar;
  }
  if ((threadIdx.x & 63) == 0) {
    keys[g] = key;
    d[g] = dv;
    edge[g] = ev;
    obst[g] = ov;
    grad[3 * g + 0] = gv[0];
    grad[3 * g + 1] = gv[1];
    grad[3 * g + 2] = gv[2];
  }
}

// Waves per SIMD the compiler must fit: four for four-edge obstacles with a
// footprint of at most six slots, whose register need (154 VGPRs at six
// slots with the own-axis intervals hoisted, three waves) then fits 128
// with the intervals taken lazily (A/B runs on c5 at six slots: four waves
// 2 % faster than three; lazy intervals at four waves, no spills, 0.8 %
// faster than hoisted ones with spills); larger footprints and edge classes
// would spill far more and keep the compiler's own choice.
template <int MF, int MI>
constexpr int kBatchWavesPerEU = (MI == 4 && MF <= 6) ? 4 : 1;

// One launch per footprint-size group: MF footprint slots, MI obstacle edge
// class, NW waves per work-group (64 NW obstacles per tile).
template <int MF, int MI, int NW>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(kBatchWavesPerEU<MF, MI>)))
void batch_kernel(BatchArgs A) {
  __shared__ int s_item;
  __shared__ float4 st[kMaxStageBlock];
  __shared__ float4 rft[kMaxStageBlock * MF];
  __shared__ uint64_t wk[NW][kMaxStageBlock];
  __shared__ uint64_t wa[NW][kMaxStageBlock];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;

  for (int round = 0;; ++round) {
    if (A.direct) {
      if (round > 0) break;
      if (threadIdx.x == 0) s_item = (int)blockIdx.x;
    } else if (threadIdx.x == 0) {
      s_item = (int)atomicAdd(&A.ctrl[0], 1u);
    }
    __syncthreads();
    const int it = uniform(s_item);
    if (it >= A.n_items) break;
    const BatchItem item = A.items[it];
    const int inst = uniform(item.inst), s0 = uniform(item.s0), ns = uniform(item.ns);
    const int o0 = uniform(item.o0), no = uniform(item.no), tile = uniform(item.tile);
    const BatchInst in = A.insts[inst];
    const FpConst& F = fp_const(A.fps, inst);

    // obstacle of this lane (indices local to the instance; edges global)
    const int ol = w * 64 + lane;
    const bool active = ol < no;
    int e0 = 0, mi = 0;
    if (active) {
      const int* off = A.off + in.obst_off;
      e0 = off[o0 + ol];
      mi = off[o0 + ol + 1] - e0;
      e0 += in.edge_off;
    }
    const bool local_bad = active && e0 < in.edge_off;   // negative local offset
    fill_stage_table<MF>(F, A.poses, in.pose_off + s0, ns, st, rft, 64 * NW);
    __syncthreads();

    if (w * 64 < no) {
      auto emit = [&](int t, uint64_t key, uint64_t a) {
        if (lane == 0) { wk[w][t] = key; wa[w][t] = a; }
      };
      // lazy own-axis intervals: at four waves per SIMD the hoisted form
      // needs more registers than fit (spills), the lazy one none
      wave_stages<MF, MI, decltype(emit), true>(F, A.ax, A.ay, A.bx, A.by, e0, mi,
                                                in.edge_off + in.E, active, local_bad,
                                                o0 + w * 64, ns, st, rft, emit);
    } else if (lane == 0) {
      for (int t = 0; t < ns; ++t) { wk[w][t] = kEmptyKey; wa[w][t] = 0; }
    }
    __syncthreads();
    for (int t = threadIdx.x; t < ns; t += 64 * NW) {
      uint64_t k = wk[0][t], a = wa[0][t];
#pragma unroll
      for (int v = 1; v < NW; ++v)
        if (wk[v][t] < k) { k = wk[v][t]; a = wa[v][t]; }
      const size_t slot = (size_t)in.part_off + (size_t)(s0 + t) * in.nt + tile;
      A.partial[slot] = k;
      A.aux[slot] = a;
    }
    __syncthreads();
  }
}

// ev0 / ev1 (may be null): events the dispatch itself records at its start
// and end (kernel timer).
template <int MF, int MI>
hipError_t launch_batch_t(int nw, int grid, const BatchArgs& a, hipStream_t st, hipEvent_t ev0,
                          hipEvent_t ev1) {
  if (nw == 1)
    hipExtLaunchKernelGGL(batch_kernel<MF, MI, 1>, dim3(grid), dim3(64), 0, st, ev0, ev1, 0, a);
  else
    hipExtLaunchKernelGGL(batch_kernel<MF, MI, 4>, dim3(grid), dim3(256), 0, st, ev0, ev1, 0, a);
  return hipGetLastError();
}

template <int MF, int MI>
hipError_t batch_occupancy_t(int nw, int* blocks_per_cu) {
  if (nw == 1)
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, batch_kernel<MF, MI, 1>, 64, 0);
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, batch_kernel<MF, MI, 4>, 256, 0);
}

// Per footprint-size entry points (instantiated in psdf_batch_mf*.hip).
template <int MF>
hipError_t launch_batch_mf(int mi_class, int nw, int grid, const BatchArgs& a, hipStream_t st,
                           hipEvent_t ev0, hipEvent_t ev1) {
  if (mi_class == 4) return launch_batch_t<MF, 4>(nw, grid, a, st, ev0, ev1);
  if (mi_class == 8) return launch_batch_t<MF, 8>(nw, grid, a, st, ev0, ev1);
  return launch_batch_t<MF, 16>(nw, grid, a, st, ev0, ev1);
}

template <int MF>
hipError_t batch_occupancy_mf(int mi_class, int nw, int* blocks_per_cu) {
  if (mi_class == 4) return batch_occupancy_t<MF, 4>(nw, blocks_per_cu);
  if (mi_class == 8) return batch_occupancy_t<MF, 8>(nw, blocks_per_cu);
  return batch_occupancy_t<MF, 16>(nw, blocks_per_cu);
}

#define PSDF_EXTERN_BATCH(MF)                                                                  \
  extern template hipError_t launch_batch_mf<MF>(int, int, int, const BatchArgs&, hipStream_t, \
                                                 hipEvent_t, hipEvent_t);                      \
  extern template hipError_t batch_occupancy_mf<MF>(int, int, int*);
PSDF_EXTERN_BATCH(3)
PSDF_EXTERN_BATCH(4)
PSDF_EXTERN_BATCH(5)
PSDF_EXTERN_BATCH(6)
PSDF_EXTERN_BATCH(7)
PSDF_EXTERN_BATCH(8)
PSDF_EXTERN_BATCH(16)

}  // namespace psdf
