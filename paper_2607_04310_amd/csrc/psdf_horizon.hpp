// Horizon pass of the screened batch: every obstacle's bounding circle and
// each instance's horizon list (the obstacles its stages screen), launched by
// psdf_batch_screened / psdf_batch_screened_bound before the per-stage
// screening kernels (psdf_screen.hpp).
#pragma once

#include <hip/hip_runtime.h>

#include "psdf_batch.hpp"
#include "psdf_mlp.hpp"
#include "psdf_screen.hpp"

namespace psdf {

// Bounding circle (cx, cy, r, 0) of an obstacle with edges [a, b) of an
// instance, from its edges in one pass, r inflated to cover rounding.  An
// empty obstacle gets cx = NaN (never screened); an invalid one (bad range,
// more than MI edges or a non-finite coordinate) r = +inf (always a
// candidate), and so does an open chain of two or more edges: the axis test
// sees the convex hull of its points, whose closing edge gives no axis, so
// the certificate's separation argument does not hold for it.  All MI edge
// loads are issued together (indices clamped into the obstacle's range; a
// four-edge obstacle at 16-byte aligned addresses takes one vector load per
// array); edges past the obstacle's own count add nothing.
template <int MI>
__device__ float4 obstacle_circle(const BatchInst& in, const float* __restrict__ ax,
                                  const float* __restrict__ ay, const float* __restrict__ bx,
                                  const float* __restrict__ by, int a, int b) {
  const int mi = b - a;
  float4 c = make_float4(__builtin_nanf(""), 0.f, 0.f, 0.f);
  if (mi != 0) {
    c = make_float4(0.f, 0.f, __builtin_huge_valf(), 0.f);
    if (mi > 0 && mi <= MI && a >= 0 && b <= in.E) {
      float px[2 * MI], py[2 * MI];
      const int e0 = in.edge_off + a;
      const uintptr_t al = reinterpret_cast<uintptr_t>(ax + e0) | reinterpret_cast<uintptr_t>(ay + e0) |
                           reinterpret_cast<uintptr_t>(bx + e0) | reinterpret_cast<uintptr_t>(by + e0);
      if (MI >= 4 && mi == 4 && (al & 15u) == 0) {
        // four edges at 16-byte aligned addresses: one vector load per array
        const float4 a4 = *reinterpret_cast<const float4*>(ax + e0);
        const float4 b4 = *reinterpret_cast<const float4*>(ay + e0);
        const float4 c4 = *reinterpret_cast<const float4*>(bx + e0);
        const float4 d4 = *reinterpret_cast<const float4*>(by + e0);
        const float xa[4] = {a4.x, a4.y, a4.z, a4.w}, ya[4] = {b4.x, b4.y, b4.z, b4.w};
        const float xb[4] = {c4.x, c4.y, c4.z, c4.w}, yb[4] = {d4.x, d4.y, d4.z, d4.w};
#pragma unroll
        for (int j = 0; j < MI; ++j) {
          const int jj = j < 4 ? j : 3;
          px[2 * j] = xa[jj]; py[2 * j] = ya[jj];
          px[2 * j + 1] = xb[jj]; py[2 * j + 1] = yb[jj];
        }
      } else {
#pragma unroll
        for (int j = 0; j < MI; ++j) {
          const int e = e0 + min(j, mi - 1);
          px[2 * j] = ax[e]; py[2 * j] = ay[e];
          px[2 * j + 1] = bx[e]; py[2 * j + 1] = by[e];
        }
      }
      float sx = 0.f, sy = 0.f;
      bool finite = true;
#pragma unroll
      for (int j = 0; j < MI; ++j) {
        if (j < mi) {
          sx += px[2 * j] + px[2 * j + 1];
          sy += py[2 * j] + py[2 * j + 1];
          finite = finite && isfinite(px[2 * j]) && isfinite(py[2 * j]) &&
                   isfinite(px[2 * j + 1]) && isfinite(py[2 * j + 1]);
        }
      }
      // closed polygon: B_j == A_{j+1} bitwise, around the boundary
      bool closed = mi >= 3;
#pragma unroll
      for (int j = 0; j < MI; ++j)
        if (j < mi) {
          const int nx = j + 1 < mi ? j + 1 : 0;
          float ax1 = px[0], ay1 = py[0];
#pragma unroll
          for (int q = 1; q < MI; ++q)
            if (q == nx) { ax1 = px[2 * q]; ay1 = py[2 * q]; }
          closed = closed && __float_as_uint(px[2 * j + 1]) == __float_as_uint(ax1) &&
                   __float_as_uint(py[2 * j + 1]) == __float_as_uint(ay1);
        }
      if (finite && (closed || mi == 1)) {
        const float cx = sx / (2.f * mi), cy = sy / (2.f * mi);
        float r2 = 0.f;
#pragma unroll
        for (int j = 0; j < 2 * MI; ++j)
          if (j < 2 * mi) {
            const float dx = px[j] - cx, dy = py[j] - cy;
            r2 = fmaxf(r2, fmaf(dx, dx, dy * dy));
          }
        c = make_float4(cx, cy, sqrtf(r2) * (1.0f + 1e-6f) + 1e-6f, 0.f);
      }
    }
  }
  return c;
}

// Horizon list of each instance: every stage position of the instance lies
// within R of the centre c_p of their bounding box, so for every stage s and
// obstacle i
//   |p_s - c_i| - r_i - rmax - gamma >= |c_p - c_i| - R - r_i - rmax - gamma =: hb_i,
// a lower bound of the stage's circle bound and hence of sd_i.  Grid
// (kHorizonSplit, instances): work-group c takes the c-th block of the
// instance's obstacles, computes their bounding circles (obstacle_circle),
// and appends its (about) kHorizonPool / kHorizonSplit lowest-hb obstacles to
// the list as (circle, index); the list thus holds every obstacle among the
// kHorizonPool / kHorizonSplit lowest of the whole instance.  The smallest hb
// left out (atomic minimum over the blocks) bounds every excluded obstacle at
// every stage.  A non-finite stage position disables the list (-1); a list
// longer than kHorizonCap (tie blocks) is not used by the stage pass either:
// the instance's stages then take the full evaluation.  On entry the
// instance's count is 0 and its bound +inf (plan creation, then the end of
// every screened call: its finish kernel, or in the bound form its last
// fallback launch).  Work-group (0, 0) also clears the n_sctrl screening
// counters (failed-stage counts) that the call's screen launches append
// with.  With a network the grid has one more
// column, whose first work-group builds the network's fragment table.
// circ (may be null): the instances' bounding circles taken once per edge
// set (circle_kernel, psdf_batch_stage), indexed like the lists; without it
// the circles are derived from the edges here.  The circle (or offset)
// loads are issued before the stage positions' bounding box is reduced, so
// their latency overlaps that phase.
// List length: each stage's lower-bound pass reads the whole list, and the
// bound of the obstacles left out must stay above the stages' minima for the
// certificate (on c5, 512 certifies every stage; 256 fails 6 % of them).
constexpr int kHorizonPool = 512;
constexpr int kHorizonSplit = 16;
constexpr int kHorizonKeys = kScreenMaxM / kHorizonSplit / kScreenThreads;   // 4

template <int MI>
__global__ __launch_bounds__(kScreenThreads) void horizon_kernel(
    const FpConst* __restrict__ fps, const BatchInst* __restrict__ insts,
    const float* __restrict__ poses, const float* __restrict__ ax, const float* __restrict__ ay,
    const float* __restrict__ bx, const float* __restrict__ by, const int* __restrict__ off,
    const float4* __restrict__ circ, float4* __restrict__ hlist, int* __restrict__ hcount,
    uint32_t* __restrict__ hrest, const float* __restrict__ theta, uint4* __restrict__ frag,
    unsigned* __restrict__ sctrl, int n_sctrl) {
  __shared__ int scan[kScreenThreads];
  // one slot per combined reduction below (none is reused, so none needs a
  // barrier after its reads): 5 + 2 + 3 + 2 groups of kWaves words
  __shared__ uint32_t rs[12 * kWaves];
  __shared__ int s_base;
  if (blockIdx.x == 0 && blockIdx.y == 0 && (int)threadIdx.x < n_sctrl) sctrl[threadIdx.x] = 0u;
  if (blockIdx.x == kHorizonSplit) {
    // the extra column: the screener network's per-lane weight fragments,
    // once per call (one wave), so that every stage's work-group reads them
    // with coalesced vector loads instead of gathering the parameters
    if (blockIdx.y == 0 && theta && threadIdx.x < 64) {
      MlpFrag f;
      mlp_load(theta, f);
      mlp_frag_store(f, frag);
    }
    return;
  }
  const int inst = blockIdx.y, part = blockIdx.x, tid = threadIdx.x;
  const BatchInst in = insts[inst];
  const FpConst& F = fp_const(fps, inst);   // uniform fields: scalar loads
  const int M = in.M;
  const int chunk = (M + kHorizonSplit - 1) / kHorizonSplit;
  const int o0 = part * chunk, o1 = min(M, o0 + chunk);
  if (o0 >= o1) return;   // empty block: nothing to add
  // the thread's obstacles: their staged circles, or their edge ranges,
  // loaded together (an index past the block is clamped to its last
  // obstacle, o1 - 1 < M)
  float4 cq[kHorizonKeys];
  int ea[kHorizonKeys], eb[kHorizonKeys];
#pragma unroll
  for (int q = 0; q < kHorizonKeys; ++q) {
    const int o = min(o0 + tid + kScreenThreads * q, o1 - 1);
    if (circ) {
      cq[q] = circ[in.circ_off + o];
      ea[q] = eb[q] = 0;
    } else {
      cq[q] = make_float4(0.f, 0.f, 0.f, 0.f);
      ea[q] = off[in.obst_off + o];
      eb[q] = off[in.obst_off + o + 1];
    }
  }
  // bounding box of the stage positions (orderable keys: min of x, y, -x, -y)
  uint32_t bx0 = 0xffffffffu, by0 = 0xffffffffu, bx1 = 0xffffffffu, by1 = 0xffffffffu;
  int bad = 0;
  // the thread's first stage position stays in registers for the radius
  // pass below (all of them when N <= kScreenThreads)
  float x0 = 0.f, y0 = 0.f;
  for (int t = tid; t < in.N; t += kScreenThreads) {
    const float* p = poses + 3 * (in.pose_off + t);
    const float x = p[0], y = p[1];
    if (t == tid) { x0 = x; y0 = y; }
    if (!(isfinite(x) && isfinite(y))) { bad = 1; continue; }
    bx0 = min(bx0, orderable(x)); by0 = min(by0, orderable(y));
    bx1 = min(bx1, orderable(-x)); by1 = min(by1, orderable(-y));
  }
  {
    uint32_t mn[4] = {bx0, by0, bx1, by1};
    int sm[1] = {bad};
    block_reduce<4, 1>(mn, sm, rs);
    bx0 = mn[0]; by0 = mn[1]; bx1 = mn[2]; by1 = mn[3];
    bad = sm[0];
  }
  if (bad > 0 || in.N == 0) {
    if (tid == 0 && part == 0) hcount[inst] = -1;
    return;
  }
  const float cx = 0.5f * (from_orderable(bx0) - from_orderable(bx1));
  const float cy = 0.5f * (from_orderable(by0) - from_orderable(by1));
  // R = max distance of a stage position from the centre (max via the
  // orderable image of -d)
  uint32_t nr = 0xffffffffu;
  for (int t = tid; t < in.N; t += kScreenThreads) {
    float x = x0, y = y0;
    if (t != tid) {
      const float* p = poses + 3 * (in.pose_off + t);
      x = p[0];
      y = p[1];
    }
    const float dx = x - cx, dy = y - cy;
    nr = min(nr, orderable(-sqrtf(fmaf(dx, dx, dy * dy))));
  }
  {
    uint32_t mn[1] = {nr};
    int sm[1] = {0};
    block_reduce<1, 1>(mn, sm, rs + 5 * kWaves);
    nr = mn[0];
  }
  const float R = -from_orderable(nr) * (1.0f + 1e-6f) + 1e-6f;
  const float hoff = R + F.rmax + kLbGamma;
  uint32_t k[kHorizonKeys];
  uint32_t kmin = 0xffffffffu, kmax = 0u;
  int used = 0;
#pragma unroll
  for (int q = 0; q < kHorizonKeys; ++q) {
    const int o = o0 + tid + kScreenThreads * q;
    uint32_t key = 0xffffffffu;
    if (o < o1) {
      if (!circ) cq[q] = obstacle_circle<MI>(in, ax, ay, bx, by, ea[q], eb[q]);
      const float4 c = cq[q];
      if (c.x == c.x) {
        const float dx = cx - c.x, dy = cy - c.y;
        key = orderable(sqrtf(fmaf(dx, dx, dy * dy)) - c.z - hoff);
      }
    }
    k[q] = key;
    if (key != 0xffffffffu) { kmin = min(kmin, key); kmax = max(kmax, key); ++used; }
  }
  int n_used;
  {
    uint32_t mn[2] = {kmin, ~kmax};
    int sm[1] = {used};
    block_reduce<2, 1>(mn, sm, rs + 7 * kWaves);
    kmin = mn[0]; kmax = ~mn[1]; n_used = sm[0];
  }
  constexpr int P = kHorizonPool / kHorizonSplit;
  const uint32_t T = n_used > P ? block_threshold<kHorizonKeys>(k, kHorizonKeys, kmin, kmax,
                                                                P / 2, P, scan)
                                : 0xfffffffeu;
  int mine = 0;
  uint32_t rest = 0xffffffffu;
#pragma unroll
  for (int q = 0; q < kHorizonKeys; ++q) {
    if (k[q] == 0xffffffffu) continue;
    if (k[q] <= T) ++mine;
    else rest = min(rest, k[q]);
  }
  int total = 0;
  int at = block_scan_min(mine, rest, rs + 10 * kWaves, &total, &rest);
  if (tid == 0) {
    s_base = total > 0 ? atomicAdd(&hcount[inst], total) : 0;
    if (rest != 0xffffffffu) atomicMin(&hrest[inst], rest);
  }
  __syncthreads();
  at += s_base;
  // the instance's list has M slots and holds each obstacle at most once,
  // as its circle with the local index in .w; a count that did not start at
  // zero (a call that stopped before reopening the lists) could pass M, so
  // slots past M are not written (the stage passes then find the count
  // above M and take the full evaluation)
#pragma unroll
  for (int q = 0; q < kHorizonKeys; ++q)
    if (k[q] != 0xffffffffu && k[q] <= T) {
      const int o = o0 + tid + kScreenThreads * q;
      float4 c = cq[q];
      c.w = __int_as_float(o);
      if (at >= 0 && at < M) hlist[in.circ_off + at] = c;
      ++at;
    }
}

// The pose-independent part of the screened forms, taken once per edge set
// (psdf_batch_stage): every obstacle's bounding circle (obstacle_circle) and
// its staged row (write_row: the registers the screen kernels' exact
// evaluation loads, made by load_obstacle + own_intervals exactly as they
// do), both indexed like the horizon lists (circ_off + obstacle).  Grid
// (ceil(max M / 256), instances).
template <int MI>
__global__ __launch_bounds__(256) void stage_batch_kernel(
    const FpConst* __restrict__ fps, const BatchInst* __restrict__ insts,
    const float* __restrict__ ax, const float* __restrict__ ay, const float* __restrict__ bx,
    const float* __restrict__ by, const int* __restrict__ off, float4* __restrict__ circ,
    unsigned char* __restrict__ rows) {
  const BatchInst in = insts[blockIdx.y];
  const int o = blockIdx.x * 256 + threadIdx.x;
  if (o >= in.M) return;
  const int a = off[in.obst_off + o], b = off[in.obst_off + o + 1];
  circ[in.circ_off + o] = obstacle_circle<MI>(in, ax, ay, bx, by, a, b);
  const int mi = b - a;
  Obst<MI> ob;
  load_obstacle<MI>(ob, ax, ay, bx, by, in.edge_off + a, mi, in.edge_off + in.E,
                    fps[blockIdx.y].eps);
  if (a < 0) ob.bad = true;
  own_intervals<MI>(ob);
  write_row<MI>(rows, (size_t)in.circ_off + o, ob, a, mi);
}

}  // namespace psdf
