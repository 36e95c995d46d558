// Winner adjoint, one wave per stage.
//
// Given the winning obstacle of a stage, a whole wave (64 lanes) recomputes
// that obstacle's pipeline with the same device arithmetic as obstacle_sd
// and returns:
//   * the reported edge: the smallest per-edge pool distance, lowest index
//     on ties (the pool entries of a V_obs point A~_j or B~_j belong to edge
//     j, and for a closed polygon A~_j also to edge j - 1);
//   * the pose gradient, the reverse-mode adjoint through the active branch
//     of every min / max (Sec. IV-D active-branch subgradient): in the
//     separated branch through the winning point-segment pair (first entry on
//     ties), otherwise through the soft-min weights of the axis overlaps and,
//     for each axis, the first extreme vertices of both intervals.
// Lanes share the work: one pool entry per lane (strided), one SAT axis per
// lane; the winner's local geometry is staged in LDS.
//
// The adjoint is contracted on the fly: a local point P~ with adjoint gP
// contributes -R gP to d/dp and gP . (P~_y, -P~_x) to d/dtheta (P~ moves by
// -R^T dp + dtheta (P~_y, -P~_x)); a local edge vector v with adjoint gv
// contributes gv . (v_y, -v_x) to d/dtheta.
#pragma once

#include <hip/hip_runtime.h>

#include "psdf_device.hpp"

namespace psdf {

// Footprint constants staged in LDS for lane-indexed access.
struct FpLds {
  float vx[kMaxFp], vy[kMaxFp], ex[kMaxFp], ey[kMaxFp], einv[kMaxFp];
  float nx[kMaxFp], ny[kMaxFp], pa[kMaxFp], pb[kMaxFp];
};

// The winner's local geometry, one per wave.
struct WinnerLds {
  float tax[kMaxObst], tay[kMaxObst], vx[kMaxObst], vy[kMaxObst];
  float nx[kMaxObst], ny[kMaxObst], iv2[kMaxObst], il[kMaxObst];
  float px[2 * kMaxObst], py[2 * kMaxObst];   // V_obs: A~_k, then B~_k (open obstacles)
  unsigned epool[kMaxObst];                   // per-edge minimum d^2 (float bits)
};

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ---- cross-lane steps for a fully active wave (every lane of the wave
// takes part; results are wave-uniform).  DPP moves within rows of 16 lanes
// (quad swaps, half-row and row mirrors) reduce each row; reads of lanes 0,
// 16, 32 and 48 combine the rows.  Counts come from ballots.
constexpr int kDppXor1 = 0xB1;         // quad_perm [1, 0, 3, 2]
constexpr int kDppXor2 = 0x4E;         // quad_perm [2, 3, 0, 1]
constexpr int kDppHalfMirror = 0x141;  // lane i <- 7 - i within 8 lanes
constexpr int kDppMirror = 0x140;      // lane i <- 15 - i within 16 lanes
constexpr int kDppShr = 0x110;         // + n: lane i <- i - n within the row, 0 below

template <int C>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, C, 0xf, 0xf, true);
}
__device__ __forceinline__ uint32_t lane_u32(uint32_t x, int l) {
  return (uint32_t)__builtin_amdgcn_readlane((int)x, l);
}

__device__ __forceinline__ uint32_t fw_min_u32(uint32_t x) {
  x = min(x, dpp_u32<kDppXor1>(x));
  x = min(x, dpp_u32<kDppXor2>(x));
  x = min(x, dpp_u32<kDppHalfMirror>(x));
  x = min(x, dpp_u32<kDppMirror>(x));
  return min(min(lane_u32(x, 0), lane_u32(x, 16)), min(lane_u32(x, 32), lane_u32(x, 48)));
}

__device__ __forceinline__ int fw_sum_i32(int v) {
  uint32_t x = (uint32_t)v;
  x += dpp_u32<kDppXor1>(x);
  x += dpp_u32<kDppXor2>(x);
  x += dpp_u32<kDppHalfMirror>(x);
  x += dpp_u32<kDppMirror>(x);
  return (int)(lane_u32(x, 0) + lane_u32(x, 16) + lane_u32(x, 32) + lane_u32(x, 48));
}

template <int C>
__device__ __forceinline__ uint64_t dpp_u64(uint64_t x) {
  return ((uint64_t)dpp_u32<C>((uint32_t)(x >> 32)) << 32) | dpp_u32<C>((uint32_t)x);
}
__device__ __forceinline__ uint64_t lane_u64(uint64_t x, int l) {
  return ((uint64_t)lane_u32((uint32_t)(x >> 32), l) << 32) | lane_u32((uint32_t)x, l);
}
__device__ __forceinline__ uint64_t min_u64(uint64_t a, uint64_t b) { return b < a ? b : a; }

__device__ __forceinline__ uint64_t fw_min_u64(uint64_t x) {
  x = min_u64(x, dpp_u64<kDppXor1>(x));
  x = min_u64(x, dpp_u64<kDppXor2>(x));
  x = min_u64(x, dpp_u64<kDppHalfMirror>(x));
  x = min_u64(x, dpp_u64<kDppMirror>(x));
  return min_u64(min_u64(lane_u64(x, 0), lane_u64(x, 16)), min_u64(lane_u64(x, 32), lane_u64(x, 48)));
}

// Inclusive prefix sum over the wave; *total gets the wave's sum.
__device__ __forceinline__ int fw_scan_i32(int v, int* total) {
  uint32_t x = (uint32_t)v;
  x += dpp_u32<kDppShr + 1>(x);
  x += dpp_u32<kDppShr + 2>(x);
  x += dpp_u32<kDppShr + 4>(x);
  x += dpp_u32<kDppShr + 8>(x);
  const uint32_t t0 = lane_u32(x, 15), t1 = lane_u32(x, 31), t2 = lane_u32(x, 47),
                 t3 = lane_u32(x, 63);
  const int row = (threadIdx.x & 63) >> 4;
  x += (row > 0 ? t0 : 0u) + (row > 1 ? t1 : 0u) + (row > 2 ? t2 : 0u);
  *total = (int)(t0 + t1 + t2 + t3);
  return (int)x;
}

__device__ __forceinline__ float fw_sum_f32(float x) {
  x += __uint_as_float(dpp_u32<kDppXor1>(__float_as_uint(x)));
  x += __uint_as_float(dpp_u32<kDppXor2>(__float_as_uint(x)));
  x += __uint_as_float(dpp_u32<kDppHalfMirror>(__float_as_uint(x)));
  x += __uint_as_float(dpp_u32<kDppMirror>(__float_as_uint(x)));
  const uint32_t u = __float_as_uint(x);
  return (__uint_as_float(lane_u32(u, 0)) + __uint_as_float(lane_u32(u, 16))) +
         (__uint_as_float(lane_u32(u, 32)) + __uint_as_float(lane_u32(u, 48)));
}

__device__ __forceinline__ float fw_min_f32(float x) {
  x = fminf(x, __uint_as_float(dpp_u32<kDppXor1>(__float_as_uint(x))));
  x = fminf(x, __uint_as_float(dpp_u32<kDppXor2>(__float_as_uint(x))));
  x = fminf(x, __uint_as_float(dpp_u32<kDppHalfMirror>(__float_as_uint(x))));
  x = fminf(x, __uint_as_float(dpp_u32<kDppMirror>(__float_as_uint(x))));
  const uint32_t u = __float_as_uint(x);
  return fminf(fminf(__uint_as_float(lane_u32(u, 0)), __uint_as_float(lane_u32(u, 16))),
               fminf(__uint_as_float(lane_u32(u, 32)), __uint_as_float(lane_u32(u, 48))));
}

// Wave-wide reductions used by the kernels; every lane of the wave takes
// part (the callers reach them in wave-uniform control flow).
__device__ __forceinline__ uint32_t wave_min_u32(uint32_t x) { return fw_min_u32(x); }
__device__ __forceinline__ uint64_t wave_min_u64(uint64_t x) { return fw_min_u64(x); }
__device__ __forceinline__ float wave_min_f32(float x) { return fw_min_f32(x); }
__device__ __forceinline__ float wave_sum(float x) { return fw_sum_f32(x); }


// Copy the footprint constants into LDS, lane l <-> slot l: one vector load
// per array.  F must be addressable memory (global memory or the kernel
// argument segment), not a register copy.
__device__ __forceinline__ void stage_footprint(FpLds& L, const FpConst& F) {
  const int l = threadIdx.x & 63;
  if (l < kMaxFp) {
    L.vx[l] = F.vx[l]; L.vy[l] = F.vy[l]; L.ex[l] = F.ex[l]; L.ey[l] = F.ey[l];
    L.einv[l] = F.einv[l]; L.nx[l] = F.nx[l]; L.ny[l] = F.ny[l];
    L.pa[l] = F.pa[l]; L.pb[l] = F.pb[l];
  }
}

// Stage table of a block of ns stages starting at pose s0 (poses float[][3]):
// st[t] = (cos, sin, x, y) and rft[t * MF + l] = the footprint rotated by
// stage t's heading.  Filled by the whole work-group (nthreads lanes); the
// caller synchronises before use.
template <int MF>
__device__ __forceinline__ void fill_stage_table(const FpConst& F, const float* __restrict__ poses,
                                                 int s0, int ns, float4* st, float4* rft,
                                                 int nthreads) {
  for (int idx = threadIdx.x; idx < ns * MF; idx += nthreads) {
    const int t = idx / MF, l = idx - t * MF;
    const float* p = poses + 3 * (s0 + t);
    float sn, cs;
    sincosf(p[2], &sn, &cs);
    if (l == 0) st[t] = make_float4(cs, sn, p[0], p[1]);
    rft[idx] = rotated_slot(F, l, cs, sn);
  }
}

// Per-stage minimum over one wave's obstacles (lane <-> obstacle o, the
// lane's obstacle with its pose-independent constants in registers, edges
// [e0, e0 + mi)) for the ns stages of the table st (c, s, px, py) with their
// rotated footprints rft[t * MF + l] (rotated_slot).  For each stage
// emit(t, key, aux) receives the wave's minimum key (orderable(sd) << 32 |
// obase + lane of the first minimum, or the empty key) and that lane's
// (e0 << 32 | mi).  LAZY: see own_intervals.
template <int MF, int MIX, class Emit, bool LAZY = false>
__device__ __forceinline__ void wave_stage_loop(const FpConst& F, Obst<MIX>& o, int e0, int mi,
                                                bool active, int obase, int ns,
                                                const float4* st, const float4* rft, Emit emit) {
  const bool contributes = active && (mi != 0);
  for (int t = 0; t < ns; ++t) {
    const float4 q = st[t];
    // a non-finite pose makes every obstacle's sd NaN (min / max in the
    // pipeline would otherwise drop the NaN operands)
    const bool pose_ok = isfinite(q.x) && isfinite(q.y) && isfinite(q.z) && isfinite(q.w);
    uint32_t k = 0xffffffffu;
    if (contributes)
      k = pose_ok ? orderable(obstacle_sd<MF, MIX, LAZY>(F, o, rft + t * MF, q.z, q.w)) : 0u;
    const uint32_t kmin = wave_min_u32(k);
    uint64_t key = kEmptyKey, a = 0;
    if (kmin != 0xffffffffu) {
      const uint64_t hit = __ballot(k == kmin);
      const int first = __ffsll((unsigned long long)hit) - 1;
      key = ((uint64_t)kmin << 32) | (uint32_t)(obase + first);
      a = ((uint64_t)lane_u32((uint32_t)e0, first) << 32) | lane_u32((uint32_t)mi, first);
    }
    emit(t, key, a);
  }
}

// wave_stage_loop with the obstacle loaded from the edge arrays.  A wave
// whose obstacles all have at most one edge (free segments) takes the
// one-edge specialisation (wave_stages), the same arithmetic on one slot
// instead of MI.
template <int MF, int MIX, class Emit, bool LAZY = false>
__device__ __forceinline__ void wave_stages_t(const FpConst& F, const float* __restrict__ ax,
                                              const float* __restrict__ ay,
                                              const float* __restrict__ bx,
                                              const float* __restrict__ by, int e0, int mi,
                                              int Eend, bool active, bool bad, int obase, int ns,
                                              const float4* st, const float4* rft, Emit emit) {
  Obst<MIX> o;
  load_obstacle<MIX>(o, ax, ay, bx, by, e0, mi, Eend, F.eps);
  o.bad = o.bad || bad;
  wave_stage_loop<MF, MIX, Emit, LAZY>(F, o, e0, mi, active, obase, ns, st, rft, emit);
}

template <int MF, int MI, class Emit, bool LAZY = false>
__device__ __forceinline__ void wave_stages(const FpConst& F, const float* __restrict__ ax,
                                            const float* __restrict__ ay,
                                            const float* __restrict__ bx,
                                            const float* __restrict__ by, int e0, int mi, int Eend,
                                            bool active, bool bad, int obase, int ns,
                                            const float4* st, const float4* rft, Emit emit) {
  const bool segments = __ballot(active && mi > 1) == 0;
  if (MI > 1 && segments)
    wave_stages_t<MF, 1, Emit, LAZY>(F, ax, ay, bx, by, e0, mi, Eend, active, bad, obase, ns, st,
                                     rft, emit);
  else
    wave_stages_t<MF, MI, Emit, LAZY>(F, ax, ay, bx, by, e0, mi, Eend, active, bad, obase, ns, st,
                                      rft, emit);
}

// Whole-wave call with uniform arguments; the obstacle owns edges
// [e0, e0 + mi), 1 <= mi <= kMaxObst.  Results are uniform across the wave.
__device__ __forceinline__ void winner_adjoint(const FpConst& F, const FpLds& FL, WinnerLds& W,
                               const float* __restrict__ ax, const float* __restrict__ ay,
                               const float* __restrict__ bx, const float* __restrict__ by, int e0,
                               int mi, float c, float s, float px, float py, bool want_grad,
                               int& jstar, float g[3]) {
  const int lane = threadIdx.x & 63;
  const int m = F.m;

  // ---- stage the obstacle (lane j <-> edge j)
  bool open_edge = false;
  if (lane < mi) {
    const float a0 = ax[e0 + lane], a1 = ay[e0 + lane];
    const float b0 = bx[e0 + lane], b1 = by[e0 + lane];
    const int nxt = lane + 1 < mi ? lane + 1 : 0;
    const float n0 = ax[e0 + nxt], n1 = ay[e0 + nxt];
    open_edge = __float_as_uint(b0) != __float_as_uint(n0) || __float_as_uint(b1) != __float_as_uint(n1);
    float iv2, il, tx, ty, vx, vy;
    edge_consts(b0 - a0, b1 - a1, F.eps, iv2, il);
    local_point(a0, a1, c, s, px, py, tx, ty);
    local_vector(b0 - a0, b1 - a1, c, s, vx, vy);
    W.tax[lane] = tx; W.tay[lane] = ty; W.vx[lane] = vx; W.vy[lane] = vy;
    W.nx[lane] = -vy * il; W.ny[lane] = vx * il;
    W.iv2[lane] = iv2; W.il[lane] = il;
    W.px[lane] = tx; W.py[lane] = ty;
    W.px[mi + lane] = tx + vx; W.py[mi + lane] = ty + vy;
  }
  if (lane < kMaxObst) W.epool[lane] = 0x7f800000u;   // +inf
  const bool closed = mi >= 3 && __ballot(open_edge) == 0;
  const int nv = closed ? mi : 2 * mi;
  wave_sync();

  // ---- pools (Sec. IV-B): entry e < m*mi is robot vertex l = e / mi against
  // obstacle edge j = e % mi; the rest is V_obs point k against robot edge l.
  const int PV = m * mi, P = PV + nv * m;
  uint64_t best = ~0ull;
  for (int e = lane; e < P; e += 64) {
    float qx, qy, sax, say, svx, svy, siv;
    int ej, ej2 = -1;
    if (e < PV) {
      const int l = e / mi, j = e - l * mi;
      qx = FL.vx[l]; qy = FL.vy[l];
      sax = W.tax[j]; say = W.tay[j]; svx = W.vx[j]; svy = W.vy[j]; siv = W.iv2[j];
      ej = j;
    } else {
      const int e2 = e - PV, k = e2 / m, l = e2 - k * m;
      qx = W.px[k]; qy = W.py[k];
      sax = FL.vx[l]; say = FL.vy[l]; svx = FL.ex[l]; svy = FL.ey[l]; siv = FL.einv[l];
      ej = k < mi ? k : k - mi;
      if (closed) ej2 = k > 0 ? k - 1 : mi - 1;
    }
    const float d2 = seg_d2(qx, qy, sax, say, svx, svy, siv);
    atomicMin(&W.epool[ej], __float_as_uint(d2));
    if (ej2 >= 0) atomicMin(&W.epool[ej2], __float_as_uint(d2));
    const uint64_t key = ((uint64_t)__float_as_uint(d2) << 32) | (uint32_t)e;
    best = key < best ? key : best;
  }
  best = wave_min_u64(best);
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  wave_sync();
  {
    const uint64_t ek = lane < mi ? (((uint64_t)W.epool[lane] << 32) | (uint32_t)lane) : ~0ull;
    jstar = (int)(wave_min_u64(ek) & 0xffffffffu);
  }
  g[0] = g[1] = g[2] = 0.f;
  if (!want_grad) return;

  // ---- SAT (Sec. IV-C): lane q < m + mi owns axis q.
  const int K = m + mi;
  float dl = __builtin_huge_valf(), nxq = 0.f, nyq = 0.f;
  float lox = 0.f, loy = 0.f, hix = 0.f, hiy = 0.f;      // obstacle extremes
  float rlx = 0.f, rly = 0.f, rhx = 0.f, rhy = 0.f;      // robot extremes (obstacle axes)
  int br = 0;
  if (lane < K) {
    float alo, ahi;
    if (lane < m) {
      nxq = FL.nx[lane]; nyq = FL.ny[lane];
      alo = FL.pa[lane]; ahi = FL.pb[lane];
    } else {
      const int j = lane - m;
      nxq = W.nx[j]; nyq = W.ny[j];
      alo = __builtin_huge_valf(); ahi = -__builtin_huge_valf();
      for (int l = 0; l < m; ++l) {
        const float p = fmaf(FL.vx[l], nxq, FL.vy[l] * nyq);
        if (p < alo) { alo = p; rlx = FL.vx[l]; rly = FL.vy[l]; }
        if (p > ahi) { ahi = p; rhx = FL.vx[l]; rhy = FL.vy[l]; }
      }
    }
    float lo = __builtin_huge_valf(), hi = -__builtin_huge_valf();
    for (int k = 0; k < nv; ++k) {
      const float wx = W.px[k], wy = W.py[k];
      const float p = fmaf(wx, nxq, wy * nyq);
      if (p < lo) { lo = p; lox = wx; loy = wy; }
      if (p > hi) { hi = p; hix = wx; hiy = wy; }
    }
    const float d1 = hi - alo, d2 = ahi - lo;
    dl = fminf(d1, d2);
    br = d1 <= d2 ? 0 : 1;
  }
  const bool sep = __ballot(lane < K && dl < -F.eps_sat) != 0;

  float sx = 0.f, sy = 0.f, gth = 0.f;
  if (sep) {
    // d sd / d(d^2) through the winning pair: d^2 = |w - t V|^2, w = Q - A
    const int e = (int)(best & 0xffffffffu);
    const float d2b = __uint_as_float((uint32_t)(best >> 32));
    float qx, qy, sax, say, svx, svy, siv;
    const bool vtype = e < PV;
    if (vtype) {
      const int l = e / mi, j = e - l * mi;
      qx = FL.vx[l]; qy = FL.vy[l];
      sax = W.tax[j]; say = W.tay[j]; svx = W.vx[j]; svy = W.vy[j]; siv = W.iv2[j];
    } else {
      const int e2 = e - PV, k = e2 / m, l = e2 - k * m;
      qx = W.px[k]; qy = W.py[k];
      sax = FL.vx[l]; say = FL.vy[l]; svx = FL.ex[l]; svy = FL.ey[l]; siv = FL.einv[l];
    }
    const float coef = 1.0f / (2.0f * sqrtf(d2b));
    const float wx = qx - sax, wy = qy - say;
    const float u = fmaf(wx, svx, wy * svy) * siv;
    const float t = clamp01(u);
    const float tp = (u > 0.f && u < 1.f) ? 1.f : 0.f;
    const float rx = 2.f * coef * fmaf(-t, svx, wx), ry = 2.f * coef * fmaf(-t, svy, wy);
    const float rv = fmaf(rx, svx, ry * svy) * tp * siv;
    const float gwx = rx - rv * svx, gwy = ry - rv * svy;   // d/dw
    if (vtype) {
      // Q is a robot vertex (fixed); A = A~_j and V = v_j move with the pose
      const float gvx = -t * rx - rv * wx, gvy = -t * ry - rv * wy;
      sx = -gwx; sy = -gwy;
      gth = (-gwx) * say - (-gwy) * sax + gvx * svy - gvy * svx;
    } else {
      // Q is an obstacle point; the robot edge is fixed
      sx = gwx; sy = gwy;
      gth = gwx * qy - gwy * qx;
    }
  } else {
    // sd = -depth, depth = mu - log(sum exp(-eta (delta+ - mu))) / eta; the
    // weight of axis q is its softmax weight (hard minimum: 1 at the first
    // minimum); d delta+ / d delta = 1 for delta > 0, else 0.
    const float dp = lane < K ? fmaxf(dl, 0.0f) : __builtin_huge_valf();
    const float mu = wave_min_f32(dp);
    float w;
    if (F.hard) {
      const uint64_t k = lane < K ? (((uint64_t)__float_as_uint(dp) << 32) | (uint32_t)lane) : ~0ull;
      w = (int)(wave_min_u64(k) & 0xffffffffu) == lane ? 1.f : 0.f;
    } else {
      const float acc = wave_sum(lane < K ? expf(-F.eta * (dp - mu)) : 0.f);
      w = expf(-F.eta * (dl - mu)) / acc;
    }
    if (lane < K && dl > 0.f && w != 0.f) {
      const float gd = -w;   // d sd / d delta_q
      float gpx, gpy, ptx, pty;
      const bool upper = br == 0;   // delta = beta_i - alpha_P, else beta_P - alpha_i
      if (upper) { gpx = gd * nxq; gpy = gd * nyq; ptx = hix; pty = hiy; }
      else { gpx = -gd * nxq; gpy = -gd * nyq; ptx = lox; pty = loy; }
      sx = gpx; sy = gpy;
      gth = gpx * pty - gpy * ptx;
      if (lane >= m) {
        const int j = lane - m;
        // d delta / d n' = (P_hi - V_lo) or (V_hi - P_lo); n' = (-v_y, v_x) il
        const float gnx = upper ? gd * (hix - rlx) : gd * (rhx - lox);
        const float gny = upper ? gd * (hiy - rly) : gd * (rhy - loy);
        const float gvx = gny * W.il[j], gvy = -gnx * W.il[j];
        gth += gvx * W.vy[j] - gvy * W.vx[j];
      }
    }
    sx = wave_sum(sx); sy = wave_sum(sy); gth = wave_sum(gth);
  }
  g[0] = -(c * sx - s * sy);
  g[1] = -(s * sx + c * sy);
  g[2] = gth;
}

}  // namespace psdf
