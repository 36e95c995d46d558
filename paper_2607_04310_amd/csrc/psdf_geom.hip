// Geometry adjoint: the vector-Jacobian product of phi with respect to the
// obstacle edge endpoints and the footprint vertices, through each stage's
// winning obstacle with the active-branch subgradient of Sec. IV-D (the pose
// adjoint's rule applied to every input of the pipeline, Sec. IV-A..IV-D).
//
// One wave per stage.  The winner's local geometry is rebuilt with the same
// device arithmetic and the same selections (active pool pair, axis
// extremes, separated branch, soft-min weights) as the pose adjoint in
// psdf_winner.hpp.  The reverse pass then forms, per lane, up to four
// (point, adjoint) contributions:
//   * separated: the active point-segment pair d = |w - t V|, w = Q - A,
//     V = B - A, t = clamp(u), u = (w . V) / (|V|^2 + eps): adjoints of Q, A
//     and B, including the u-dependence of t inside (0, 1);
//   * penetration, per axis with weight w_q and delta_q > 0 (d sd / d delta_q
//     = -w_q): the two extreme points of delta_q = beta - alpha, and the
//     axis normal's dependence on its edge: a robot normal
//     n = rot(-90)(e) / |e| on the footprint vertices of e, an obstacle
//     normal n' = rot90(u) / (|u| + eps) on the obstacle edge endpoints.
// The contributions are summed per point in a fixed lane / slot order in LDS,
// rotated back to the world frame for the obstacle endpoints
// (d phi / dA = R d phi / dA~), scaled by gout[s] and added to the outputs.
// The footprint gradient is reported in the caller's vertex order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "psdf.h"
#include "psdf_host.hpp"
#include "psdf_winner.hpp"

namespace psdf {
namespace {

constexpr int kGeoWaves = 4;      // stages per work-group
constexpr int kSlots = 4;         // contributions per lane
constexpr int kRobot = 64;        // target ids: 2 j (A_j), 2 j + 1 (B_j), kRobot + l (v_l)

struct GeoLds {
  float tax[kMaxObst], tay[kMaxObst];    // A~_j
  float vx[kMaxObst], vy[kMaxObst];      // v~_j = R^T (B_j - A_j)
  float nx[kMaxObst], ny[kMaxObst];      // n'_j
  float iv2[kMaxObst], il[kMaxObst];     // 1 / (|v|^2 + eps), 1 / (|v| + eps)
  float len[kMaxObst];                   // |v|
  float px[2 * kMaxObst], py[2 * kMaxObst];   // V_obs
  alignas(16) int tgt[64][kSlots];
  alignas(16) float gx[64][kSlots];
  alignas(16) float gy[64][kSlots];
};

// Target id of V_obs point k: A~_k, or B~_{k - mi} for open obstacles.
__device__ __forceinline__ int point_target(int k, int mi) {
  return k < mi ? 2 * k : 2 * (k - mi) + 1;
}

// Clears a[0..n) and b[0..nb) (the two outputs) in one launch.
__global__ void zero2_kernel(float* __restrict__ a, int n, float* __restrict__ b, int nb) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = 0.0f;
  if (i < nb) b[i] = 0.0f;
}

__global__ __launch_bounds__(64 * kGeoWaves) void geom_bwd_kernel(
    FpConst F, const float* __restrict__ poses, int N, const float* __restrict__ ax,
    const float* __restrict__ ay, const float* __restrict__ bx, const float* __restrict__ by,
    const int* __restrict__ off, int E, int M, const uint64_t* __restrict__ keys,
    const float* __restrict__ gout, float* __restrict__ gedges, float* __restrict__ gfp) {
  __shared__ FpLds fls[kGeoWaves];
  __shared__ GeoLds gls[kGeoWaves];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int s = blockIdx.x * kGeoWaves + w;
  if (s >= N) return;
  FpLds& FL = fls[w];
  GeoLds& G = gls[w];
  const float* p = poses + 3 * s;
  const float px = p[0], py = p[1], th = p[2];
  const uint64_t key = keys[s];
  const float scale = gout[s];
  stage_footprint(FL, F);
  float sn, cs;
  sincosf(th, &sn, &cs);
  const int m = F.m;
  if (key == kEmptyKey) return;   // no obstacle: no contribution
  const int i = (int)(key & 0xffffffffu);
  bool valid = (key >> 32) != 0 && (uint64_t)i < (uint64_t)M;
  int e0 = 0, mi = 0;
  if (valid) {
    e0 = off[i];
    mi = off[i + 1] - e0;
  }
  valid = valid && mi >= 1 && mi <= kMaxObst && e0 >= 0 && e0 <= E - mi;
  if (!valid) {
    // NaN winner (non-finite pose or invalid obstacle): NaN reaches every
    // footprint vertex, which takes part in every stage
    if (lane < 2 * m) atomicAdd(&gfp[lane], __builtin_nanf(""));
    return;
  }

  // ---- the winner's local geometry (as in winner_adjoint)
  bool open_edge = false;
  if (lane < mi) {
    const float a0 = ax[e0 + lane], a1 = ay[e0 + lane];
    const float b0 = bx[e0 + lane], b1 = by[e0 + lane];
    const int nxt = lane + 1 < mi ? lane + 1 : 0;
    const float n0 = ax[e0 + nxt], n1 = ay[e0 + nxt];
    open_edge = __float_as_uint(b0) != __float_as_uint(n0) || __float_as_uint(b1) != __float_as_uint(n1);
    float iv2, il, tx, ty, vx, vy;
    edge_consts(b0 - a0, b1 - a1, F.eps, iv2, il);
    local_point(a0, a1, cs, sn, px, py, tx, ty);
    local_vector(b0 - a0, b1 - a1, cs, sn, vx, vy);
    G.tax[lane] = tx; G.tay[lane] = ty; G.vx[lane] = vx; G.vy[lane] = vy;
    G.nx[lane] = -vy * il; G.ny[lane] = vx * il;
    G.iv2[lane] = iv2; G.il[lane] = il;
    G.len[lane] = __builtin_amdgcn_sqrtf(fmaf(b0 - a0, b0 - a0, (b1 - a1) * (b1 - a1)));
    G.px[lane] = tx; G.py[lane] = ty;
    G.px[mi + lane] = tx + vx; G.py[mi + lane] = ty + vy;
  }
  const bool closed = mi >= 3 && __ballot(open_edge) == 0;
  const int nv = closed ? mi : 2 * mi;
#pragma unroll
  for (int q = 0; q < kSlots; ++q) G.tgt[lane][q] = -1;
  wave_sync();

  // ---- active pool pair: smallest (d^2, entry), entries as in winner_adjoint
  const int PV = m * mi, P = PV + nv * m;
  uint64_t best = ~0ull;
  for (int e = lane; e < P; e += 64) {
    float qx, qy, sax, say, svx, svy, siv;
    if (e < PV) {
      const int l = e / mi, j = e - l * mi;
      qx = FL.vx[l]; qy = FL.vy[l];
      sax = G.tax[j]; say = G.tay[j]; svx = G.vx[j]; svy = G.vy[j]; siv = G.iv2[j];
    } else {
      const int e2 = e - PV, k = e2 / m, l = e2 - k * m;
      qx = G.px[k]; qy = G.py[k];
      sax = FL.vx[l]; say = FL.vy[l]; svx = FL.ex[l]; svy = FL.ey[l]; siv = FL.einv[l];
    }
    const float d2 = seg_d2(qx, qy, sax, say, svx, svy, siv);
    const uint64_t k2 = ((uint64_t)__float_as_uint(d2) << 32) | (uint32_t)e;
    best = k2 < best ? k2 : best;
  }
  best = wave_min_u64(best);

  // ---- axes: lane q < m + mi owns axis q; extremes by index (first on ties)
  const int K = m + mi;
  float dl = __builtin_huge_valf(), nxq = 0.f, nyq = 0.f;
  int klo = 0, khi = 0, rlo = 0, rhi = 0, br = 0;
  if (lane < K) {
    float alo, ahi;
    if (lane < m) {
      nxq = FL.nx[lane]; nyq = FL.ny[lane];
      alo = FL.pa[lane]; ahi = FL.pb[lane];
    } else {
      const int j = lane - m;
      nxq = G.nx[j]; nyq = G.ny[j];
      alo = __builtin_huge_valf(); ahi = -__builtin_huge_valf();
    }
    float plo = __builtin_huge_valf(), phi = -__builtin_huge_valf();
    for (int l = 0; l < m; ++l) {
      const float q = fmaf(FL.vx[l], nxq, FL.vy[l] * nyq);
      if (q < plo) { plo = q; rlo = l; }
      if (q > phi) { phi = q; rhi = l; }
    }
    if (lane >= m) { alo = plo; ahi = phi; }
    float lo = __builtin_huge_valf(), hi = -__builtin_huge_valf();
    for (int k = 0; k < nv; ++k) {
      const float q = fmaf(G.px[k], nxq, G.py[k] * nyq);
      if (q < lo) { lo = q; klo = k; }
      if (q > hi) { hi = q; khi = k; }
    }
    const float d1 = hi - alo, d2 = ahi - lo;
    dl = fminf(d1, d2);
    br = d1 <= d2 ? 0 : 1;
  }
  const bool sep = __ballot(lane < K && dl < -F.eps_sat) != 0;

  // ---- reverse pass: contributions (target, local adjoint)
  int nslot = 0;
  auto put = [&](int t, float gx, float gy) {
    G.tgt[lane][nslot] = t;
    G.gx[lane][nslot] = gx;
    G.gy[lane][nslot] = gy;
    ++nslot;
  };
  if (sep) {
    if (lane == 0) {
      const int e = (int)(best & 0xffffffffu);
      const float d2b = __uint_as_float((uint32_t)(best >> 32));
      float qx, qy, sax, say, svx, svy, siv;
      int tq, ta, tb;
      if (e < PV) {
        const int l = e / mi, j = e - l * mi;
        qx = FL.vx[l]; qy = FL.vy[l];
        sax = G.tax[j]; say = G.tay[j]; svx = G.vx[j]; svy = G.vy[j]; siv = G.iv2[j];
        tq = kRobot + l; ta = 2 * j; tb = 2 * j + 1;
      } else {
        const int e2 = e - PV, k = e2 / m, l = e2 - k * m;
        qx = G.px[k]; qy = G.py[k];
        sax = FL.vx[l]; say = FL.vy[l]; svx = FL.ex[l]; svy = FL.ey[l]; siv = FL.einv[l];
        tq = point_target(k, mi); ta = kRobot + l; tb = kRobot + (l + 1 < m ? l + 1 : 0);
      }
      const float d = sqrtf(d2b);
      if (d > 0.f) {
        const float wx = qx - sax, wy = qy - say;
        const float u = fmaf(wx, svx, wy * svy) * siv;
        const float t = clamp01(u);
        const float rx = fmaf(-t, svx, wx), ry = fmaf(-t, svy, wy);
        const float grx = rx / d, gry = ry / d;
        float gwx = grx, gwy = gry;
        float gvx = -t * grx, gvy = -t * gry;
        if (u > 0.f && u < 1.f) {
          const float gu = -fmaf(grx, svx, gry * svy);
          gwx = fmaf(gu * siv, svx, gwx);
          gwy = fmaf(gu * siv, svy, gwy);
          gvx += gu * siv * (wx - 2.f * u * svx);
          gvy += gu * siv * (wy - 2.f * u * svy);
        }
        put(tq, gwx, gwy);
        put(ta, -gwx - gvx, -gwy - gvy);
        put(tb, gvx, gvy);
      }
    }
  } else {
    // soft-min weights of the axis overlaps (hard minimum: the first one)
    const float dp = lane < K ? fmaxf(dl, 0.0f) : __builtin_huge_valf();
    const float mu = wave_min_f32(dp);
    float wq;
    if (F.hard) {
      const uint64_t k = lane < K ? (((uint64_t)__float_as_uint(dp) << 32) | (uint32_t)lane) : ~0ull;
      wq = (int)(wave_min_u64(k) & 0xffffffffu) == lane ? 1.f : 0.f;
    } else {
      const float acc = wave_sum(lane < K ? expf(-F.eta * (dp - mu)) : 0.f);
      wq = expf(-F.eta * (dl - mu)) / acc;
    }
    if (lane < K && dl > 0.f && wq != 0.f) {
      const float gd = -wq;   // d sd / d delta_q
      float gnx, gny;         // adjoint of the axis normal
      if (br == 0) {
        // delta = beta_i - alpha_P: obstacle point khi, robot vertex rlo
        put(point_target(khi, mi), gd * nxq, gd * nyq);
        put(kRobot + rlo, -gd * nxq, -gd * nyq);
        gnx = gd * (G.px[khi] - FL.vx[rlo]);
        gny = gd * (G.py[khi] - FL.vy[rlo]);
      } else {
        // delta = beta_P - alpha_i: robot vertex rhi, obstacle point klo
        put(kRobot + rhi, gd * nxq, gd * nyq);
        put(point_target(klo, mi), -gd * nxq, -gd * nyq);
        gnx = gd * (FL.vx[rhi] - G.px[klo]);
        gny = gd * (FL.vy[rhi] - G.py[klo]);
      }
      if (lane < m) {
        // n = rot(-90)(e) / |e|, e = v_{l+1} - v_l:
        // d/de = (rot90(gn) - e^ (n . gn)) / |e|
        const int l = lane, l1 = l + 1 < m ? l + 1 : 0;
        const float ex = FL.ex[l], ey = FL.ey[l];
        const float L = sqrtf(fmaf(ex, ex, ey * ey));
        const float ng = fmaf(nxq, gnx, nyq * gny);
        const float gex = (-gny - ex / L * ng) / L, gey = (gnx - ey / L * ng) / L;
        put(kRobot + l1, gex, gey);
        put(kRobot + l, -gex, -gey);
      } else {
        // n' = rot90(u) k, k = 1 / (|u| + eps), u = B~_j - A~_j:
        // d/du = k rot90^T(gn) - k^2 (gn . rot90(u)) u / |u|
        const int j = lane - m;
        const float ux = G.vx[j], uy = G.vy[j], k = G.il[j], L = G.len[j];
        const float gr = fmaf(gnx, -uy, gny * ux);   // gn . rot90(u)
        const float c2 = L > 0.f ? k * k * gr / L : 0.f;
        const float gux = k * gny - c2 * ux, guy = -k * gnx - c2 * uy;
        put(2 * j + 1, gux, guy);
        put(2 * j, -gux, -guy);
      }
    }
  }
  wave_sync();

  // ---- per-point sums in lane / slot order, then the outputs
  int t = -1;
  if (lane < 2 * mi) t = lane;
  else if (lane >= 32 && lane < 32 + m) t = kRobot + (lane - 32);
  if (t < 0) return;
  // every lane's four slots as one vector read each, the adds selected (a
  // slot of another point adds +0), so the reads of many lanes are in
  // flight at once instead of one read and branch per slot
  static_assert(kSlots == 4, "the sums read a lane's slots as one vector");
  float sx = 0.f, sy = 0.f;
#pragma unroll 8
  for (int l = 0; l < 64; ++l) {
    const int4 tg = *reinterpret_cast<const int4*>(G.tgt[l]);
    const float4 ux = *reinterpret_cast<const float4*>(G.gx[l]);
    const float4 uy = *reinterpret_cast<const float4*>(G.gy[l]);
    sx += tg.x == t ? ux.x : 0.f; sy += tg.x == t ? uy.x : 0.f;
    sx += tg.y == t ? ux.y : 0.f; sy += tg.y == t ? uy.y : 0.f;
    sx += tg.z == t ? ux.z : 0.f; sy += tg.z == t ? uy.z : 0.f;
    sx += tg.w == t ? ux.w : 0.f; sy += tg.w == t ? uy.w : 0.f;
  }
  if (sx == 0.f && sy == 0.f && isfinite(scale)) return;
  if (t < kRobot) {
    // d phi / dA = R d phi / dA~
    const float wx = fmaf(cs, sx, -(sn * sy)), wy = fmaf(sn, sx, cs * sy);
    float* g = gedges + 4 * (size_t)(e0 + (t >> 1)) + 2 * (t & 1);
    atomicAdd(g, wx * scale);
    atomicAdd(g + 1, wy * scale);
  } else {
    const int l = t - kRobot;
    const int caller = F.reversed ? m - 1 - l : l;
    atomicAdd(&gfp[2 * caller], sx * scale);
    atomicAdd(&gfp[2 * caller + 1], sy * scale);
  }
}

}  // namespace
}  // namespace psdf

using namespace psdf;

extern "C" {

int psdf_bwd_geometry(const float* footprint, int32_t m, const float* poses, int32_t N,
                      const psdf_edges* edges, const psdf_params* params, const uint64_t* keys,
                      const float* gout, float* gedges, float* gfp, hipStream_t stream) {
  clear_error();
  FpConst F;
  int rc = prepare_footprint(footprint, m, params, &F);
  if (rc) return rc;
  psdf_edges e;
  rc = check_edges(edges, &e);
  if (rc) return rc;
  if (N < 0) return set_error(PSDF_EINVAL, "N = %d is negative", N);
  if (!gfp || (e.E > 0 && !gedges)) return set_error(PSDF_EINVAL, "gedges or gfp is NULL");
  if (N > 0 && (!poses || !keys || !gout))
    return set_error(PSDF_EINVAL, "poses, keys or gout is NULL");
  if ((size_t)e.E * 4 > (size_t)INT32_MAX) return set_error(PSDF_ETOOBIG, "E = %d", e.E);
  const int nz = std::max(4 * e.E, 2 * m);
  zero2_kernel<<<(nz + 255) / 256, 256, 0, stream>>>(gedges, 4 * e.E, gfp, 2 * m);
  hipError_t err = hipGetLastError();
  if (err == hipSuccess && N > 0) {
    geom_bwd_kernel<<<(N + kGeoWaves - 1) / kGeoWaves, 64 * kGeoWaves, 0, stream>>>(
        F, poses, N, e.ax, e.ay, e.bx, e.by, e.obst_off, e.E, e.M, keys, gout, gedges, gfp);
    err = hipGetLastError();
  }
  return hip_status(err);
}

}  // extern "C"
