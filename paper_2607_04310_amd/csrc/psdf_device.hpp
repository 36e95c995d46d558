// Device-side PSDF arithmetic for gfx950 (wave64, FP32 VALU).
//
// One lane evaluates one obstacle against one stage pose at a time: the
// obstacle's world-frame edges and their stage-invariant constants live in
// registers and are reused for every stage the lane visits; the footprint
// constants are wave-uniform, and the footprint rotated by each stage's
// heading is shared by the work-group in LDS.  Everything is written with
// explicit fmaf and compiled with -ffp-contract=off, so every kernel that
// inlines these functions produces bit-identical results for the same inputs.
//
// Pipeline per (stage, obstacle), Sec. IV-A items 1-4, evaluated in the frame
// of the stage pose translated to the origin but not rotated: the obstacle
// is translated (A_j - p) and the footprint rotated (R v_l, R u_l), which
// gives the same distances and axis overlaps as the paper's local frame
// R^T (A - p) (a rigid motion of both sets):
//   2. every point-segment distance in the segment's own frame: with the
//      unit direction u and normal n of the segment, a = (P - A) . u and
//      b = (P - A) . n, d^2 = b^2 + (a - clamp(a, 0, |B - A|))^2, which is
//      |P - A - t (B - A)|^2 with t = clamp(u, 0, 1) of Sec. IV-B (eps -> 0);
//      d_v over (robot vertex, obstacle edge), d_e over (V_obs point, robot
//      edge)
//   3. SAT over {n_l} U {n'_j = rot90(B_j - A_j) / (|B_j - A_j| + eps)}: the
//      across coordinates b above are the axis projections less a constant,
//      so the intervals come from the same numbers; an obstacle's interval on
//      its own axes does not depend on the pose and is taken once per
//      obstacle; delta(n) = min(beta_i - alpha_P, beta_P - alpha_i),
//      separated if any delta < -eps_sat; soft-min depth
//      -(1/eta) log sum exp(-eta max(delta, 0)) in max-shifted form
//   4. sd = sqrt(min(d_v^2, d_e^2)) if separated else -depth
// The squared norms |v_j|^2 + eps and |v_j| + eps are rotation invariant and
// are taken once per obstacle from the world-frame edge.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace psdf {

constexpr int kMaxFp = 16;    // footprint vertices
constexpr int kMaxObst = 16;  // edges per obstacle
constexpr uint64_t kEmptyKey = ~0ull;

// Footprint constants in the robot-local frame (counter-clockwise), prepared
// once on the host in double precision and rounded to float.  Slots l >= m
// repeat vertex / edge / axis m - 1, which leaves every min / max / any
// reduction unchanged; only the soft-min sum masks them.
struct FpConst {
  int m;
  int hard;        // 1: hard minimum (eta <= 0 or +inf)
  int reversed;    // 1: the caller's vertex order was clockwise (slot l = caller m - 1 - l)
  float eps, eps_sat, eta;
  float vx[kMaxFp], vy[kMaxFp];  // vertices v_l
  float ex[kMaxFp], ey[kMaxFp];  // robot edge E_l = [v_l, v_{l+1}] as v_{l+1} - v_l
  float einv[kMaxFp];            // 1 / (|e_l|^2 + eps)
  float nx[kMaxFp], ny[kMaxFp];  // outward unit normals n_l
  float pa[kMaxFp], pb[kMaxFp];  // robot interval [alpha_P(n_l), beta_P(n_l)]
  // robot edge frames for the pools: unit direction u_l = e_l / |e_l|,
  // length |e_l|, and the offsets v_l . u_l, v_l . n_l
  float ux[kMaxFp], uy[kMaxFp], len[kMaxFp], cu[kMaxFp], cn[kMaxFp];
  // robot interval on its own axis less the offset: alpha_P - v_l . n_l and
  // beta_P - v_l . n_l
  float oa[kMaxFp], ob[kMaxFp];
  // Screening certificate constants: rmax bounds |v_l| (every footprint
  // point is within rmax of the pose origin); tau_sep is the distance above
  // which two convex sets are declared separated by the axis test whatever
  // the rounding (eps_sat / kappa + margin, kappa = cos of half the largest
  // exterior angle of the footprint).
  float rmax, tau_sep;
};

// One obstacle in registers, with its pose-independent constants.  Slots
// j >= mi repeat edge mi - 1, which leaves every min / max / any-reduction
// unchanged; only the soft-min sum masks them.
template <int MI>
struct Obst {
  float ax[MI], ay[MI];   // A_j, world
  float bx[MI], by[MI];   // B_j, world (extra V_obs points of an open obstacle)
  float ux[MI], uy[MI];   // (B_j - A_j) / (|B_j - A_j| + eps); n'_j = (-uy, ux)
  float len[MI];          // |B_j - A_j|
  float olo[MI], ohi[MI]; // interval of (W - A_j) . n'_j over W in V_obs (when own)
  int mi;
  bool own;               // olo / ohi computed (on first need, own_intervals)
  bool closed;            // B_j == A_{j+1} for all j (bitwise): V_obs = {A_j}
  bool bad;               // edge count or range invalid, or a non-finite
                          // coordinate: the result is NaN
};

__device__ __forceinline__ float clamp01(float u) { return __builtin_amdgcn_fmed3f(u, 0.0f, 1.0f); }

// Orderable 32-bit image of a float: unsigned order == float order; every NaN
// maps to 0, below all numbers, so that a NaN result wins the minimum.
__device__ __forceinline__ uint32_t orderable(float f) {
  uint32_t u = __float_as_uint(f);
  if (f != f) return 0u;
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float from_orderable(uint32_t k) {
  uint32_t u = (k & 0x80000000u) ? (k & 0x7fffffffu) : ~k;
  return __uint_as_float(u);
}

// Rotation-invariant constants of an edge with world vector (dx, dy):
// iv2 = 1 / (|v|^2 + eps) and il = 1 / (|v| + eps) (hardware reciprocal and
// square root, about 1 ulp).  Every kernel derives them through this
// function, so they agree bit for bit.
__device__ __forceinline__ void edge_consts(float dx, float dy, float eps, float& iv2, float& il) {
  const float l2 = fmaf(dx, dx, dy * dy);
  iv2 = __builtin_amdgcn_rcpf(l2 + eps);
  il = __builtin_amdgcn_rcpf(__builtin_amdgcn_sqrtf(l2) + eps);
}

// Local frame of a world point / vector: R(theta)^T (P - p) and R^T w.
__device__ __forceinline__ void local_point(float x, float y, float c, float s, float px, float py,
                                            float& lx, float& ly) {
  const float dx = x - px, dy = y - py;
  lx = fmaf(c, dx, s * dy);
  ly = fmaf(c, dy, -(s * dx));
}
__device__ __forceinline__ void local_vector(float wx, float wy, float c, float s, float& lx,
                                             float& ly) {
  lx = fmaf(c, wx, s * wy);
  ly = fmaf(c, wy, -(s * wx));
}

template <int MI>
__device__ __forceinline__ void load_obstacle(Obst<MI>& o, const float* __restrict__ ax,
                                              const float* __restrict__ ay,
                                              const float* __restrict__ bx,
                                              const float* __restrict__ by, int e0, int mi, int E,
                                              float eps) {
  o.mi = mi;
  o.bad = (mi < 0) || (mi > MI) || (e0 < 0) || (e0 > E - mi);
  const int n = o.bad ? 1 : (mi < 1 ? 1 : mi);
  const int base = o.bad ? 0 : e0;
  const bool any = !o.bad && mi > 0;
  // a four-edge obstacle whose edges start at 16-byte aligned addresses
  // (rectangles in a CSR set of rectangles) takes one vector load per array;
  // the values are the same either way
  const uintptr_t al = reinterpret_cast<uintptr_t>(ax + base) | reinterpret_cast<uintptr_t>(ay + base) |
                       reinterpret_cast<uintptr_t>(bx + base) | reinterpret_cast<uintptr_t>(by + base);
  const bool vec = MI >= 4 && any && n == 4 && (al & 15u) == 0;
  float4 v0 = make_float4(0.f, 0.f, 0.f, 0.f), v1 = v0, v2 = v0, v3 = v0;
  if (vec) {
    v0 = *reinterpret_cast<const float4*>(ax + base);
    v1 = *reinterpret_cast<const float4*>(ay + base);
    v2 = *reinterpret_cast<const float4*>(bx + base);
    v3 = *reinterpret_cast<const float4*>(by + base);
  }
  const float x0[4] = {v0.x, v0.y, v0.z, v0.w}, y0[4] = {v1.x, v1.y, v1.z, v1.w};
  const float x1[4] = {v2.x, v2.y, v2.z, v2.w}, y1[4] = {v3.x, v3.y, v3.z, v3.w};
#pragma unroll
  for (int j = 0; j < MI; ++j) {
    const int jj = j < n ? j : n - 1;
    float a0 = 0.f, a1 = 0.f, b0 = 0.f, b1 = 0.f;
    if (vec) {
      const int q = j < 4 ? j : 3;
      a0 = x0[q]; a1 = y0[q];
      b0 = x1[q]; b1 = y1[q];
    } else if (any) {
      a0 = ax[base + jj]; a1 = ay[base + jj];
      b0 = bx[base + jj]; b1 = by[base + jj];
    }
    o.ax[j] = a0; o.ay[j] = a1;
    o.bx[j] = b0; o.by[j] = b1;
    const float dx = b0 - a0, dy = b1 - a1;
    float iv2, il;
    edge_consts(dx, dy, eps, iv2, il);
    o.ux[j] = dx * il;
    o.uy[j] = dy * il;
    o.len[j] = __builtin_amdgcn_sqrtf(fmaf(dx, dx, dy * dy));
  }
  bool finite = true;
#pragma unroll
  for (int j = 0; j < MI; ++j)
    finite = finite && isfinite(o.ax[j]) && isfinite(o.ay[j]) && isfinite(o.bx[j]) && isfinite(o.by[j]);
  o.bad = o.bad || !finite;
  bool closed = mi >= 3;
#pragma unroll
  for (int j = 0; j < MI; ++j) {
    const float nx = (j + 1 < mi) ? o.ax[(j + 1) % MI] : o.ax[0];
    const float ny = (j + 1 < mi) ? o.ay[(j + 1) % MI] : o.ay[0];
    if (j < mi) closed = closed && (__float_as_uint(o.bx[j]) == __float_as_uint(nx)) &&
                         (__float_as_uint(o.by[j]) == __float_as_uint(ny));
  }
  o.closed = closed;
  o.own = false;
}

// Own-axis intervals (Sec. IV-C), relative to A_j: pose independent, needed
// only at stages that no robot axis separates, so taken on first need.  With
// LAZY the obstacle's coordinates pass through empty asm statements first (no
// instruction, the same values), which keeps the compiler from computing the
// intervals ahead of that need, so a wave whose lanes are all separated by a
// robot axis skips them (the plain path at one stage per wave, where each
// wave meets its obstacles once).  Without it the compiler takes them once,
// ahead of the stage loop (the batch kernel's many-stage items, where that
// is cheaper).
template <int MI, bool LAZY = false>
__device__ __forceinline__ void own_intervals(Obst<MI>& o) {
  float ax[MI], ay[MI], ux[MI], uy[MI];
#pragma unroll
  for (int k = 0; k < MI; ++k) {
    ax[k] = o.ax[k]; ay[k] = o.ay[k]; ux[k] = o.ux[k]; uy[k] = o.uy[k];
    if (LAZY) asm volatile("" : "+v"(ax[k]), "+v"(ay[k]), "+v"(ux[k]), "+v"(uy[k]));
  }
#pragma unroll
  for (int j = 0; j < MI; ++j) {
    float lo = __builtin_huge_valf(), hi = -__builtin_huge_valf();
#pragma unroll
    for (int k = 0; k < MI; ++k) {
      const float q = fmaf(ay[k] - ay[j], ux[j], -((ax[k] - ax[j]) * uy[j]));
      lo = fminf(lo, q);
      hi = fmaxf(hi, q);
    }
    if (!o.closed) {
#pragma unroll
      for (int k = 0; k < MI; ++k) {
        const float q = fmaf(o.by[k] - ay[j], ux[j], -((o.bx[k] - ax[j]) * uy[j]));
        lo = fminf(lo, q);
        hi = fmaxf(hi, q);
      }
    }
    o.olo[j] = lo;
    o.ohi[j] = hi;
  }
  o.own = true;
}

// The footprint rotated by a stage heading (c, s) = (cos, sin): slot l of rf
// holds (R v_l, R u_l), u_l the unit direction of robot edge l.
__device__ __forceinline__ float4 rotated_slot(const FpConst& F, int l, float c, float s) {
  const float vx = F.vx[l], vy = F.vy[l], ux = F.ux[l], uy = F.uy[l];
  return make_float4(fmaf(c, vx, -(s * vy)), fmaf(s, vx, c * vy), fmaf(c, ux, -(s * uy)),
                     fmaf(s, ux, c * uy));
}

// Squared distance from point (px, py) to the segment [a, a + v], with
// iv2 = 1 / (|v|^2 + eps).  Also returns u for the adjoint.
__device__ __forceinline__ float seg_d2(float px, float py, float ax, float ay, float vx, float vy,
                                        float iv2) {
  const float wx = px - ax, wy = py - ay;
  const float u = fmaf(wx, vx, wy * vy) * iv2;
  const float t = clamp01(u);
  const float rx = fmaf(-t, vx, wx), ry = fmaf(-t, vy, wy);
  return fmaf(rx, rx, ry * ry);
}

// Distance term of a point against a segment, in the segment's frame: with
// a = (P - A) . u (along the unit direction u) and b = (P - A) . n (across),
// the squared point-segment distance is b^2 + (a - clamp(a, 0, L))^2, which
// is |P - A - t v|^2 with t = clamp(u, 0, 1) of Sec. IV-B (eps -> 0).  The
// across component b is the separating-axis projection that the pipeline
// needs anyway, less a per-segment constant.
__device__ __forceinline__ float frame_d2(float a, float b, float L) {
  const float c = a - __builtin_amdgcn_fmed3f(a, 0.0f, L);
  return fmaf(b, b, c * c);
}

// sd(P0(x), P^i) of one obstacle at one stage (Sec. IV-D).  MF is the number
// of footprint slots evaluated: the exact m (3..8) or 16 (padded); rf holds
// the footprint rotated by the stage heading (rotated_slot, MF slots) and
// (px, py) is the stage position.
template <int MF, int MI, bool LAZY = false>
__device__ __forceinline__ float obstacle_sd(const FpConst& F, Obst<MI>& o,
                                             const float4* rf, float px, float py) {
  // the obstacle translated to the pose origin, and its edge frames' offsets
  // ca = (A_j - p) . u_j, cb = (A_j - p) . n'_j
  float tax[MI], tay[MI], ca[MI], cb[MI];
#pragma unroll
  for (int j = 0; j < MI; ++j) {
    tax[j] = o.ax[j] - px;
    tay[j] = o.ay[j] - py;
    ca[j] = fmaf(tax[j], o.ux[j], tay[j] * o.uy[j]);
    cb[j] = fmaf(tay[j], o.ux[j], -(tax[j] * o.uy[j]));
  }

  // Robot vertices against obstacle edges (d_v, Sec. IV-B); the across
  // coordinate b is the robot's projection on n'_j less cb_j (Sec. IV-C).
  float dv2 = __builtin_huge_valf(), de2 = __builtin_huge_valf();
  float rlo[MI], rhi[MI];
#pragma unroll
  for (int j = 0; j < MI; ++j) { rlo[j] = __builtin_huge_valf(); rhi[j] = -__builtin_huge_valf(); }
#pragma unroll
  for (int l = 0; l < MF; ++l) {
    const float4 r = rf[l];
#pragma unroll
    for (int j = 0; j < MI; ++j) {
      const float a = fmaf(r.x, o.ux[j], fmaf(r.y, o.uy[j], -ca[j]));
      const float b = fmaf(r.y, o.ux[j], fmaf(-r.x, o.uy[j], -cb[j]));
      rlo[j] = fminf(rlo[j], b);
      rhi[j] = fmaxf(rhi[j], b);
      dv2 = fminf(dv2, frame_d2(a, b, o.len[j]));
    }
  }
  // Obstacle points against robot edges (d_e): in robot edge l's frame
  // (U = R u_l, N = R n_l = (U_y, -U_x)), b is the obstacle's projection on
  // the robot axis less v_l . n_l.
  float ra_lo[MF], ra_hi[MF];
#pragma unroll
  for (int l = 0; l < MF; ++l) { ra_lo[l] = __builtin_huge_valf(); ra_hi[l] = -__builtin_huge_valf(); }
  auto visit = [&](float wx, float wy) {
#pragma unroll
    for (int l = 0; l < MF; ++l) {
      const float4 r = rf[l];
      const float a = fmaf(wx, r.z, fmaf(wy, r.w, -F.cu[l]));
      const float b = fmaf(wx, r.w, fmaf(-wy, r.z, -F.cn[l]));
      ra_lo[l] = fminf(ra_lo[l], b);
      ra_hi[l] = fmaxf(ra_hi[l], b);
      de2 = fminf(de2, frame_d2(a, b, F.len[l]));
    }
  };
#pragma unroll
  for (int k = 0; k < MI; ++k) visit(tax[k], tay[k]);
  if (!o.closed) {
#pragma unroll
    for (int k = 0; k < MI; ++k) visit(o.bx[k] - px, o.by[k] - py);
  }

  // Overlaps and the separating-axis test: the robot axes, then, where none
  // of them separates, the obstacle's axes (sep is their disjunction either
  // way, and the overlaps are only used when no axis separates).
  float dl[MF + MI];
  bool sep = false;
#pragma unroll
  for (int l = 0; l < MF; ++l) {
    dl[l] = fminf(ra_hi[l] - F.oa[l], F.ob[l] - ra_lo[l]);
    sep = sep || (dl[l] < -F.eps_sat);
  }
  if (!sep) {
    if (!o.own) own_intervals<MI, LAZY>(o);
#pragma unroll
    for (int j = 0; j < MI; ++j) {
      dl[MF + j] = fminf(o.ohi[j] - rlo[j], rhi[j] - o.olo[j]);
      sep = sep || (dl[MF + j] < -F.eps_sat);
    }
  }

  float sd = sqrtf(fminf(dv2, de2));
  if (!sep) {
    // Soft-min depth over the |N^i| = m + mi axes (padded slots excluded).
    float mu = __builtin_huge_valf();
#pragma unroll
    for (int q = 0; q < MF + MI; ++q) mu = fminf(mu, fmaxf(dl[q], 0.0f));
    float depth = mu;
    if (!F.hard) {
      float acc = 0.0f;
#pragma unroll
      for (int q = 0; q < MF + MI; ++q) {
        const bool live = q < MF ? (q < F.m) : (q - MF < o.mi);
        if (live) acc += expf(-F.eta * (fmaxf(dl[q], 0.0f) - mu));
      }
      depth = mu - logf(acc) / F.eta;
    }
    sd = -depth;
  }
  if (o.bad) sd = __builtin_nanf("");
  return sd;
}

}  // namespace psdf
