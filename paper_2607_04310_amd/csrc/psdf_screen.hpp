// Certified screening of a batch: for each stage, a cheap conservative lower
// bound LB_i on sd_i for every obstacle, a pool of the P lowest-LB obstacles,
// a ranking of the pool's edges (the MLP score, or the edge's distance to the
// pose origin when no network is given), exact evaluation (obstacle_sd) of
// the obstacles owning the top-K edges, and a certificate: the candidates'
// minimum phi_K is the stage's PSDF value if every other obstacle has
//   LB_i > max(phi_K, tau_sep).
// Then sd_i >= LB_i > phi_K for every excluded obstacle, so the screened key
// (and winner, and gradient) equal the full evaluation's bit for bit.  A
// stage that fails the certificate is appended to a list that the fallback
// kernel evaluates in full.
//
// Lower bounds (world frame, pose origin p, footprint radius rmax about the
// origin; every footprint point is within rmax of p):
//  * every obstacle: its bounding circle (c_i, r_i), computed once per call
//    (obstacle_circle, in the horizon pass) or once per edge set
//    (psdf_batch_stage), gives
//    dist(P0(x), P^i) >= |p - c_i| - r_i - rmax;
//  * an instance's stages share a horizon bound (horizon_kernel) for the
//    obstacles left out of the instance's list;
//  * excluded pool members, only when the circle bounds do not certify: for
//    a closed convex polygon not containing p, dist(p, P^i) is the smallest
//    point-segment distance from p to its edges, so
//    dist(P0(x), P^i) >= dist(p, P^i) - rmax; a free segment (one edge) has
//    no interior, and an open chain of two or more edges gets -inf (the axis
//    test sees its convex hull, whose closing edge gives no axis).
// Both subtract gamma to absorb FP32 rounding; an invalid obstacle gets -inf.
// Two convex sets at distance r > tau_sep are separated by the axis test
// (the largest axis gap is at least kappa r), so their sd is d_sep >= r >= LB.
#pragma once

#include <hip/hip_runtime.h>

#include "psdf_batch.hpp"
#include "psdf_mlp.hpp"
#include "psdf_staged.hpp"

namespace psdf {

constexpr int kScreenThreads = 256;
constexpr int kScreenKeysPerThread = 64;                       // obstacles per thread and instance
constexpr int kScreenMaxM = kScreenThreads * kScreenKeysPerThread;   // 16384, the most screened
constexpr int kStageKeys = 8;                                  // horizon entries per thread (stage pass)
constexpr int kHorizonCap = kScreenThreads * kStageKeys;       // 2048
constexpr int kPoolCap = 512;                                  // pool capacity (ties included)
constexpr int kFeatSlots = 1024;                               // slots per feature chunk (MLP ranking)
constexpr float kLbGamma = 1e-3f;


struct ScreenArgs {
  const FpConst* fps;
  const BatchInst* insts;
  const int* stage_inst;   // global stage row -> instance
  const int4* stages;      // this launch's stages: (stage row, instance, the instance's
                           // circ_off, its obstacle count M), so that a stage's first
                           // loads wait on one record only
  int n_stages;
  const float* poses;
  const float* ax;
  const float* ay;
  const float* bx;
  const float* by;
  const int* off;
  const unsigned char* rows;  // staged obstacle rows (circ_off + local index), or nullptr
  const float4* hlist;     // per instance (at circ_off): the circles its stages screen, the
                           // obstacle's local index in .w (int bits)
  const int* hcount;       // per instance: length of hlist, or -1 for every obstacle
  const uint32_t* hrest;   // per instance: lower-bound key of every obstacle not in hlist
  const float* theta;      // MLP parameters, or nullptr: rank by edge distance
  const uint4* frag;       // the network's lane fragments (built by horizon_kernel), used with theta
  int pool;                // P
  int topk;                // K
  uint64_t* keys;
  int* failed;             // this launch's failed-stage list
  unsigned* ctrl;          // [0] failed count (zero on entry), [1] unused
  int* stage_cand;         // optional: candidates evaluated per stage
  int* stage_cert;         // optional: 1 if certified
  uint64_t* cand_keys;     // optional: the candidates' minimum key (before any fallback)
  // finish 1 (the bound form): the screen kernel writes a certified stage's
  // outputs itself, and the fallback's last tile of a failed stage writes
  // that stage's (no finish kernel); fdone counts a failed slot's tiles
  int finish;
  float* d;
  int* edge;
  int* obst;
  float* grad;
  int* fdone;              // this launch's, parallel to failed
  // reset_n > 0: the fallback's work-group 0 reopens the horizon lists
  // (count 0, bound +inf) after the call's last screen launch
  int reset_n;
  int* reset_hcount;
  uint32_t* reset_hrest;
};

// Obstacle o (local index) of instance `in` in registers: from its staged
// row when the screened call has rows, else from the offsets and the edges
// (load_obstacle; an out-of-range first edge marks it invalid).  mi gets
// its edge count (0 for an inactive lane).
template <int MI>
__device__ __forceinline__ void screen_obstacle(Obst<MI>& ob, const ScreenArgs& A,
                                                const BatchInst& in, int o, bool act, float eps,
                                                int& mi) {
  if (A.rows) {
    int a;
    row_obstacle<MI>(ob, A.rows, (size_t)in.circ_off + (act ? o : 0), act, a, mi);
    return;
  }
  int e0 = 0;
  mi = 0;
  if (act) {
    e0 = A.off[in.obst_off + o];
    mi = A.off[in.obst_off + o + 1] - e0;
    e0 += in.edge_off;
  }
  load_obstacle<MI>(ob, A.ax, A.ay, A.bx, A.by, e0, mi, in.edge_off + in.E, eps);
  if (act && e0 < in.edge_off) ob.bad = true;
}

__device__ __forceinline__ float obstacle_lb(float px, float py, const float* __restrict__ ax,
                                             const float* __restrict__ ay,
                                             const float* __restrict__ bx,
                                             const float* __restrict__ by, int e0, int mi, int Ebeg,
                                             int Eend, float eps, float rmax) {
  if (mi == 0) return __builtin_huge_valf();
  if (mi < 0 || mi > kMaxObst || e0 < Ebeg || e0 > Eend - mi) return -__builtin_huge_valf();
  float d2 = __builtin_huge_valf();
  bool pos = true, neg = true, closed = mi >= 3, finite = true;
  for (int j = 0; j < mi; ++j) {
    const float a0 = ax[e0 + j], a1 = ay[e0 + j], b0 = bx[e0 + j], b1 = by[e0 + j];
    const int nx = j + 1 < mi ? j + 1 : 0;
    closed = closed && __float_as_uint(b0) == __float_as_uint(ax[e0 + nx]) &&
             __float_as_uint(b1) == __float_as_uint(ay[e0 + nx]);
    finite = finite && isfinite(a0) && isfinite(a1) && isfinite(b0) && isfinite(b1);
    float iv2, il;
    edge_consts(b0 - a0, b1 - a1, eps, iv2, il);
    d2 = fminf(d2, seg_d2(px, py, a0, a1, b0 - a0, b1 - a1, iv2));
    const float cr = (b0 - a0) * (py - a1) - (b1 - a1) * (px - a0);
    pos = pos && cr >= 0.f;
    neg = neg && cr <= 0.f;
  }
  if (!finite || (closed && (pos || neg)) || (!closed && mi >= 2)) return -__builtin_huge_valf();
  return sqrtf(d2) - rmax - kLbGamma;
}

constexpr int kWaves = kScreenThreads / 64;

// ---- one four-edge-class obstacle per quad of lanes (staged rows)
//
// sd of the obstacle of staged row r, evaluated by the four lanes of a quad,
// lane j <-> edge slot j (the row's repeated slots included), equal bit for
// bit to obstacle_sd<MF, 4> on row_obstacle's registers: each lane takes
// edge j against every robot vertex and the obstacle point(s) of slot j
// against every robot edge with the same operations, the minima and maxima
// are then reduced across the quad (the order of a minimum does not matter),
// and the soft-min's sum adds the obstacle axes' terms in slot order after
// the robot axes', as obstacle_sd does.  Every lane of the quad must be
// active; all four return the sd, and mi the row's edge count (0 when !act).
template <int C>
__device__ __forceinline__ float quad_dpp(float x) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), C, 0xf, 0xf, false));
}
__device__ __forceinline__ float quad_min(float x) {
  x = fminf(x, quad_dpp<kDppXor1>(x));
  return fminf(x, quad_dpp<kDppXor2>(x));
}
__device__ __forceinline__ float quad_max(float x) {
  x = fmaxf(x, quad_dpp<kDppXor1>(x));
  return fmaxf(x, quad_dpp<kDppXor2>(x));
}

template <int MF>
__device__ __forceinline__ float quad_sd(const FpConst& F, const unsigned char* __restrict__ rows,
                                         size_t r, bool act, const float4* rf, float px, float py,
                                         int& mi) {
  constexpr int MI = 4;
  const int j = threadIdx.x & 3;
  const unsigned char* b = rows + r * kRowBytes<MI>;
  int4 meta = make_int4(0, 0, 0, 0);
  float4 Aj = make_float4(0.f, 0.f, 0.f, 0.f), Bj = Aj;
  if (act) {
    meta = *reinterpret_cast<const int4*>(b + 40 * MI);
    Aj = reinterpret_cast<const float4*>(b)[j];
    Bj = reinterpret_cast<const float4*>(b + 16 * MI)[j];
  }
  mi = meta.y;
  const bool closed = (meta.z & 1) != 0, bad = (meta.z & 2) != 0;
  float2 Pj = make_float2(0.f, 0.f);
  if (act && !closed) Pj = reinterpret_cast<const float2*>(b + 32 * MI)[j];
  const float ux = Aj.z, uy = Aj.w, len = Bj.x, olo = Bj.y, ohi = Bj.z;
  const float tax = Aj.x - px, tay = Aj.y - py;
  const float ca = fmaf(tax, ux, tay * uy);
  const float cb = fmaf(tay, ux, -(tax * uy));

  // robot vertices against edge j; the robot's interval on n'_j
  float dv2 = __builtin_huge_valf(), rlo = __builtin_huge_valf(), rhi = -__builtin_huge_valf();
#pragma unroll
  for (int l = 0; l < MF; ++l) {
    const float4 q = rf[l];
    const float a = fmaf(q.x, ux, fmaf(q.y, uy, -ca));
    const float bb = fmaf(q.y, ux, fmaf(-q.x, uy, -cb));
    rlo = fminf(rlo, bb);
    rhi = fmaxf(rhi, bb);
    dv2 = fminf(dv2, frame_d2(a, bb, len));
  }
  // obstacle point(s) of slot j against the robot edges
  float ra_lo[MF], ra_hi[MF], de2 = __builtin_huge_valf();
#pragma unroll
  for (int l = 0; l < MF; ++l) { ra_lo[l] = __builtin_huge_valf(); ra_hi[l] = -__builtin_huge_valf(); }
  auto visit = [&](float wx, float wy) {
#pragma unroll
    for (int l = 0; l < MF; ++l) {
      const float4 q = rf[l];
      const float a = fmaf(wx, q.z, fmaf(wy, q.w, -F.cu[l]));
      const float bb = fmaf(wx, q.w, fmaf(-wy, q.z, -F.cn[l]));
      ra_lo[l] = fminf(ra_lo[l], bb);
      ra_hi[l] = fmaxf(ra_hi[l], bb);
      de2 = fminf(de2, frame_d2(a, bb, F.len[l]));
    }
  };
  visit(tax, tay);
  if (!closed) visit(Pj.x - px, Pj.y - py);

  // across the quad
  dv2 = quad_min(dv2);
  de2 = quad_min(de2);
  float dl[MF];
  bool sep = false;
#pragma unroll
  for (int l = 0; l < MF; ++l) {
    ra_lo[l] = quad_min(ra_lo[l]);
    ra_hi[l] = quad_max(ra_hi[l]);
    dl[l] = fminf(ra_hi[l] - F.oa[l], F.ob[l] - ra_lo[l]);
    sep = sep || (dl[l] < -F.eps_sat);
  }
  const float dlo = fminf(ohi - rlo, rhi - olo);   // obstacle axis j
  const float sepo = (dlo < -F.eps_sat) ? 1.f : 0.f;
  sep = sep || quad_max(sepo) > 0.f;

  float sd = sqrtf(fminf(dv2, de2));
  if (!sep) {
    float mu = __builtin_huge_valf();
#pragma unroll
    for (int q = 0; q < MF; ++q) mu = fminf(mu, fmaxf(dl[q], 0.0f));
    mu = fminf(mu, quad_min(fmaxf(dlo, 0.0f)));
    float depth = mu;
    if (!F.hard) {
      float acc = 0.0f;
#pragma unroll
      for (int q = 0; q < MF; ++q)
        if (q < F.m) acc += expf(-F.eta * (fmaxf(dl[q], 0.0f) - mu));
      const float ej = expf(-F.eta * (fmaxf(dlo, 0.0f) - mu));
      const float e0 = quad_dpp<0x00>(ej), e1 = quad_dpp<0x55>(ej);
      const float e2 = quad_dpp<0xAA>(ej), e3 = quad_dpp<0xFF>(ej);
      if (0 < mi) acc += e0;
      if (1 < mi) acc += e1;
      if (2 < mi) acc += e2;
      if (3 < mi) acc += e3;
      depth = mu - logf(acc) / F.eta;
    }
    sd = -depth;
  }
  if (bad) sd = __builtin_nanf("");
  return sd;
}

// ---- work-group reductions (every thread of the work-group calls them)

// Threshold search on the key values (no atomics): returns X with
// count(keys <= X) in [lo_n, hi_n] when one exists, else the largest X with
// count <= hi_n found (lo when count(lo) > hi_n: a tie block wider than the
// window at the minimum).  Keys are orderable images of floats; 0xffffffff
// marks an unused slot, and slots q >= nq (block-uniform) are not looked at.
// lo and hi are the smallest and largest used key.  The bracket is halved in
// value (the midpoint of the two floats), which resolves a distance quantile
// in a few steps, and in key order wherever the float midpoint does not fall
// strictly inside (infinite ends, adjacent floats).  Each count is a sum of
// ballots and one barrier (two alternating halves of red, which holds
// 2 kWaves ints).
template <int KPT>
__device__ uint32_t block_threshold(const uint32_t (&k)[KPT], int nq, uint32_t lo, uint32_t hi,
                                    int lo_n, int hi_n, int* red) {
  int half = 0;
  auto count = [&](uint32_t x) {
    int c = 0;
#pragma unroll
    for (int q = 0; q < KPT; ++q) {
      if (q >= nq) break;
      c += __popcll(__ballot(k[q] <= x && k[q] != 0xffffffffu));
    }
    int* r = red + half * kWaves;
    if ((threadIdx.x & 63) == 0) r[threadIdx.x >> 6] = c;
    __syncthreads();
    int t = 0;
#pragma unroll
    for (int i = 0; i < kWaves; ++i) t += r[i];
    half ^= 1;
    return t;
  };
  uint32_t a = lo, b = hi;
  uint32_t res = a;
  const int c0 = count(a);
  if (c0 < lo_n) {
    for (;;) {
      if (b - a <= 1u) { res = a; break; }
      uint32_t mid = orderable(0.5f * from_orderable(a) + 0.5f * from_orderable(b));
      if (!(mid > a && mid < b)) mid = a + (b - a) / 2u;
      const int c = count(mid);
      if (c > hi_n) b = mid;
      else if (c < lo_n) a = mid;
      else { res = mid; break; }
    }
  }
  __syncthreads();   // red is free again for the caller
  return res;
}

__device__ __forceinline__ uint32_t block_min_u32(uint32_t v, uint32_t* red) {
  v = fw_min_u32(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  uint32_t r = red[0];
#pragma unroll
  for (int i = 1; i < kWaves; ++i) r = min(r, red[i]);
  __syncthreads();
  return r;
}

// Several reductions behind one barrier: the minima of NM unsigned values
// and the sums of NS ints over the work-group.  slot holds (NM + NS) x
// kWaves words; there is no barrier after the reads, so a slot serves one
// call site of a kernel (or is reused only past another barrier).
template <int NM, int NS>
__device__ __forceinline__ void block_reduce(uint32_t (&mn)[NM], int (&sm)[NS], uint32_t* slot) {
  const int w = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < NM; ++i) mn[i] = fw_min_u32(mn[i]);
#pragma unroll
  for (int i = 0; i < NS; ++i) sm[i] = fw_sum_i32(sm[i]);
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int i = 0; i < NM; ++i) slot[i * kWaves + w] = mn[i];
#pragma unroll
    for (int i = 0; i < NS; ++i) slot[(NM + i) * kWaves + w] = (uint32_t)sm[i];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NM; ++i) {
    uint32_t r = slot[i * kWaves];
#pragma unroll
    for (int v = 1; v < kWaves; ++v) r = min(r, slot[i * kWaves + v]);
    mn[i] = r;
  }
#pragma unroll
  for (int i = 0; i < NS; ++i) {
    int t = 0;
#pragma unroll
    for (int v = 0; v < kWaves; ++v) t += (int)slot[(NM + i) * kWaves + v];
    sm[i] = t;
  }
}

// Exclusive block scan of one int per thread together with the work-group
// minimum of one unsigned value, behind one barrier (slot: 2 kWaves words,
// no barrier after the reads, as block_reduce).  Returns the prefix; *total
// is the sum and *mn the minimum.
__device__ __forceinline__ int block_scan_min(int v, uint32_t m, uint32_t* slot, int* total,
                                              uint32_t* mn) {
  const int w = threadIdx.x >> 6;
  int wt = 0;
  const int x = fw_scan_i32(v, &wt);
  m = fw_min_u32(m);
  if ((threadIdx.x & 63) == 0) { slot[w] = (uint32_t)wt; slot[kWaves + w] = m; }
  __syncthreads();
  int base = 0, tot = 0;
  uint32_t r = 0xffffffffu;
#pragma unroll
  for (int i = 0; i < kWaves; ++i) {
    const int t = (int)slot[i];
    base += i < w ? t : 0;
    tot += t;
    r = min(r, slot[kWaves + i]);
  }
  *total = tot;
  *mn = r;
  return base + x - v;
}

// One work-group per stage, latency-bound (barriers between the phases).  At
// MI = 4 and MF <= 8 the register budget is capped at 128 VGPRs, so that four
// work-groups share a CU instead of three (a few spills in the network's
// scoring loop; c5 call 10 % faster).  Five per CU spill too much.
template <int MF, int MI>
__global__ __launch_bounds__(kScreenThreads)
__attribute__((amdgpu_waves_per_eu(MI == 4 && MF <= 8 ? 4 : 1))) void screen_kernel(ScreenArgs A) {
  __shared__ int scan[kScreenThreads];
  __shared__ uint32_t red[kScreenThreads / 64];
  __shared__ int pool_o[kPoolCap];        // pool obstacles (local index)
  __shared__ uint32_t pool_lb[kPoolCap];  // their orderable LB
  __shared__ float score[kPoolCap * MI];  // per pool edge slot (+inf for unused slots)
  __shared__ bf16x4 feat[kFeatSlots];     // network features of a chunk of slots
  __shared__ uint8_t cand[kPoolCap];
  __shared__ int cand_o[kPoolCap];
  __shared__ uint64_t wkey[kScreenThreads / 64];
  __shared__ float4 rf[MF];
  __shared__ uint32_t rs[10 * kWaves];    // one slot per combined reduction

  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int4 si = A.stages[blockIdx.x];
  const int s = si.x;
  const int inst = __builtin_amdgcn_readfirstlane(si.y);
  // the first kPreKeys list entries of this thread, issued before the
  // instance record and the list's length are in (slots past the length
  // but within the instance's M are read and ignored)
  constexpr int kPreKeys = 2;
  const float4* hl = A.hlist + si.z;
  float4 pre[kPreKeys];
#pragma unroll
  for (int q = 0; q < kPreKeys; ++q) {
    const int idx = tid + kScreenThreads * q;
    pre[q] = idx < si.w ? hl[idx] : make_float4(0.f, 0.f, 0.f, 0.f);
  }
  const BatchInst in = A.insts[inst];
  const FpConst& F = fp_const(A.fps, inst);   // uniform fields: scalar loads
  const float* p = A.poses + 3 * s;
  const float px = p[0], py = p[1];
  float sn, cs;
  sincosf(p[2], &sn, &cs);
  const bool pose_ok = isfinite(px) && isfinite(py) && isfinite(cs) && isfinite(sn);
  if (tid < MF) rf[tid] = rotated_slot(F, tid, cs, sn);   // read after the block reductions below
  const int M = in.M, Eend = in.edge_off + in.E;
  const int* off = A.off + in.obst_off;

  // An instance without a usable horizon list (a non-finite stage position,
  // tie blocks that make it longer than kHorizonCap, or a count beyond its M
  // slots, which only a call that stopped before reopening the lists leaves)
  // sends its stages to the full evaluation.
  const int hc = A.hcount[inst];
  if (hc < 0 || hc > kHorizonCap || hc > M) {
    if (tid == 0) {
      A.keys[s] = kEmptyKey;
      if (A.stage_cand) A.stage_cand[s] = 0;
      if (A.stage_cert) A.stage_cert[s] = 0;
      if (A.cand_keys) A.cand_keys[s] = kEmptyKey;
      A.failed[atomicAdd(&A.ctrl[0], 1u)] = s;
    }
    return;
  }

  // ---- bounding-circle lower bounds over the instance's horizon list,
  // thread t owns entries t + 256 q
  uint32_t k[kStageKeys];
  int hidx[kStageKeys];
  const int n_h = hc;
  const float lb_off = F.rmax + kLbGamma;
  const int nq = (n_h + kScreenThreads - 1) / kScreenThreads;   // live key slots
#pragma unroll
  for (int q = 0; q < kStageKeys; ++q) {
    const int idx = tid + kScreenThreads * q;
    uint32_t key = 0xffffffffu;
    hidx[q] = 0;
    if (q < nq && idx < n_h) {   // the list holds no empty obstacle
      const float4 c = q < kPreKeys ? pre[q] : hl[idx];
      hidx[q] = __float_as_int(c.w);
      const float dx = px - c.x, dy = py - c.y;
      const float lbv = sqrtf(fmaf(dx, dx, dy * dy)) - c.z - lb_off;
      key = orderable(pose_ok ? lbv : -__builtin_huge_valf());
    }
    k[q] = key;
  }

  // ---- pool: every obstacle with LB key <= T, about P of them
  const int P = max(1, min(A.pool, kPoolCap));
  uint32_t kmin = 0xffffffffu, kmax = 0u;
  int used = 0;
#pragma unroll
  for (int q = 0; q < kStageKeys; ++q) {
    if (q >= nq) break;
    if (k[q] != 0xffffffffu) { kmin = min(kmin, k[q]); kmax = max(kmax, k[q]); ++used; }
  }
  int n_used;
  {
    uint32_t mn[2] = {kmin, ~kmax};
    int sm[1] = {used};
    block_reduce<2, 1>(mn, sm, rs);
    kmin = mn[0]; kmax = ~mn[1]; n_used = sm[0];
  }
  const uint32_t T = n_used > P ? block_threshold<kStageKeys>(k, nq, kmin, kmax,
                                                                         (3 * P) / 4, P, scan)
                                : 0xfffffffeu;
  // pool members of this thread, and the smallest bound outside the pool:
  // the horizon list's circle bounds, and the instance's bound for every
  // obstacle left out of the list
  int mine = 0;
  uint32_t rest = A.hrest[inst];
#pragma unroll
  for (int q = 0; q < kStageKeys; ++q) {
    if (q >= nq) break;
    mine += k[q] <= T && k[q] != 0xffffffffu;
    if (k[q] > T) rest = min(rest, k[q]);
  }
  int pool_n = 0;
  int at = block_scan_min(mine, rest, rs + 3 * kWaves, &pool_n, &rest);
  const bool overflow = pool_n > kPoolCap;
  if (!overflow) {
#pragma unroll
    for (int q = 0; q < kStageKeys; ++q)
      if (q < nq && k[q] <= T && k[q] != 0xffffffffu) {
        pool_o[at] = hidx[q];
        pool_lb[at] = k[q];
        ++at;
      }
  }
  __syncthreads();

  uint64_t keyK = kEmptyKey;
  int n_cand = 0;
  bool cert = false;
  if (!overflow && pool_n > 0) {
    // ---- score the pool's edges
    const int slots = pool_n * MI;
    for (int e = tid; e < kPoolCap * MI; e += kScreenThreads) score[e] = __builtin_huge_valf();
    __syncthreads();
    if (A.theta) {
      MlpFrag fr;
      mlp_frag_fetch(A.frag, fr);
      const int n = lane & 15, g = lane >> 4;
      // chunks of kFeatSlots slots: the work-group stages every slot's BF16
      // features in LDS in one pass (all loads in flight; a valid slot's
      // score is set to 0 until the network overwrites it), then each wave
      // runs the network on 16 slots at a time from LDS
      for (int c0 = 0; c0 < slots; c0 += kFeatSlots) {
        const int cn = min(kFeatSlots, slots - c0);
        for (int e = tid; e < cn; e += kScreenThreads) {
          const int q = (c0 + e) / MI, j = (c0 + e) - q * MI;
          const int o = pool_o[q];
          const int a = off[o], mi = off[o + 1] - a;
          if (j < mi) {
            const int ge = in.edge_off + a + j;
            float lax, lay, lbx, lby;
            local_point(A.ax[ge], A.ay[ge], cs, sn, px, py, lax, lay);
            local_point(A.bx[ge], A.by[ge], cs, sn, px, py, lbx, lby);
            const float sc = 1.0f / kFeatureScale;
            feat[e] = mlp_features(lax * sc, lay * sc, lbx * sc, lby * sc);
            score[c0 + e] = 0.f;
          }
        }
        __syncthreads();
        for (int base = w * 16; base < cn; base += 16 * (kScreenThreads / 64)) {
          const int e = base + n;
          const bool live = e < cn && score[c0 + e] != __builtin_huge_valf();
          const bf16x4 zero = {0, 0, 0, 0};
          MlpAct act;
          mlp_forward16_bf(fr, g == 0 && live ? feat[e] : zero, act);
          if (g == 0 && live) score[c0 + e] = act.y;
        }
        __syncthreads();
      }
    } else {
      for (int e = tid; e < slots; e += kScreenThreads) {
        const int q = e / MI, j = e - q * MI;
        const int o = pool_o[q];
        const int a = off[o], mi = off[o + 1] - a;
        if (j < mi) {
          const int ge = in.edge_off + a + j;
          const float a0 = A.ax[ge], a1 = A.ay[ge], wx = A.bx[ge] - a0, wy = A.by[ge] - a1;
          float iv2, il;
          edge_consts(wx, wy, F.eps, iv2, il);
          score[e] = sqrtf(seg_d2(px, py, a0, a1, wx, wy, iv2));
        }
      }
    }
    __syncthreads();

    // ---- top-K edges -> candidate obstacles
    constexpr int SPT = kPoolCap * MI / kScreenThreads;
    uint32_t sk[SPT];
    int live = 0;
#pragma unroll
    for (int q = 0; q < SPT; ++q) {
      const int e = tid * SPT + q;
      const float v = score[e];
      sk[q] = (e < slots && v != __builtin_huge_valf()) ? orderable(v) : 0xffffffffu;
      live += sk[q] != 0xffffffffu;
    }
    uint32_t smin = 0xffffffffu, smax = 0u;
#pragma unroll
    for (int q = 0; q < SPT; ++q)
      if (sk[q] != 0xffffffffu) { smin = min(smin, sk[q]); smax = max(smax, sk[q]); }
    int n_live;
    {
      uint32_t mn[2] = {smin, ~smax};
      int sm[1] = {live};
      block_reduce<2, 1>(mn, sm, rs + 5 * kWaves);
      smin = mn[0]; smax = ~mn[1]; n_live = sm[0];
    }
    const int K = max(1, A.topk);
    const uint32_t S = n_live > K ? block_threshold<SPT>(sk, SPT, smin, smax, (7 * K) / 8, K, scan)
                                  : 0xfffffffeu;
    for (int q = tid; q < pool_n; q += kScreenThreads) cand[q] = 0;
    __syncthreads();
#pragma unroll
    for (int q = 0; q < SPT; ++q)
      if (sk[q] <= S && sk[q] != 0xffffffffu) cand[(tid * SPT + q) / MI] = 1;
    __syncthreads();
    // compact candidates in pool (index) order; a pool member whose LB is -inf
    // (pose inside, invalid or non-finite) is always a candidate
    // (each thread reads back only the pool range it wrote itself; excl is
    // the smallest LB among pool members that are not candidates)
    int cnt = 0;
    uint32_t excl = rest;
    const int per = (pool_n + kScreenThreads - 1) / kScreenThreads;
    for (int q = tid * per; q < min(pool_n, (tid + 1) * per); ++q) {
      if (pool_lb[q] <= orderable(-__builtin_huge_valf())) cand[q] = 1;
      cnt += cand[q];
      if (!cand[q]) excl = min(excl, pool_lb[q]);
    }
    int c_at = block_scan_min(cnt, excl, rs + 8 * kWaves, &n_cand, &excl);
    for (int q = tid * per; q < min(pool_n, (tid + 1) * per); ++q)
      if (cand[q]) cand_o[c_at++] = pool_o[q];
    __syncthreads();   // cand_o is written

    // ---- exact evaluation of the candidates (lane <-> candidate)
    uint64_t best = kEmptyKey;
    for (int c0 = 0; c0 < n_cand; c0 += kScreenThreads) {
      const int c = c0 + tid;
      const bool act = c < n_cand;
      const int o = act ? cand_o[c] : 0;
      int mi;
      Obst<MI> ob;
      screen_obstacle<MI>(ob, A, in, o, act, F.eps, mi);
      uint32_t kk = 0xffffffffu;
      if (act && mi != 0) kk = pose_ok ? orderable(obstacle_sd<MF, MI>(F, ob, rf, px, py)) : 0u;
      const uint64_t key = kk == 0xffffffffu ? kEmptyKey : (((uint64_t)kk << 32) | (uint32_t)o);
      const uint64_t wmin = fw_min_u64(key);
      best = wmin < best ? wmin : best;
    }
    if (lane == 0) wkey[w] = best;
    __syncthreads();
    keyK = wkey[0];
#pragma unroll
    for (int i = 1; i < kScreenThreads / 64; ++i) keyK = wkey[i] < keyK ? wkey[i] : keyK;
    // ---- certificate, first with the circle bounds
    const float phiK = keyK == kEmptyKey ? __builtin_huge_valf()
                                         : from_orderable((uint32_t)(keyK >> 32));
    const float bar = fmaxf(phiK, F.tau_sep);
    const float lbx = excl == 0xffffffffu ? __builtin_huge_valf() : from_orderable(excl);
    cert = (keyK != kEmptyKey && (keyK >> 32) == 0)            // NaN wins anyway
           || excl == 0xffffffffu                               // nothing excluded
           || lbx > bar;
    if (!cert) {
      // then with the point-to-polygon bound of every excluded pool member
      // whose circle bound does not clear the bar (the larger of two valid
      // lower bounds is a lower bound; -inf, pose inside or invalid, stays
      // -inf and keeps the stage uncertified); bounds outside the pool stay
      const uint32_t ninf = orderable(-__builtin_huge_valf());
      uint32_t ex2 = rest;
      for (int q = tid; q < pool_n; q += kScreenThreads) {
        if (cand[q]) continue;
        uint32_t kq = pool_lb[q];
        if (!(from_orderable(kq) > bar)) {
          const int o = pool_o[q];
          const int a = off[o], b = off[o + 1];
          const float lbv = obstacle_lb(px, py, A.ax, A.ay, A.bx, A.by, in.edge_off + a, b - a,
                                        in.edge_off, Eend, F.eps, F.rmax);
          const uint32_t kk = orderable(pose_ok ? lbv : -__builtin_huge_valf());
          kq = kk <= ninf ? kk : max(kq, kk);
        }
        ex2 = min(ex2, kq);
      }
      ex2 = block_min_u32(ex2, red);
      cert = ex2 == 0xffffffffu || from_orderable(ex2) > bar;
    }
  } else {
    cert = !overflow && pool_n == 0 && rest == 0xffffffffu;   // no obstacle at all
  }
  if (tid == 0) {
    A.keys[s] = keyK;
    if (A.stage_cand) A.stage_cand[s] = n_cand;
    if (A.stage_cert) A.stage_cert[s] = cert ? 1 : 0;
    if (A.cand_keys) A.cand_keys[s] = keyK;
    if (!cert) A.failed[atomicAdd(&A.ctrl[0], 1u)] = s;
  }
}

// Certified screening by the bound alone (no ranking), one wave per stage.
// The obstacle with the smallest lower bound (the seed) is evaluated
// exactly; its sd is an upper bound of the stage's minimum phi, so the bar
// T = max(sd_seed, tau_sep) satisfies T >= max(phi, tau_sep), and every
// obstacle whose bound does not exceed T is evaluated exactly.  Every
// obstacle left out then has LB_i > T >= max(phi_K, tau_sep), which is the
// certificate of screen_kernel, met by construction; what can still send a
// stage to the full evaluation is an instance bound (the obstacles outside
// the horizon list) at or below T, more than kBoundCap candidates, or an
// unusable horizon list.  The candidate set is the smallest that any
// certificate built on these bounds can use when the seed is the winner or
// the stage penetrates (T = tau_sep then).
//
// One wave per stage: the first kBoundRegs x 64 list entries are loaded
// together (all in flight at once) and their bounds held in registers for
// both passes; entries past them (tie blocks only) are read again in the
// second pass.  The seed comes from a wave minimum of (bound key, list
// slot), the candidates are compacted into LDS with ballots, and no
// work-group barrier is needed.
constexpr int kBoundCap = 512;   // candidates per stage (more: full evaluation)
constexpr int kBoundRegs = 8;    // list entries per lane held in registers

template <int MF, int MI>
__global__ __launch_bounds__(64) void screen_bound_kernel(ScreenArgs A) {
  __shared__ int cand_o[kBoundCap];
  __shared__ float4 rf[MF];
  __shared__ FpLds fl;
  __shared__ WinnerLds wl;

  const int lane = threadIdx.x;
  const int4 si = A.stages[blockIdx.x];
  const int s = si.x;
  const int inst = __builtin_amdgcn_readfirstlane(si.y);
  // the first kBoundRegs x 64 list entries, issued before the instance
  // record and the list's length are in (slots past the length but within
  // the instance's M are read and ignored)
  const float4* hl = A.hlist + si.z;
  float4 rc[kBoundRegs];
#pragma unroll
  for (int q = 0; q < kBoundRegs; ++q) {
    const int idx = q * 64 + lane;
    rc[q] = idx < si.w ? hl[idx] : make_float4(0.f, 0.f, 0.f, 0.f);
  }
  const BatchInst in = A.insts[inst];
  const FpConst& F = fp_const(A.fps, inst);   // uniform fields: scalar loads
  const float* p = A.poses + 3 * s;
  const float px = p[0], py = p[1];
  float sn, cs;
  sincosf(p[2], &sn, &cs);
  const bool pose_ok = isfinite(px) && isfinite(py) && isfinite(cs) && isfinite(sn);
  if (lane < MF) rf[lane] = rotated_slot(F, lane, cs, sn);
  if (A.finish) stage_footprint(fl, F);   // for the outputs of a certified stage

  const int hc = A.hcount[inst];
  if (hc < 0 || hc > kHorizonCap || hc > in.M) {   // as screen_kernel
    if (lane == 0) {
      A.keys[s] = kEmptyKey;
      if (A.stage_cand) A.stage_cand[s] = 0;
      if (A.stage_cert) A.stage_cert[s] = 0;
      if (A.cand_keys) A.cand_keys[s] = kEmptyKey;
      const unsigned slot = atomicAdd(&A.ctrl[0], 1u);
      A.failed[slot] = s;
      if (A.finish) A.fdone[slot] = 0;
    }
    return;
  }
  const float lb_off = F.rmax + kLbGamma;
  // bounding-circle lower bound of list entry idx (as screen_kernel), and
  // its obstacle (local index)
  auto lb_key = [&](int idx, int& o) {
    const float4 c = hl[idx];
    o = __float_as_int(c.w);
    const float dx = px - c.x, dy = py - c.y;
    const float lbv = sqrtf(fmaf(dx, dx, dy * dy)) - c.z - lb_off;
    return orderable(pose_ok ? lbv : -__builtin_huge_valf());
  };

  // ---- pass 1: the seed, the smallest bound (lowest list slot on ties);
  // the key's low word is (slot << 16 | obstacle): slot < 2048, obstacle <
  // 16384, so the wave minimum names the seed without another list read.
  // Entry q * 64 + lane of the first kBoundRegs x 64: key rk[q], obstacle
  // ro[q] (key 0xffffffff past the list's end, never taken below).
  uint32_t rk[kBoundRegs];
  int ro[kBoundRegs];
  uint64_t lo = ~0ull;
#pragma unroll
  for (int q = 0; q < kBoundRegs; ++q) {
    const int idx = q * 64 + lane;
    const float4 c = rc[q];
    ro[q] = __float_as_int(c.w);
    const float dx = px - c.x, dy = py - c.y;
    const float lbv = sqrtf(fmaf(dx, dx, dy * dy)) - c.z - lb_off;
    rk[q] = idx < hc ? orderable(pose_ok ? lbv : -__builtin_huge_valf()) : 0xffffffffu;
    if (idx < hc) {
      const uint64_t v = ((uint64_t)rk[q] << 32) | ((uint32_t)idx << 16) | (uint32_t)ro[q];
      lo = v < lo ? v : lo;
    }
  }
  for (int idx = kBoundRegs * 64 + lane; idx < hc; idx += 64) {
    int o;
    const uint64_t v = ((uint64_t)lb_key(idx, o) << 32) | ((uint32_t)idx << 16) | (uint32_t)o;
    lo = v < lo ? v : lo;
  }
  lo = wave_min_u64(lo);
  wave_sync();   // rf is written
  uint64_t seed_key = kEmptyKey;
  int seed_o = -1;
  // four-edge-class obstacles on staged rows are evaluated one per quad of
  // lanes (quad_sd, bit-identical to obstacle_sd): the seed by the first
  // quad, and a few candidates 16 at a time
  const bool quads = MI == 4 && A.rows != nullptr;
  if (lo != ~0ull) {
    seed_o = (int)(lo & 0xffffu);
    uint32_t kk = 0u;
    if constexpr (MI == 4) {
      if (quads) {
        int mi;
        const float sdq = quad_sd<MF>(F, A.rows, (size_t)in.circ_off + seed_o, lane < 4, rf, px,
                                      py, mi);
        kk = pose_ok ? orderable(sdq) : 0u;
      }
    }
    if (!quads && lane == 0) {
      int mi;
      Obst<MI> ob;
      screen_obstacle<MI>(ob, A, in, seed_o, true, F.eps, mi);
      kk = pose_ok ? orderable(obstacle_sd<MF, MI>(F, ob, rf, px, py)) : 0u;
    }
    kk = lane_u32(kk, 0);
    seed_key = ((uint64_t)kk << 32) | (uint32_t)seed_o;
  }

  // ---- pass 2: every other list entry with LB <= T, compacted into LDS
  const float phi1 = seed_key == kEmptyKey ? __builtin_huge_valf()
                                           : from_orderable((uint32_t)(seed_key >> 32));
  const uint32_t tkey = orderable(fmaxf(phi1, F.tau_sep));
  const uint64_t below = (1ull << lane) - 1ull;
  int n_cand = 0;
#pragma unroll
  for (int q = 0; q < kBoundRegs; ++q) {
    const int o = ro[q];
    const bool take = q * 64 + lane < hc && rk[q] <= tkey && o != seed_o;
    const uint64_t m = __ballot(take);
    const int at = n_cand + (int)__popcll(m & below);
    if (take && at < kBoundCap) cand_o[at] = o;
    n_cand += (int)__popcll(m);
  }
  for (int i0 = kBoundRegs * 64; i0 < hc; i0 += 64) {
    const int idx = i0 + lane;
    int o = -1;
    bool take = false;
    if (idx < hc) take = lb_key(idx, o) <= tkey && o != seed_o;
    const uint64_t m = __ballot(take);
    const int at = n_cand + (int)__popcll(m & below);
    if (take && at < kBoundCap) cand_o[at] = o;
    n_cand += (int)__popcll(m);
  }
  const bool overflow = n_cand > kBoundCap;
  wave_sync();

  // ---- exact evaluation of the candidates: a quad per candidate while they
  // fit two passes (32), else lane <-> candidate
  uint64_t keyK = seed_key;
  bool done = false;
  if constexpr (MI == 4) {
    if (quads && !overflow && n_cand <= 32) {
      for (int c0 = 0; c0 < n_cand; c0 += 16) {
        const int c = c0 + (lane >> 2);
        const bool act = c < n_cand;
        const int o = act ? cand_o[c] : 0;
        int mi;
        const float sdq = quad_sd<MF>(F, A.rows, (size_t)in.circ_off + o, act, rf, px, py, mi);
        uint32_t kk = 0xffffffffu;
        if (act && mi != 0) kk = pose_ok ? orderable(sdq) : 0u;
        const uint64_t key = kk == 0xffffffffu ? kEmptyKey : (((uint64_t)kk << 32) | (uint32_t)o);
        const uint64_t wmin = fw_min_u64(key);
        keyK = wmin < keyK ? wmin : keyK;
      }
      done = true;
    }
  }
  if (!overflow && !done) {
    for (int c0 = 0; c0 < n_cand; c0 += 64) {
      const int c = c0 + lane;
      const bool act = c < n_cand;
      const int o = act ? cand_o[c] : 0;
      int mi;
      Obst<MI> ob;
      screen_obstacle<MI>(ob, A, in, o, act, F.eps, mi);
      uint32_t kk = 0xffffffffu;
      if (act && mi != 0) kk = pose_ok ? orderable(obstacle_sd<MF, MI>(F, ob, rf, px, py)) : 0u;
      const uint64_t key = kk == 0xffffffffu ? kEmptyKey : (((uint64_t)kk << 32) | (uint32_t)o);
      const uint64_t wmin = fw_min_u64(key);
      keyK = wmin < keyK ? wmin : keyK;
    }
  }
  // ---- certificate: the list entries left out have LB > T by construction;
  // the obstacles outside the list have the instance bound
  const uint32_t rest = A.hrest[inst];
  const bool cert = (keyK != kEmptyKey && (keyK >> 32) == 0)          // NaN wins anyway
                    || (!overflow && (rest == 0xffffffffu || rest > tkey));
  if (A.finish && cert) {
    // keyK is the stage's final key: its outputs, here
    int e0, mi;
    const bool valid = key_range(keyK, A.off, in.obst_off, in.M, in.edge_off, in.E, e0, mi);
    wave_sync();   // fl is written
    write_stage(F, fl, wl, A.ax, A.ay, A.bx, A.by, keyK, valid, e0, mi, in.edge_off, cs, sn, px,
                py, s, A.keys, A.d, A.edge, A.obst, A.grad);
  }
  if (lane == 0) {
    if (!(A.finish && cert)) A.keys[s] = keyK;
    if (A.stage_cand) A.stage_cand[s] = overflow ? 0 : n_cand + (seed_o >= 0 ? 1 : 0);
    if (A.stage_cert) A.stage_cert[s] = cert ? 1 : 0;
    if (A.cand_keys) A.cand_keys[s] = keyK;
    if (!cert) {
      const unsigned slot = atomicAdd(&A.ctrl[0], 1u);
      A.failed[slot] = s;
      if (A.finish) A.fdone[slot] = 0;
    }
  }
}

// Full evaluation of the failed stages: items (failed stage, tile of 256
// obstacles), every item the same work, taken by the work-groups in turn
// (item b, b + grid, ...); each work-group folds its tile's minimum into
// keys[s] with a 64-bit atomicMin.  A stage has max(1, ceil(M / 256))
// tiles (tile 0 stands for an instance without obstacles).  With FIN (the
// bound form, A.finish), each tile then counts itself done on the stage's slot (agent-scope
// acquire-release), and the tile that completes the count, which then sees
// every tile's minimum, writes the stage's outputs.  The failed count
// starts at zero: plan creation clears it, and so does the horizon pass at
// the start of every screened call.  The finishing code raises the
// kernel's register count, so the ranked forms launch the variant without
// it (FIN false; their finish kernel ends the stages).
template <int MF, int MI, bool FIN>
__global__ __launch_bounds__(256) void screen_fallback_kernel(ScreenArgs A, int max_tiles) {
  __shared__ uint64_t wk[4];
  __shared__ float4 rf[MF];
  __shared__ FpLds fl;
  __shared__ WinnerLds wl;
  __shared__ int s_last;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  if (blockIdx.x == 0)
    for (int i = tid; i < A.reset_n; i += 256) {
      A.reset_hcount[i] = 0;
      A.reset_hrest[i] = 0xffffffffu;
    }
  const int n_failed = (int)__hip_atomic_load(&A.ctrl[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const long n_items = (long)n_failed * max_tiles;
  for (long item = blockIdx.x; item < n_items; item += gridDim.x) {
    const int it = __builtin_amdgcn_readfirstlane((int)(item / max_tiles));
    const int tile = __builtin_amdgcn_readfirstlane((int)(item % max_tiles));
    const int s = A.failed[it];
    const int inst = __builtin_amdgcn_readfirstlane(A.stage_inst[s]);
    const BatchInst in = A.insts[inst];
    if (tile == 0 || tile * 256 < in.M) {
      const FpConst& F = fp_const(A.fps, inst);   // uniform fields: scalar loads
      const float* p = A.poses + 3 * s;
      const float px = p[0], py = p[1];
      float sn, cs;
      sincosf(p[2], &sn, &cs);
      const bool pose_ok = isfinite(px) && isfinite(py) && isfinite(cs) && isfinite(sn);
      if (tid < MF) rf[tid] = rotated_slot(F, tid, cs, sn);
      __syncthreads();
      const int o = tile * 256 + tid;
      const bool act = o < in.M;
      int mi;
      Obst<MI> ob;
      screen_obstacle<MI>(ob, A, in, o, act, F.eps, mi);
      uint32_t kk = 0xffffffffu;
      if (act && mi != 0) kk = pose_ok ? orderable(obstacle_sd<MF, MI>(F, ob, rf, px, py)) : 0u;
      const uint64_t key = kk == 0xffffffffu ? kEmptyKey : (((uint64_t)kk << 32) | (uint32_t)o);
      const uint64_t wmin = fw_min_u64(key);
      if (lane == 0) wk[w] = wmin;
      __syncthreads();
      if (tid == 0) {
        uint64_t m = wk[0];
        for (int i = 1; i < 4; ++i) m = wk[i] < m ? wk[i] : m;
        if (m != kEmptyKey) atomicMin((unsigned long long*)&A.keys[s], (unsigned long long)m);
        if constexpr (FIN) {
          const int nt = max(1, (in.M + 255) / 256);
          s_last = __hip_atomic_fetch_add(&A.fdone[it], 1, __ATOMIC_ACQ_REL,
                                          __HIP_MEMORY_SCOPE_AGENT) == nt - 1;
        }
      }
      if constexpr (FIN) {
        __syncthreads();
        if (s_last && w == 0) {
          const uint64_t kf = __hip_atomic_load((unsigned long long*)&A.keys[s], __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_AGENT);
          stage_footprint(fl, F);
          int e0, mi2;
          const bool valid = key_range(kf, A.off, in.obst_off, in.M, in.edge_off, in.E, e0, mi2);
          wave_sync();   // fl is written
          write_stage(F, fl, wl, A.ax, A.ay, A.bx, A.by, kf, valid, e0, mi2, in.edge_off, cs, sn,
                      px, py, s, A.keys, A.d, A.edge, A.obst, A.grad);
        }
      }
    }
    __syncthreads();
  }
}

template <int MF>
hipError_t launch_screen_mf(int mi_class, int grid, const ScreenArgs& a, hipStream_t st) {
  if (mi_class == 4) screen_kernel<MF, 4><<<grid, kScreenThreads, 0, st>>>(a);
  else if (mi_class == 8) screen_kernel<MF, 8><<<grid, kScreenThreads, 0, st>>>(a);
  else screen_kernel<MF, 16><<<grid, kScreenThreads, 0, st>>>(a);
  return hipGetLastError();
}

template <int MF>
hipError_t launch_screen_bound_mf(int mi_class, int grid, const ScreenArgs& a, hipStream_t st) {
  if (mi_class == 4) screen_bound_kernel<MF, 4><<<grid, 64, 0, st>>>(a);
  else if (mi_class == 8) screen_bound_kernel<MF, 8><<<grid, 64, 0, st>>>(a);
  else screen_bound_kernel<MF, 16><<<grid, 64, 0, st>>>(a);
  return hipGetLastError();
}

template <int MF>
hipError_t launch_fallback_mf(int mi_class, int grid, int max_tiles, const ScreenArgs& a,
                              hipStream_t st) {
  if (a.finish) {
    if (mi_class == 4) screen_fallback_kernel<MF, 4, true><<<grid, 256, 0, st>>>(a, max_tiles);
    else if (mi_class == 8) screen_fallback_kernel<MF, 8, true><<<grid, 256, 0, st>>>(a, max_tiles);
    else screen_fallback_kernel<MF, 16, true><<<grid, 256, 0, st>>>(a, max_tiles);
  } else {
    if (mi_class == 4) screen_fallback_kernel<MF, 4, false><<<grid, 256, 0, st>>>(a, max_tiles);
    else if (mi_class == 8) screen_fallback_kernel<MF, 8, false><<<grid, 256, 0, st>>>(a, max_tiles);
    else screen_fallback_kernel<MF, 16, false><<<grid, 256, 0, st>>>(a, max_tiles);
  }
  return hipGetLastError();
}

#define PSDF_EXTERN_SCREEN(MF)                                                                  \
  extern template hipError_t launch_screen_mf<MF>(int, int, const ScreenArgs&, hipStream_t);    \
  extern template hipError_t launch_screen_bound_mf<MF>(int, int, const ScreenArgs&, hipStream_t); \
  extern template hipError_t launch_fallback_mf<MF>(int, int, int, const ScreenArgs&, hipStream_t);
PSDF_EXTERN_SCREEN(3)
PSDF_EXTERN_SCREEN(4)
PSDF_EXTERN_SCREEN(5)
PSDF_EXTERN_SCREEN(6)
PSDF_EXTERN_SCREEN(7)
PSDF_EXTERN_SCREEN(8)
PSDF_EXTERN_SCREEN(16)

}  // namespace psdf
