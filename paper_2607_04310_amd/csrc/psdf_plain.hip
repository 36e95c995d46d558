// Plain PSDF path for gfx950: psdf_eval, psdf_grad, psdf_bwd, psdf_encode_padded.
//
// Kernel sequence of one call (all on the caller's stream, no host sync):
//   main_kernel      per-work-group partial minimum of (sd, obstacle) per stage
//                    (psdf_kernels.hpp)
//   epilogue_kernel  one wave per stage: reduce the partial keys, recompute the
//                    winning obstacle with the wave-parallel adjoint
//                    (psdf_winner.hpp), write keys, d, edge, obst, gradient
// or, for at most 256 obstacles of at most four edges, small_kernel alone
// (both steps for a stage in one launch, bit for bit the same outputs).
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>
#include <vector>

#include "psdf.h"
#include "psdf_kernels.hpp"
#include "psdf_winner.hpp"

namespace psdf {

constexpr int kEpiWaves = 1;   // stages per epilogue work-group

// mode 0: value, winner and edge; 1: plus gradient; 2: bwd (gradient scaled
// by gout[s], written to grad only; keys are read, not reduced).  In modes 0
// and 1 each of d / edge / obst, grad and hj may be null; hj[s] receives the
// linearised safety constraint (phi - dmin, -dphi/dx, -dphi/dy, -dphi/dtheta)
// (mode 1 only).
struct EpiOut {
  uint64_t* keys;
  const float* gout;
  int mode;
  float dmin;
  float* d;
  int* edge;
  int* obst;
  float* grad;
  float* hj;
};

// One wave finishes stage s from its winning key: the winner's edge range
// (e0, mi) comes from the aux word (have_aux) or from the offsets; the wave
// recomputes the winner (winner_adjoint) and lane 0 writes the outputs.
__device__ __forceinline__ void epilogue_finish(const FpConst& F, FpLds& FL, WinnerLds& WL,
                                                const float* __restrict__ ax,
                                                const float* __restrict__ ay,
                                                const float* __restrict__ bx,
                                                const float* __restrict__ by,
                                                const int* __restrict__ off, int E, int M, int s,
                                                float px, float py, float cs, float sn,
                                                uint64_t key, int e0, int mi, bool have_aux,
                                                float scale, const EpiOut& O) {
  const int lane = threadIdx.x & 63;
  const float nan = __builtin_nanf("");
  float dv, g[3] = {0.f, 0.f, 0.f};
  int ev = -1, ov = -1;
  const int i = (int)(key & 0xffffffffu);
  bool valid = key != kEmptyKey && (key >> 32) != 0 && (uint64_t)i < (uint64_t)M;
  if (valid && !have_aux) {
    e0 = off[i];
    mi = off[i + 1] - e0;
  }
  valid = valid && mi >= 1 && mi <= kMaxObst && e0 >= 0 && e0 <= E - mi;
  if (key == kEmptyKey) {
    dv = __builtin_huge_valf();
  } else if (!valid) {
    // NaN result, or a key that names no obstacle of this edge set
    dv = nan;
    g[0] = g[1] = g[2] = nan;
  } else {
    int jstar = 0;
    winner_adjoint(F, FL, WL, ax, ay, bx, by, e0, mi, cs, sn, px, py, O.mode != 0, jstar, g);
    dv = from_orderable((uint32_t)(key >> 32));
    ov = i;
    ev = e0 + jstar;
  }
  if (lane != 0) return;
  if (O.mode == 2) {
    O.grad[3 * s + 0] = g[0] * scale;
    O.grad[3 * s + 1] = g[1] * scale;
    O.grad[3 * s + 2] = g[2] * scale;
    return;
  }
  if (O.d) {
    O.d[s] = dv;
    O.edge[s] = ev;
    O.obst[s] = ov;
  }
  if (O.mode == 1 && O.grad) {
    O.grad[3 * s + 0] = g[0];
    O.grad[3 * s + 1] = g[1];
    O.grad[3 * s + 2] = g[2];
  }
  if (O.mode == 1 && O.hj) {
    O.hj[4 * s + 0] = dv - O.dmin;
    O.hj[4 * s + 1] = -g[0];
    O.hj[4 * s + 2] = -g[1];
    O.hj[4 * s + 3] = -g[2];
  }
}

// One wave per stage: reduce the stage's gx partial keys (a few columns per
// lane), then finish the stage.
__global__ __launch_bounds__(64 * kEpiWaves) void epilogue_kernel(
    FpConst F, const float* __restrict__ poses, int N, const float* __restrict__ ax,
    const float* __restrict__ ay, const float* __restrict__ bx, const float* __restrict__ by,
    const int* __restrict__ off, int E, int M, const uint64_t* __restrict__ partial, int gx,
    EpiOut O) {
  __shared__ FpLds fl[kEpiWaves];
  __shared__ WinnerLds wl[kEpiWaves];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int s = blockIdx.x * kEpiWaves + w;
  if (s >= N) return;
  // Every independent load in flight at once: the pose, the partial keys and
  // their aux words (or the stored key), the footprint constants.
  const float* p = poses + 3 * s;
  const float px = p[0], py = p[1], th = p[2];
  uint64_t key = kEmptyKey, a = 0;
  float scale = 1.0f;
  // (key, aux) per column; the winning column's aux word carries the
  // obstacle's edge range
  const ulonglong2* prow = reinterpret_cast<const ulonglong2*>(partial) + (size_t)s * gx;
  if (O.mode == 2) {
    key = O.keys[s];
    scale = O.gout[s];
  } else if (lane < gx) {
    const ulonglong2 v = prow[lane];
    key = v.x;
    a = v.y;
  }
  stage_footprint(fl[w], F);
  if (O.mode != 2) {
    // keys are unique (they carry the obstacle index), so the scan order is
    // free: four columns per lane in flight
    int j = lane + 64;
    for (; j + 192 < gx; j += 256) {
      ulonglong2 v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) v[u] = prow[j + 64 * u];
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (v[u].x < key) { key = v[u].x; a = v[u].y; }
    }
    for (; j < gx; j += 64) {
      const ulonglong2 v = prow[j];
      if (v.x < key) { key = v.x; a = v.y; }
    }
  }
  float sn, cs;
  sincosf(th, &sn, &cs);

  int e0 = 0, mi = 0;
  bool have_aux = false;
  if (O.mode != 2) {
    const uint64_t kmin = wave_min_u64(key);
    const uint64_t hit = __ballot(key == kmin);
    const int first = __ffsll((unsigned long long)hit) - 1;
    a = lane_u64(a, first);
    key = kmin;
    if (lane == 0) O.keys[s] = key;
    e0 = (int)(uint32_t)(a >> 32);
    mi = (int)(uint32_t)(a & 0xffffffffu);
    have_aux = true;
  }
  wave_sync();
  epilogue_finish(F, fl[w], wl[w], ax, ay, bx, by, off, E, M, s, px, py, cs, sn, key, e0, mi,
                  have_aux, scale, O);
}

// Many columns (few stages, many obstacles): one work-group per stage
// reduces the keys alone (eight columns per lane in flight), loads the
// winning column's aux word, and its first wave finishes the stage.
constexpr int kWideThreads = 256;
constexpr int kWideColumns = 256;   // wider rows than this take this kernel

__global__ __launch_bounds__(kWideThreads) void epilogue_wide_kernel(
    FpConst F, const float* __restrict__ poses, int N, const float* __restrict__ ax,
    const float* __restrict__ ay, const float* __restrict__ bx, const float* __restrict__ by,
    const int* __restrict__ off, int E, int M, const uint64_t* __restrict__ partial, int gx,
    EpiOut O) {
  __shared__ FpLds fl;
  __shared__ WinnerLds wl;
  __shared__ uint64_t red[kWideThreads / 64];
  __shared__ uint64_t s_aux;
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const int s = blockIdx.x;
  const ulonglong2* prow = reinterpret_cast<const ulonglong2*>(partial) + (size_t)s * gx;
  uint64_t key = kEmptyKey;
  int col = 0;
  int j = tid;
  for (; j + 7 * kWideThreads < gx; j += 8 * kWideThreads) {
    uint64_t k[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) k[u] = prow[j + u * kWideThreads].x;
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (k[u] < key) { key = k[u]; col = j + u * kWideThreads; }
  }
  for (; j < gx; j += kWideThreads)
    if (prow[j].x < key) { key = prow[j].x; col = j; }
  const uint64_t wmin = wave_min_u64(key);
  if (lane == 0) red[w] = wmin;
  if (w == 0) stage_footprint(fl, F);
  __syncthreads();
  uint64_t kmin = red[0];
#pragma unroll
  for (int v = 1; v < kWideThreads / 64; ++v) kmin = red[v] < kmin ? red[v] : kmin;
  // keys are unique, so exactly one thread holds kmin (none if all are empty)
  if (kmin != kEmptyKey && key == kmin) s_aux = prow[col].y;
  __syncthreads();
  if (w != 0) return;
  const float* p = poses + 3 * s;
  const float px = p[0], py = p[1];
  float sn, cs;
  sincosf(p[2], &sn, &cs);
  const uint64_t a = kmin != kEmptyKey ? s_aux : 0;
  if (lane == 0) O.keys[s] = kmin;
  epilogue_finish(F, fl, wl, ax, ay, bx, by, off, E, M, s, px, py, cs, sn, kmin,
                  (int)(uint32_t)(a >> 32), (int)(uint32_t)(a & 0xffffffffu), true, 1.0f, O);
}

static int mf_slots(int m) { return m <= 8 ? m : 16; }

#define PSDF_BY_MF(FN, ...)                                      \
  [&]() -> hipError_t {                                          \
    switch (mf_slots(F.m)) {                                     \
      case 3: return FN<3>(__VA_ARGS__);                         \
      case 4: return FN<4>(__VA_ARGS__);                         \
      case 5: return FN<5>(__VA_ARGS__);                         \
      case 6: return FN<6>(__VA_ARGS__);                         \
      case 7: return FN<7>(__VA_ARGS__);                         \
      case 8: return FN<8>(__VA_ARGS__);                         \
      default: return FN<16>(__VA_ARGS__);                       \
    }                                                            \
  }()

int partial_columns(int M, const LaunchShape& ls) { return (M + ls.blk - 1) / ls.blk; }

// Small edge sets (1 <= M <= 256 obstacles of at most four edges): NW waves
// hold every obstacle of a stage (lane <-> obstacle, wave w takes obstacles
// 64 w ...), take the stage's minimum with the same wave_stages arithmetic as
// main_kernel, and the first wave finishes the stage at once
// (epilogue_finish): one launch instead of two.  The result is the
// two-kernel result bit for bit: keys are unique, so the minimum over the
// waves' (key, aux) pairs is what the epilogue would have reduced.  One
// stage per work-group of NW waves (one-wave work-groups spread the stages
// over the CUs).
constexpr int kSmallMaxM = 256;

template <int MF, int NW>
__global__ __launch_bounds__(64 * NW) void small_kernel(
    FpConst F, const float* __restrict__ poses, int N, const float* __restrict__ ax,
    const float* __restrict__ ay, const float* __restrict__ bx, const float* __restrict__ by,
    const int* __restrict__ off, int E, int M, EpiOut O) {
  __shared__ float4 st[1];
  __shared__ float4 rft[MF];
  __shared__ FpLds fl[1];
  __shared__ WinnerLds wl[1];
  __shared__ uint64_t wk[NW], wa[NW];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int s = blockIdx.x;
  if (s >= N) return;   // the whole work-group
  const int obase = 64 * w;
  const bool active = obase + lane < M;
  int e0 = 0, mi = 0;
  if (active) {
    e0 = off[obase + lane];
    mi = off[obase + lane + 1] - e0;
  }
  const float* p = poses + 3 * s;
  const float px = p[0], py = p[1];
  float sn, cs;
  sincosf(p[2], &sn, &cs);
  // the stage table, as fill_stage_table builds it (written by the stage's
  // first wave)
  if (w == 0) {
    if (lane < MF) rft[lane] = rotated_slot(F, lane, cs, sn);
    if (lane == 0) st[0] = make_float4(cs, sn, px, py);
    stage_footprint(fl[0], F);
  }
  if (NW == 1) wave_sync();
  else __syncthreads();
  uint64_t key = kEmptyKey, a = 0;   // uniform across the wave
  if (obase < M) {
    auto emit = [&](int, uint64_t k, uint64_t x) {
      key = k;
      a = x;
    };
    wave_stages<MF, 4>(F, ax, ay, bx, by, e0, mi, E, active, false, obase, 1, st, rft, emit);
  }
  if (NW > 1) {
    if (lane == 0) {
      wk[w] = key;
      wa[w] = a;
    }
    __syncthreads();
    if (w != 0) return;
#pragma unroll
    for (int v = 1; v < NW; ++v)
      if (wk[v] < key) {
        key = wk[v];
        a = wa[v];
      }
  }
  if (lane == 0) O.keys[s] = key;
  epilogue_finish(F, fl[0], wl[0], ax, ay, bx, by, off, E, M, s, px, py, cs, sn, key,
                  (int)(uint32_t)(a >> 32), (int)(uint32_t)(a & 0xffffffffu), true, 1.0f, O);
}

template <int MF>
hipError_t launch_small_mf(const FpConst& F, const float* poses, int N, const psdf_edges& e,
                           const EpiOut& O, hipStream_t st) {
  if (e.M <= 64)
    small_kernel<MF, 1><<<N, 64, 0, st>>>(F, poses, N, e.ax, e.ay, e.bx, e.by, e.obst_off, e.E,
                                          e.M, O);
  else
    small_kernel<MF, 4><<<N, 256, 0, st>>>(F, poses, N, e.ax, e.ay, e.bx, e.by, e.obst_off, e.E,
                                           e.M, O);
  return hipGetLastError();
}

bool small_path(const psdf_edges& e) {
  return e.M >= 1 && e.M <= kSmallMaxM && obst_class(e.mbar) == 4;
}


hipError_t launch_plain(const FpConst& F, const float* poses, int N, const psdf_edges& e,
                        uint64_t* partial, const LaunchShape& ls, hipStream_t st) {
  if (e.M == 0) return hipSuccess;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  if (!timer_kernel_events(&ev0, &ev1)) ev0 = ev1 = nullptr;
  return PSDF_BY_MF(launch_main_mf, obst_class(e.mbar), ls, F, poses, N, e, partial, st, ev0,
                    ev1);
}

hipError_t launch_epilogue(const FpConst& F, const float* poses, int N, const psdf_edges& e,
                           const uint64_t* partial, int gx, uint64_t* keys, const float* gout,
                           int mode, float dmin, float* d, int* edge, int* obst, float* grad,
                           float* hj, hipStream_t st) {
  const EpiOut O{keys, gout, mode, dmin, d, edge, obst, grad, hj};
  if (mode != 2 && gx > kWideColumns) {
    epilogue_wide_kernel<<<N, kWideThreads, 0, st>>>(F, poses, N, e.ax, e.ay, e.bx, e.by,
                                                     e.obst_off, e.E, e.M, partial, gx, O);
  } else {
    const int blocks = (N + kEpiWaves - 1) / kEpiWaves;
    epilogue_kernel<<<blocks, 64 * kEpiWaves, 0, st>>>(F, poses, N, e.ax, e.ay, e.bx, e.by,
                                                       e.obst_off, e.E, e.M, partial, gx, O);
  }
  return hipGetLastError();
}

// ------------------------------------------------------------------ validation

__global__ void validate_init_kernel(int* __restrict__ result, int M) {
  result[0] = 0;
  result[1] = M;
}

// One thread per obstacle: its offsets, then (valid range only) its edges.
__global__ void validate_kernel(const float* __restrict__ ax, const float* __restrict__ ay,
                                const float* __restrict__ bx, const float* __restrict__ by,
                                const int* __restrict__ off, int E, int M, int mbar,
                                int* __restrict__ result) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= M) return;
  const int a = off[i], b = off[i + 1];
  bool bad = b < a || b - a > mbar || a < 0 || b > E;
  for (int j = a; !bad && j < b; ++j)
    bad = !(isfinite(ax[j]) && isfinite(ay[j]) && isfinite(bx[j]) && isfinite(by[j]));
  if (bad) {
    atomicAdd(&result[0], 1);
    atomicMin(&result[1], i);
  }
}

// ------------------------------------------------------------------ EncodeEdges

__global__ void encode_count_kernel(const uint8_t* __restrict__ S, int Mbar, int mbar,
                                    int* __restrict__ cnt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= Mbar) return;
  int c = 0;
  for (int j = 0; j < mbar; ++j) c += S[(size_t)i * mbar + j] != 0;
  cnt[i] = c;
}

// Exclusive scan of cnt[0..n) into off[0..n] by one work-group of 1024 lanes.
__global__ __launch_bounds__(1024) void encode_scan_kernel(const int* __restrict__ cnt, int n,
                                                            int* __restrict__ off) {
  __shared__ int part[1024];
  const int t = threadIdx.x;
  const int chunk = (n + 1023) / 1024;
  const int lo = min(n, t * chunk), hi = min(n, lo + chunk);
  int sum = 0;
  for (int i = lo; i < hi; ++i) sum += cnt[i];
  part[t] = sum;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    const int v = t >= o ? part[t - o] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int run = part[t] - sum;
  for (int i = lo; i < hi; ++i) { off[i] = run; run += cnt[i]; }
  if (t == 1023) off[n] = part[1023];
}

__global__ void encode_scatter_kernel(const float* __restrict__ A, const float* __restrict__ B,
                                      const uint8_t* __restrict__ S, int Mbar, int mbar,
                                      const int* __restrict__ off, float* __restrict__ ax,
                                      float* __restrict__ ay, float* __restrict__ bx,
                                      float* __restrict__ by) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= Mbar) return;
  int w = off[i];
  for (int j = 0; j < mbar; ++j) {
    const size_t r = (size_t)i * mbar + j;
    if (S[r]) {
      ax[w] = A[2 * r]; ay[w] = A[2 * r + 1];
      bx[w] = B[2 * r]; by[w] = B[2 * r + 1];
      ++w;
    }
  }
}

}  // namespace psdf

// ------------------------------------------------------------------ C ABI

using namespace psdf;

extern "C" {

const char* psdf_last_error(void) { return last_error(); }

const char* psdf_version(void) { return "psdf-gfx950 0.1"; }

// A staged table attached to the edge set must have been made for it (same
// E, M and edge class) with the call's eps, and be large enough.
static int check_staged(const psdf_edges& e, const FpConst& F) {
  const psdf_staged* s = e.staged;
  if (!s) return PSDF_OK;
  const int cls = obst_class(e.mbar);
  if (s->E != e.E || s->M != e.M || s->mi_class != cls)
    return set_error(PSDF_EINVAL,
                     "staged table made for E = %d, M = %d, edge class %d; the edge set has "
                     "E = %d, M = %d, edge class %d",
                     s->E, s->M, s->mi_class, e.E, e.M, cls);
  const void* src[5] = {e.ax, e.ay, e.bx, e.by, e.obst_off};
  for (int k = 0; k < 5; ++k)
    if (s->src[k] != src[k])
      return set_error(PSDF_EINVAL,
                       "staged table made from other edge arrays (stage this edge set again)");
  if (__builtin_memcmp(&s->eps, &F.eps, sizeof(float)) != 0)
    return set_error(PSDF_EINVAL, "staged table made with eps = %g, the call has eps = %g",
                     (double)s->eps, (double)F.eps);
  if (e.M > 0) {
    if (!s->table) return set_error(PSDF_EINVAL, "staged table pointer is NULL");
    if ((reinterpret_cast<uintptr_t>(s->table) & 15u) != 0)
      return set_error(PSDF_EINVAL, "staged table is not 16-byte aligned");
    if (s->bytes < staged_table_bytes(e.M, cls))
      return set_error(PSDF_EINVAL, "staged table of %zu bytes, %zu needed", s->bytes,
                       staged_table_bytes(e.M, cls));
  }
  return PSDF_OK;
}

static int plain_common(const float* footprint, int32_t m, const float* poses, int32_t N,
                        const psdf_edges* edges, const psdf_params* params, FpConst& F,
                        psdf_edges& e) {
  int rc = prepare_footprint(footprint, m, params, &F);
  if (rc) return rc;
  rc = check_edges(edges, &e);
  if (rc) return rc;
  rc = check_staged(e, F);
  if (rc) return rc;
  if (N < 0) return set_error(PSDF_EINVAL, "N = %d is negative", N);
  if (N > 0 && !poses) return set_error(PSDF_EINVAL, "poses is NULL");
  return PSDF_OK;
}

size_t psdf_staged_bytes(int32_t M, int32_t mbar) {
  if (M <= 0 || M > kStagedMaxM || mbar < 1 || mbar > kMaxObst) return 0;
  return staged_table_bytes(M, obst_class(mbar));
}

int psdf_stage_edges(const psdf_edges* edges, const psdf_params* params, void* table,
                     size_t table_bytes, psdf_staged* out, hipStream_t stream) {
  clear_error();
  psdf_edges e;
  int rc = check_edges(edges, &e);
  if (rc) return rc;
  if (!out) return set_error(PSDF_EINVAL, "out is NULL");
  const float eps = params ? params->eps : 1e-12f;
  if (!(eps >= 0.f)) return set_error(PSDF_EINVAL, "eps must be >= 0");
  const int cls = obst_class(e.mbar);
  if (e.M > kStagedMaxM)
    return set_error(PSDF_ETOOBIG, "M = %d obstacles, at most %d can be staged", e.M, kStagedMaxM);
  const size_t need = psdf_staged_bytes(e.M, e.mbar);
  if (need > 0) {
    if (!table) return set_error(PSDF_EINVAL, "table is NULL");
    if ((reinterpret_cast<uintptr_t>(table) & 15u) != 0)
      return set_error(PSDF_EINVAL, "table is not 16-byte aligned");
    if (table_bytes < need)
      return set_error(PSDF_EWS, "table of %zu bytes, %zu needed", table_bytes, need);
    const StagedView v = staged_view(table, e.M, cls);
    const int grid = (v.Mp + 255) / 256;
    if (cls == 4)
      stage_edges_kernel<4><<<grid, 256, 0, stream>>>(e.ax, e.ay, e.bx, e.by, e.obst_off, e.E,
                                                      e.M, eps, v);
    else if (cls == 8)
      stage_edges_kernel<8><<<grid, 256, 0, stream>>>(e.ax, e.ay, e.bx, e.by, e.obst_off, e.E,
                                                      e.M, eps, v);
    else
      stage_edges_kernel<16><<<grid, 256, 0, stream>>>(e.ax, e.ay, e.bx, e.by, e.obst_off, e.E,
                                                       e.M, eps, v);
    const hipError_t err = hipGetLastError();
    if (err != hipSuccess) return hip_status(err);
  }
  out->table = table;
  out->bytes = table_bytes;
  out->E = e.E;
  out->M = e.M;
  out->mi_class = cls;
  out->eps = eps;
  const void* src[5] = {e.ax, e.ay, e.bx, e.by, e.obst_off};
  for (int k = 0; k < 5; ++k) out->src[k] = src[k];
  return PSDF_OK;
}

size_t psdf_workspace_bytes(int32_t N, int32_t M) {
  if (N <= 0 || M <= 0) return 0;
  // a 16-byte (key, aux) partial per stage and work-group, at most one
  // work-group per 64 obstacles
  return 2 * (size_t)N * (size_t)((M + 63) / 64) * sizeof(uint64_t);
}

static int plain_run(const float* footprint, int32_t m, const float* poses, int32_t N,
                     const psdf_edges* edges, const psdf_params* params, float* d, int32_t* edge,
                     int32_t* obst, float* grad, uint64_t* keys, void* ws, size_t ws_bytes,
                     int mode, hipStream_t stream) {
  clear_error();
  FpConst F;
  psdf_edges e;
  int rc = plain_common(footprint, m, poses, N, edges, params, F, e);
  if (rc) return rc;
  if (N == 0) return PSDF_OK;
  if (!d || !edge || !obst || !keys || (mode == 1 && !grad))
    return set_error(PSDF_EINVAL, "an output pointer is NULL");
  const size_t need = psdf_workspace_bytes(N, e.M);
  if (need > 0 && (!ws || ws_bytes < need))
    return set_error(PSDF_EWS, "workspace of %zu bytes, %zu needed", ws_bytes, need);
  if (need > 0 && (reinterpret_cast<uintptr_t>(ws) & 15u) != 0)
    return set_error(PSDF_EINVAL, "workspace is not 16-byte aligned");
  if (small_path(e)) {
    const EpiOut O{keys, nullptr, mode, 0.0f, d, edge, obst, grad, nullptr};
    return hip_status(PSDF_BY_MF(launch_small_mf, F, poses, N, e, O, stream));
  }
  const LaunchShape ls = tuned_shape(F.m, e.mbar, N, e.M);
  uint64_t* partial = static_cast<uint64_t*>(ws);
  hipError_t err = launch_plain(F, poses, N, e, partial, ls, stream);
  if (err == hipSuccess)
    err = launch_epilogue(F, poses, N, e, partial, e.M > 0 ? partial_columns(e.M, ls) : 0, keys,
                          nullptr, mode, 0.0f, d, edge, obst, grad, nullptr, stream);
  return hip_status(err);
}

int psdf_time_stage_min(const float* footprint, int32_t m, const float* poses, int32_t N,
                        const psdf_edges* edges, const psdf_params* params, void* ws,
                        size_t ws_bytes, int32_t reps, hipStream_t stream, float* ms) {
  clear_error();
  FpConst F;
  psdf_edges e;
  int rc = plain_common(footprint, m, poses, N, edges, params, F, e);
  if (rc) return rc;
  if (!ms || reps < 1) return set_error(PSDF_EINVAL, "ms is NULL or reps < 1");
  *ms = 0.f;
  if (N == 0 || e.M == 0) return PSDF_OK;
  const size_t need = psdf_workspace_bytes(N, e.M);
  if (!ws || ws_bytes < need)
    return set_error(PSDF_EWS, "workspace of %zu bytes, %zu needed", ws_bytes, need);
  if ((reinterpret_cast<uintptr_t>(ws) & 15u) != 0)
    return set_error(PSDF_EINVAL, "workspace is not 16-byte aligned");
  if (reps > 100000) return set_error(PSDF_EINVAL, "reps = %d, at most 100000", reps);
  const LaunchShape ls = tuned_shape(F.m, e.mbar, N, e.M);
  uint64_t* partial = static_cast<uint64_t*>(ws);
  // one event pair per launch, recorded by the dispatch itself at its start
  // and end: the mean is the kernel's own duration, whatever the host's
  // enqueue rate
  std::vector<hipEvent_t> ev(2 * (size_t)reps, nullptr);
  hipError_t err = hipSuccess;
  for (size_t k = 0; k < ev.size() && err == hipSuccess; ++k) err = hipEventCreate(&ev[k]);
  for (int r = 0; r < reps && err == hipSuccess; ++r)
    err = PSDF_BY_MF(launch_main_mf, obst_class(e.mbar), ls, F, poses, N, e, partial, stream,
                     ev[2 * r], ev[2 * r + 1]);
  if (err == hipSuccess) err = hipEventSynchronize(ev.back());
  double total = 0.0;
  for (int r = 0; r < reps && err == hipSuccess; ++r) {
    float t = 0.f;
    err = hipEventElapsedTime(&t, ev[2 * r], ev[2 * r + 1]);
    total += t;
  }
  for (hipEvent_t x : ev)
    if (x) (void)hipEventDestroy(x);
  if (err == hipSuccess) *ms = (float)(total / reps);
  return hip_status(err);
}

int psdf_eval(const float* footprint, int32_t m, const float* poses, int32_t N,
              const psdf_edges* edges, const psdf_params* params, float* d, int32_t* edge,
              int32_t* obst, uint64_t* keys, void* ws, size_t ws_bytes, hipStream_t stream) {
  return plain_run(footprint, m, poses, N, edges, params, d, edge, obst, nullptr, keys, ws,
                   ws_bytes, 0, stream);
}

int psdf_grad(const float* footprint, int32_t m, const float* poses, int32_t N,
              const psdf_edges* edges, const psdf_params* params, float* d, int32_t* edge,
              int32_t* obst, float* grad, uint64_t* keys, void* ws, size_t ws_bytes,
              hipStream_t stream) {
  return plain_run(footprint, m, poses, N, edges, params, d, edge, obst, grad, keys, ws,
                   ws_bytes, 1, stream);
}

// ------------------------------------------------------------------ no-alloc form

// Library-owned scratch of psdf_grad_noalloc: one copy per GPU, held until
// the process ends.  In host code the name is only a stand-in for the
// symbol; the device address comes from hipGetSymbolAddress, taken once per
// device (with that device current) on the entry point's first call there.
static __device__ __align__(256) uint8_t scratch[PSDF_NOALLOC_WS_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

int scratch_for_current_device(void** out) {
  int dev = -1;
  hipError_t err = hipGetDevice(&dev);
  if (err != hipSuccess) return hip_status(err);
  if (dev < 0 || dev >= kMaxDevices)
    return set_error(PSDF_EINVAL, "device %d: at most %d devices", dev, kMaxDevices);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    err = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (err != hipSuccess) return hip_status(err);
    if (!ptr) return set_error(PSDF_EHIP, "no device address for the scratch buffer");
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return PSDF_OK;
}
}  // namespace

int psdf_grad_noalloc(const float* footprint, int32_t m, const float* poses, int32_t N,
                      const psdf_edges* edges, const psdf_params* params, float* d,
                      int32_t* edge, int32_t* obst, float* grad, uint64_t* keys,
                      hipStream_t stream) {
  clear_error();
  FpConst F;
  psdf_edges e;
  int rc = plain_common(footprint, m, poses, N, edges, params, F, e);
  if (rc) return rc;
  if (N == 0) return PSDF_OK;
  const size_t need = psdf_workspace_bytes(N, e.M);
  if (need > PSDF_NOALLOC_WS_BYTES)
    return set_error(PSDF_ETOOBIG,
                     "N = %d stages and M = %d obstacles need %zu bytes of scratch; the "
                     "no-alloc form holds %zu",
                     N, e.M, need, (size_t)PSDF_NOALLOC_WS_BYTES);
  void* ws = nullptr;
  if (need > 0) {
    rc = scratch_for_current_device(&ws);
    if (rc) return rc;
  }
  // every partial the kernels read is written by the same call, so the
  // buffer needs no clearing between calls
  return plain_run(footprint, m, poses, N, edges, params, d, edge, obst, grad, keys, ws, need, 1,
                   stream);
}

int psdf_constraints(const float* footprint, int32_t m, const float* poses, int32_t N,
                     const psdf_edges* edges, const psdf_params* params, float d_min, float* hj,
                     float* hj_host, uint64_t* keys, void* ws, size_t ws_bytes,
                     hipStream_t stream) {
  clear_error();
  FpConst F;
  psdf_edges e;
  int rc = plain_common(footprint, m, poses, N, edges, params, F, e);
  if (rc) return rc;
  if (N == 0) return PSDF_OK;
  if (!hj || !keys) return set_error(PSDF_EINVAL, "hj or keys is NULL");
  if (!std::isfinite(d_min)) return set_error(PSDF_EINVAL, "d_min is not finite");
  const size_t need = psdf_workspace_bytes(N, e.M);
  if (need > 0 && (!ws || ws_bytes < need))
    return set_error(PSDF_EWS, "workspace of %zu bytes, %zu needed", ws_bytes, need);
  if (need > 0 && (reinterpret_cast<uintptr_t>(ws) & 15u) != 0)
    return set_error(PSDF_EINVAL, "workspace is not 16-byte aligned");
  hipError_t err = hipSuccess;
  if (small_path(e)) {
    const EpiOut O{keys, nullptr, 1, d_min, nullptr, nullptr, nullptr, nullptr, hj};
    err = PSDF_BY_MF(launch_small_mf, F, poses, N, e, O, stream);
  } else {
    const LaunchShape ls = tuned_shape(F.m, e.mbar, N, e.M);
    uint64_t* partial = static_cast<uint64_t*>(ws);
    err = launch_plain(F, poses, N, e, partial, ls, stream);
    if (err == hipSuccess)
      err = launch_epilogue(F, poses, N, e, partial, e.M > 0 ? partial_columns(e.M, ls) : 0, keys,
                            nullptr, 1, d_min, nullptr, nullptr, nullptr, nullptr, hj, stream);
  }
  if (err == hipSuccess && hj_host)
    err = hipMemcpyAsync(hj_host, hj, (size_t)N * 4 * sizeof(float), hipMemcpyDeviceToHost, stream);
  return hip_status(err);
}

int psdf_bwd(const float* footprint, int32_t m, const float* poses, int32_t N,
             const psdf_edges* edges, const psdf_params* params, const uint64_t* keys,
             const float* gout, float* gpose, hipStream_t stream) {
  clear_error();
  FpConst F;
  psdf_edges e;
  int rc = plain_common(footprint, m, poses, N, edges, params, F, e);
  if (rc) return rc;
  if (N == 0) return PSDF_OK;
  if (!keys || !gout || !gpose) return set_error(PSDF_EINVAL, "keys, gout or gpose is NULL");
  return hip_status(launch_epilogue(F, poses, N, e, nullptr, 0, const_cast<uint64_t*>(keys), gout,
                                    2, 0.0f, nullptr, nullptr, nullptr, gpose, nullptr, stream));
}

int psdf_sd_matrix(const float* footprint, int32_t m, const float* poses, int32_t N,
                   const psdf_edges* edges, const psdf_params* params, float* sd,
                   hipStream_t stream) {
  clear_error();
  FpConst F;
  psdf_edges e;
  int rc = plain_common(footprint, m, poses, N, edges, params, F, e);
  if (rc) return rc;
  if (N == 0 || e.M == 0) return PSDF_OK;
  if (!sd) return set_error(PSDF_EINVAL, "sd is NULL");
  if ((N + kSdmatStageBlock - 1) / kSdmatStageBlock > 65535)
    return set_error(PSDF_ETOOBIG, "N = %d; at most %d stages", N, 65535 * kSdmatStageBlock);
  return hip_status(PSDF_BY_MF(launch_sdmat_mf, obst_class(e.mbar), F, poses, N, e, sd, stream));
}

size_t psdf_encode_ws_bytes(int32_t Mbar) { return Mbar > 0 ? (size_t)Mbar * sizeof(int) : 0; }

int psdf_validate_edges(const psdf_edges* edges, int32_t* result, hipStream_t stream) {
  clear_error();
  psdf_edges e;
  const int rc = check_edges(edges, &e);
  if (rc) return rc;
  if (!result) return set_error(PSDF_EINVAL, "result is NULL");
  validate_init_kernel<<<1, 1, 0, stream>>>(result, e.M);
  hipError_t err = hipGetLastError();
  if (err == hipSuccess && e.M > 0) {
    validate_kernel<<<(e.M + 255) / 256, 256, 0, stream>>>(e.ax, e.ay, e.bx, e.by, e.obst_off, e.E,
                                                           e.M, e.mbar, result);
    err = hipGetLastError();
  }
  return hip_status(err);
}

int psdf_encode_padded(const float* A, const float* B, const uint8_t* S, int32_t Mbar,
                       int32_t mbar, float* ax, float* ay, float* bx, float* by,
                       int32_t* obst_off, void* ws, size_t ws_bytes, hipStream_t stream) {
  clear_error();
  if (Mbar < 0 || mbar < 0) return set_error(PSDF_EINVAL, "negative padded size");
  if (!obst_off) return set_error(PSDF_EINVAL, "obst_off is NULL");
  if (Mbar == 0) {
    encode_scan_kernel<<<1, 1024, 0, stream>>>(nullptr, 0, obst_off);
    return hip_status(hipGetLastError());
  }
  if (!A || !B || !S || !ax || !ay || !bx || !by || !ws)
    return set_error(PSDF_EINVAL, "a padded input, CSR output or workspace pointer is NULL");
  if (ws_bytes < psdf_encode_ws_bytes(Mbar))
    return set_error(PSDF_EWS, "workspace of %zu bytes, %zu needed", ws_bytes,
                     psdf_encode_ws_bytes(Mbar));
  int* cnt = static_cast<int*>(ws);
  const int g = (Mbar + 255) / 256;
  encode_count_kernel<<<g, 256, 0, stream>>>(S, Mbar, mbar, cnt);
  encode_scan_kernel<<<1, 1024, 0, stream>>>(cnt, Mbar, obst_off);
  encode_scatter_kernel<<<g, 256, 0, stream>>>(A, B, S, Mbar, mbar, obst_off, ax, ay, bx, by);
  return hip_status(hipGetLastError());
}

}  // extern "C"
