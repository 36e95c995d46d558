// Staged edge set: the pose-independent constants of every obstacle, taken
// once when the environment changes (Alg. 1, EncodeEdges) instead of in every
// work-group of every call.
//
// For an edge class MI (4, 8 or 16 slots) and M obstacles, Mp = M rounded up
// to 64, the table holds slot-major planes so that lane <-> obstacle loads
// are coalesced (lane i reads element i of each plane):
//   rec0  float4[MI][Mp]  (A_j.x, A_j.y, u_j.x, u_j.y), u_j = (B_j - A_j) / (|B_j - A_j| + eps)
//   rec1  float4[MI][Mp]  (|B_j - A_j|, own-axis interval lo, hi, 0)     (Sec. IV-C)
//   rec2  float2[MI][Mp]  B_j (the extra points of an open obstacle)
//   meta  int4[Mp]        (first edge e0, edge count mi, closed | bad << 1, 0)
// Slot j of an obstacle is exactly the register slot j of load_obstacle +
// own_intervals (padded slots repeat edge mi - 1), computed by those same
// functions, so a kernel that reads the table evaluates bit for bit what a
// kernel that loads the edges evaluates.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>

#include "psdf_device.hpp"

namespace psdf {

struct StagedView {
  const float4* rec0;
  const float4* rec1;
  const float2* rec2;
  const int4* meta;
  int Mp;
};

// Largest M a table describes (its row count stays well inside int).
constexpr int kStagedMaxM = 1 << 28;

inline int staged_rows(int M) { return (int)(((long long)M + 63) / 64 * 64); }

// Bytes of the table, and the offsets of its planes from its start.
inline size_t staged_table_bytes(int M, int MI) {
  return (size_t)staged_rows(M) * (size_t)(40 * MI + 16);
}
inline StagedView staged_view(const void* table, int M, int MI) {
  const size_t Mp = (size_t)staged_rows(M);
  const char* b = static_cast<const char*>(table);
  StagedView v;
  v.rec0 = reinterpret_cast<const float4*>(b);
  v.rec1 = reinterpret_cast<const float4*>(b + 16 * MI * Mp);
  v.rec2 = reinterpret_cast<const float2*>(b + 32 * MI * Mp);
  v.meta = reinterpret_cast<const int4*>(b + 40 * MI * Mp);
  v.Mp = (int)Mp;
  return v;
}

// One lane per table row: obstacle i < M through load_obstacle and
// own_intervals; rows M..Mp-1 are zero (an empty obstacle).
template <int MI>
__global__ __launch_bounds__(256) void stage_edges_kernel(
    const float* __restrict__ ax, const float* __restrict__ ay, const float* __restrict__ bx,
    const float* __restrict__ by, const int* __restrict__ off, int E, int M, float eps,
    StagedView v) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= v.Mp) return;
  float4* rec0 = const_cast<float4*>(v.rec0);
  float4* rec1 = const_cast<float4*>(v.rec1);
  float2* rec2 = const_cast<float2*>(v.rec2);
  int4* meta = const_cast<int4*>(v.meta);
  const size_t Mp = (size_t)v.Mp;
  if (i >= M) {
#pragma unroll
    for (int j = 0; j < MI; ++j) {
      rec0[j * Mp + i] = make_float4(0.f, 0.f, 0.f, 0.f);
      rec1[j * Mp + i] = make_float4(0.f, 0.f, 0.f, 0.f);
      rec2[j * Mp + i] = make_float2(0.f, 0.f);
    }
    meta[i] = make_int4(0, 0, 0, 0);
    return;
  }
  const int e0 = off[i], mi = off[i + 1] - e0;
  Obst<MI> o;
  load_obstacle<MI>(o, ax, ay, bx, by, e0, mi, E, eps);
  own_intervals<MI>(o);
#pragma unroll
  for (int j = 0; j < MI; ++j) {
    rec0[j * Mp + i] = make_float4(o.ax[j], o.ay[j], o.ux[j], o.uy[j]);
    rec1[j * Mp + i] = make_float4(o.len[j], o.olo[j], o.ohi[j], 0.f);
    rec2[j * Mp + i] = make_float2(o.bx[j], o.by[j]);
  }
  meta[i] = make_int4(e0, mi, (o.closed ? 1 : 0) | (o.bad ? 2 : 0), 0);
}

// Obstacle slot registers of row i from the table (lane <-> row); the
// extra points B_j are read only for an open obstacle (a closed one never
// uses them).  r0 / r1 are the row's rec0 / rec1 entries, loaded by the
// caller ahead of time.
template <int MIX, int MI>
__device__ __forceinline__ void staged_obstacle(Obst<MIX>& o, const StagedView& v, int i,
                                                bool active, const float4 (&r0)[MI],
                                                const float4 (&r1)[MI], int mi, int flags) {
  o.mi = mi;
  o.closed = (flags & 1) != 0;
  o.bad = (flags & 2) != 0;
  o.own = true;
  const bool open = active && !o.closed;
#pragma unroll
  for (int j = 0; j < MIX; ++j) {
    o.ax[j] = r0[j].x; o.ay[j] = r0[j].y; o.ux[j] = r0[j].z; o.uy[j] = r0[j].w;
    o.len[j] = r1[j].x; o.olo[j] = r1[j].y; o.ohi[j] = r1[j].z;
    float2 b = make_float2(0.f, 0.f);
    if (open) b = v.rec2[(size_t)j * v.Mp + i];
    o.bx[j] = b.x; o.by[j] = b.y;
  }
}

// Row-major form for gathers (the screened batch, psdf_batch_stage): one row
// of 40 * MI + 16 bytes per obstacle, indexed like the horizon lists
// (circ_off + local obstacle):
//   float4 [MI]  (A_j.x, A_j.y, u_j.x, u_j.y)
//   float4 [MI]  (|B_j - A_j|, own-axis interval lo, hi, 0)
//   float2 [MI]  B_j (read only for an open obstacle)
//   int4         (local first edge a, edge count mi, closed | bad << 1, 0)
// A lane that evaluates a scattered obstacle reads its row with one round
// trip (the meta and slot loads are issued together) instead of an offset
// load followed by the edge loads, and skips the per-lane setup.
template <int MI>
constexpr int kRowBytes = 40 * MI + 16;

template <int MI>
__device__ __forceinline__ void write_row(unsigned char* __restrict__ rows, size_t r,
                                          const Obst<MI>& o, int a, int mi) {
  unsigned char* b = rows + r * kRowBytes<MI>;
  float4* A = reinterpret_cast<float4*>(b);
  float4* B = reinterpret_cast<float4*>(b + 16 * MI);
  float2* P = reinterpret_cast<float2*>(b + 32 * MI);
#pragma unroll
  for (int j = 0; j < MI; ++j) {
    A[j] = make_float4(o.ax[j], o.ay[j], o.ux[j], o.uy[j]);
    B[j] = make_float4(o.len[j], o.olo[j], o.ohi[j], 0.f);
    P[j] = make_float2(o.bx[j], o.by[j]);
  }
  *reinterpret_cast<int4*>(b + 40 * MI) = make_int4(a, mi, (o.closed ? 1 : 0) | (o.bad ? 2 : 0), 0);
}

// The obstacle of row r as the registers load_obstacle + own_intervals
// would hold (an inactive lane gets the empty obstacle); a and mi receive
// the row's local first edge and edge count.
template <int MI>
__device__ __forceinline__ void row_obstacle(Obst<MI>& o, const unsigned char* __restrict__ rows,
                                             size_t r, bool act, int& a, int& mi) {
  const unsigned char* b = rows + r * kRowBytes<MI>;
  int4 meta = make_int4(0, 0, 0, 0);
  float4 A[MI], B[MI];
#pragma unroll
  for (int j = 0; j < MI; ++j) {
    A[j] = make_float4(0.f, 0.f, 0.f, 0.f);
    B[j] = make_float4(0.f, 0.f, 0.f, 0.f);
  }
  if (act) {
    meta = *reinterpret_cast<const int4*>(b + 40 * MI);
#pragma unroll
    for (int j = 0; j < MI; ++j) {
      A[j] = reinterpret_cast<const float4*>(b)[j];
      B[j] = reinterpret_cast<const float4*>(b + 16 * MI)[j];
    }
  }
  a = meta.x;
  mi = meta.y;
  o.mi = mi;
  o.closed = (meta.z & 1) != 0;
  o.bad = (meta.z & 2) != 0;
  o.own = true;
  const bool open = act && !o.closed;
#pragma unroll
  for (int j = 0; j < MI; ++j) {
    o.ax[j] = A[j].x; o.ay[j] = A[j].y; o.ux[j] = A[j].z; o.uy[j] = A[j].w;
    o.len[j] = B[j].x; o.olo[j] = B[j].y; o.ohi[j] = B[j].z;
    float2 q = make_float2(0.f, 0.f);
    if (open) q = reinterpret_cast<const float2*>(b + 32 * MI)[j];
    o.bx[j] = q.x; o.by[j] = q.y;
  }
}

}  // namespace psdf
