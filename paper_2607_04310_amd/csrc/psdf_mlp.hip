// Screener MLP kernels: inference on feature rows, the training step
// (forward, backward, deterministic gradient reduction, Adam) and the label
// generator (features and exact per-edge pool distances of sampled
// (stage, edge) pairs).
#include <hip/hip_runtime.h>

#include <cmath>

#include "psdf.h"
#include "psdf_batch.hpp"
#include "psdf_host.hpp"
#include "psdf_mlp.hpp"

namespace psdf {

constexpr int kMlpWaves = 4;          // waves per work-group
constexpr int kGradRow = kMlpParams + 1;   // per-wave partial gradient row (+ loss)

// y[i] for feature rows X[i][0..3], one wave per 16-row group.
__global__ __launch_bounds__(64 * kMlpWaves) void mlp_forward_kernel(const float* __restrict__ th,
                                                                      const float* __restrict__ X,
                                                                      int B, float* __restrict__ y) {
  MlpFrag f;
  mlp_load(th, f);
  const int lane = threadIdx.x & 63, n = lane & 15, g = lane >> 4;
  const int wave = blockIdx.x * kMlpWaves + (threadIdx.x >> 6);
  const int stride = gridDim.x * kMlpWaves;
  for (int grp = wave; grp * 16 < B; grp += stride) {
    const int i = grp * 16 + n;
    float x0 = 0.f, x1 = 0.f, x2 = 0.f, x3 = 0.f;
    if (i < B) { x0 = X[4 * i]; x1 = X[4 * i + 1]; x2 = X[4 * i + 2]; x3 = X[4 * i + 3]; }
    MlpAct a;
    mlp_forward16(f, x0, x1, x2, x3, a);
    if (g == 0 && i < B) y[i] = a.y;
  }
}

// Forward + backward of the mean squared error over B rows; each wave
// handles `gpw` groups of 16 rows and writes its partial gradient (and
// partial sum of squared errors) to row `wave` of part[][kGradRow].
__global__ __launch_bounds__(64 * kMlpWaves) void mlp_grad_kernel(const float* __restrict__ th,
                                                                   const float* __restrict__ X,
                                                                   const float* __restrict__ T,
                                                                   int B, int gpw,
                                                                   float* __restrict__ part) {
  __shared__ short lh1[kMlpWaves][16][kH];
  __shared__ short ldh2[kMlpWaves][16][kH];
  __shared__ short ldh1[kMlpWaves][16][kH];
  __shared__ short lx[kMlpWaves][16][kIn];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, n = lane & 15, g = lane >> 4;
  const int wave = blockIdx.x * kMlpWaves + w;
  MlpFrag f;
  mlp_load(th, f);
  // W2^T fragments: A[i = unit u1 = 16 mb1 + n][k = permuted u2]
  bf16x8 a2t[4][2];
#pragma unroll
  for (int mb = 0; mb < 4; ++mb)
#pragma unroll
    for (int kb = 0; kb < 2; ++kb)
#pragma unroll
      for (int r = 0; r < 8; ++r)
        a2t[mb][kb][r] = to_bf16(th[kOffW2 + perm_unit(kb, g, r) * kH + 16 * mb + n]);

  f32x4 gW2[4][4], gW1[4];
  float gb1[4][4], gb2[4][4], gw3[4][4], gb3 = 0.f, sse = 0.f;
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    gW1[a] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      gW2[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
      gb1[a][b] = gb2[a][b] = gw3[a][b] = 0.f;
    }
  }
  const float inv_b = 2.0f / (float)B;
  for (int q = 0; q < gpw; ++q) {
    const int i = (wave * gpw + q) * 16 + n;
    const bool valid = i < B;
    float x0 = 0.f, x1 = 0.f, x2 = 0.f, x3 = 0.f, t = 0.f;
    if (valid) { x0 = X[4 * i]; x1 = X[4 * i + 1]; x2 = X[4 * i + 2]; x3 = X[4 * i + 3]; t = T[i]; }
    MlpAct a;
    mlp_forward16(f, x0, x1, x2, x3, a);
    const float err = valid ? a.y - t : 0.f;
    const float dy = err * inv_b;
    if (g == 0) { sse += err * err; gb3 += dy; }
    // layer 3 and the output gradient of layer 2
    short dh2b[4][4];
#pragma unroll
    for (int mb = 0; mb < 4; ++mb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const float pre = a.h2pre[mb][r];
        gw3[mb][r] = fmaf(dy, fmaxf(pre, 0.f), gw3[mb][r]);
        const float dh = pre > 0.f ? dy * f.w3[mb][r] : 0.f;
        gb2[mb][r] += dh;
        dh2b[mb][r] = to_bf16(dh);
      }
    bf16x8 bop[2];
#pragma unroll
    for (int kb = 0; kb < 2; ++kb)
#pragma unroll
      for (int r = 0; r < 8; ++r) bop[kb][r] = r < 4 ? dh2b[2 * kb][r] : dh2b[2 * kb + 1][r - 4];
    // dh1 = (W2^T dh2) * [h1pre > 0]
    short dh1b[4][4];
#pragma unroll
    for (int mb = 0; mb < 4; ++mb) {
      f32x4 acc = {0.f, 0.f, 0.f, 0.f};
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a2t[mb][0], bop[0], acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a2t[mb][1], bop[1], acc, 0, 0, 0);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const float dh = a.h1pre[mb][r] > 0.f ? acc[r] : 0.f;
        gb1[mb][r] += dh;
        dh1b[mb][r] = to_bf16(dh);
      }
    }
    // transpose h1, dh2, dh1 (units x rows -> rows x units) through LDS
#pragma unroll
    for (int mb = 0; mb < 4; ++mb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int u = 16 * mb + 4 * g + r;
        lh1[w][n][u] = r < 4 ? a.b2op[mb >> 1][(mb & 1) * 4 + r] : 0;
        ldh2[w][n][u] = dh2b[mb][r];
        ldh1[w][n][u] = dh1b[mb][r];
      }
    if (g == 0) {
      lx[w][n][0] = to_bf16(x0); lx[w][n][1] = to_bf16(x1);
      lx[w][n][2] = to_bf16(x2); lx[w][n][3] = to_bf16(x3);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // dW2[u2][u1] += sum_rows dh2[u2][row] h1[u1][row]   (K = 16 rows)
#pragma unroll
    for (int m2 = 0; m2 < 4; ++m2) {
      bf16x4 A;
#pragma unroll
      for (int r = 0; r < 4; ++r) A[r] = ldh2[w][4 * g + r][16 * m2 + n];
#pragma unroll
      for (int m1 = 0; m1 < 4; ++m1) {
        bf16x4 Bv;
#pragma unroll
        for (int r = 0; r < 4; ++r) Bv[r] = lh1[w][4 * g + r][16 * m1 + n];
        gW2[m2][m1] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A, Bv, gW2[m2][m1], 0, 0, 0);
      }
    }
    // dW1[u1][k] += sum_rows dh1[u1][row] x[row][k]   (k < 4 of 16 columns)
    bf16x4 Bx;
#pragma unroll
    for (int r = 0; r < 4; ++r) Bx[r] = n < kIn ? lx[w][4 * g + r][n < kIn ? n : 0] : (short)0;
#pragma unroll
    for (int mb = 0; mb < 4; ++mb) {
      bf16x4 A;
#pragma unroll
      for (int r = 0; r < 4; ++r) A[r] = ldh1[w][4 * g + r][16 * mb + n];
      gW1[mb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A, Bx, gW1[mb], 0, 0, 0);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
  // ---- write this wave's partial gradient
  float* row = part + (size_t)wave * kGradRow;
#pragma unroll
  for (int m2 = 0; m2 < 4; ++m2)
#pragma unroll
    for (int m1 = 0; m1 < 4; ++m1)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        row[kOffW2 + (16 * m2 + 4 * g + r) * kH + 16 * m1 + n] = gW2[m2][m1][r];
  if (n < kIn) {
#pragma unroll
    for (int mb = 0; mb < 4; ++mb)
#pragma unroll
      for (int r = 0; r < 4; ++r) row[kOffW1 + (16 * mb + 4 * g + r) * kIn + n] = gW1[mb][r];
  }
  // biases and w3: sum over the 16 rows held by lanes of one group g
#pragma unroll
  for (int mb = 0; mb < 4; ++mb)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      float v1 = gb1[mb][r], v2 = gb2[mb][r], v3 = gw3[mb][r];
#pragma unroll
      for (int o = 1; o < 16; o <<= 1) {
        v1 += __shfl_xor(v1, o);
        v2 += __shfl_xor(v2, o);
        v3 += __shfl_xor(v3, o);
      }
      if (n == 0) {
        const int u = 16 * mb + 4 * g + r;
        row[kOffB1 + u] = v1;
        row[kOffB2 + u] = v2;
        row[kOffW3 + u] = v3;
      }
    }
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    gb3 += __shfl_xor(gb3, o);
    sse += __shfl_xor(sse, o);
  }
  if (lane == 0) {
    row[kOffB3] = gb3;
    row[kMlpParams] = sse;
  }
}

// Sum the per-wave partial rows into grad[kGradRow]; with lr > 0 also apply
// one Adam step to theta (m, v moments; step counts from 1).
// grad[kMlpParams] receives the mean squared error.  A work-group owns 64
// consecutive columns; wave q adds rows q, q + 4, q + 8, ... in that order
// (four rows in flight per lane) and wave 0 adds the four wave sums in wave
// order, so the result does not depend on timing.
constexpr int kReduceWaves = 4;
__global__ __launch_bounds__(64 * kReduceWaves) void mlp_reduce_adam_kernel(
    float* __restrict__ th, float* __restrict__ m, float* __restrict__ v,
    const float* __restrict__ part, int waves, int B, int step, float lr,
    float* __restrict__ grad, float* __restrict__ loss) {
  __shared__ float red[kReduceWaves][64];
  const int lane = threadIdx.x & 63, q = threadIdx.x >> 6;
  const int p = blockIdx.x * 64 + lane;
  float s = 0.f;
  if (p < kGradRow) {
    const float* col = part + p;
    constexpr int R = kReduceWaves;
    int k = q;
    for (; k + 3 * R < waves; k += 4 * R) {
      const float a0 = col[(size_t)k * kGradRow], a1 = col[(size_t)(k + R) * kGradRow];
      const float a2 = col[(size_t)(k + 2 * R) * kGradRow], a3 = col[(size_t)(k + 3 * R) * kGradRow];
      s += a0; s += a1; s += a2; s += a3;
    }
    for (; k < waves; k += R) s += col[(size_t)k * kGradRow];
  }
  red[q][lane] = s;
  __syncthreads();
  if (q != 0 || p >= kGradRow) return;
  s = red[0][lane];
#pragma unroll
  for (int w = 1; w < kReduceWaves; ++w) s += red[w][lane];
  if (p == kMlpParams) {
    if (grad) grad[p] = s / (float)B;
    if (loss) *loss = s / (float)B;
    return;
  }
  if (grad) grad[p] = s;
  if (lr > 0.f) {
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float mm = b1 * m[p] + (1.f - b1) * s;
    const float vv = b2 * v[p] + (1.f - b2) * s * s;
    m[p] = mm;
    v[p] = vv;
    const float mh = mm / (1.f - powf(b1, (float)step));
    const float vh = vv / (1.f - powf(b2, (float)step));
    th[p] -= lr * mh / (sqrtf(vh) + eps);
  }
}

// Features and labels of sampled (stage, edge) pairs: X[i] = the edge's
// robot-frame endpoints / feature scale; t[i] = the edge's pool distance,
// the minimum over the robot vertices to the edge and over its endpoints to
// the robot edges (Sec. IV-B), clipped to [0, 5] m.
__global__ void screen_label_kernel(const FpConst* __restrict__ fps,
                                    const BatchInst* __restrict__ insts,
                                    const int* __restrict__ stage_inst,
                                    const float* __restrict__ poses, const float* __restrict__ ax,
                                    const float* __restrict__ ay, const float* __restrict__ bx,
                                    const float* __restrict__ by, const int* __restrict__ stage,
                                    const int* __restrict__ edge, int n, int S,
                                    float* __restrict__ X, float* __restrict__ T) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int s = stage[i];
  float f0 = NAN, f1 = NAN, f2 = NAN, f3 = NAN, lab = NAN;
  if (s >= 0 && s < S) {
    const int inst = stage_inst[s];
    const BatchInst in = insts[inst];
    const FpConst& F = fps[inst];
    const int j = edge[i];
    if (j >= 0 && j < in.E) {
      const int ge = in.edge_off + j;
      const float* p = poses + 3 * s;
      float sn, cs;
      sincosf(p[2], &sn, &cs);
      float lax, lay, vx, vy;
      local_point(ax[ge], ay[ge], cs, sn, p[0], p[1], lax, lay);
      local_vector(bx[ge] - ax[ge], by[ge] - ay[ge], cs, sn, vx, vy);
      float iv2, il;
      edge_consts(bx[ge] - ax[ge], by[ge] - ay[ge], F.eps, iv2, il);
      const float lbx = lax + vx, lby = lay + vy;
      float d2 = __builtin_huge_valf();
      for (int l = 0; l < F.m; ++l) {
        float vlx = 0.f, vly = 0.f, elx = 0.f, ely = 0.f, ei = 0.f;
#pragma unroll
        for (int q = 0; q < kMaxFp; ++q)
          if (q == l) { vlx = F.vx[q]; vly = F.vy[q]; elx = F.ex[q]; ely = F.ey[q]; ei = F.einv[q]; }
        d2 = fminf(d2, seg_d2(vlx, vly, lax, lay, vx, vy, iv2));
        d2 = fminf(d2, seg_d2(lax, lay, vlx, vly, elx, ely, ei));
        d2 = fminf(d2, seg_d2(lbx, lby, vlx, vly, elx, ely, ei));
      }
      const float sc = 1.0f / kFeatureScale;
      f0 = lax * sc; f1 = lay * sc; f2 = lbx * sc; f3 = lby * sc;
      lab = fminf(fmaxf(sqrtf(d2), 0.f), 5.0f);
    }
  }
  X[4 * i] = f0; X[4 * i + 1] = f1; X[4 * i + 2] = f2; X[4 * i + 3] = f3;
  T[i] = lab;
}

hipError_t launch_labels(const FpConst* fps, const BatchInst* insts, const int* stage_inst,
                         const float* poses, const float* ax, const float* ay, const float* bx,
                         const float* by, const int* stage, const int* edge, int n, int S, float* X,
                         float* T, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  screen_label_kernel<<<(n + 255) / 256, 256, 0, st>>>(fps, insts, stage_inst, poses, ax, ay, bx,
                                                        by, stage, edge, n, S, X, T);
  return hipGetLastError();
}

static int grad_waves(int B) {
  const int groups = (B + 15) / 16;
  return groups < 256 ? (groups > 0 ? groups : 1) : 256;
}

}  // namespace psdf

using namespace psdf;

extern "C" {

int psdf_mlp_forward(const float* theta, const float* X, int32_t B, float* y, hipStream_t stream) {
  clear_error();
  if (B < 0) return set_error(PSDF_EINVAL, "B = %d", B);
  if (B == 0) return PSDF_OK;
  if (!theta || !X || !y) return set_error(PSDF_EINVAL, "NULL argument");
  const int groups = (B + 15) / 16;
  const int blocks = (groups + kMlpWaves - 1) / kMlpWaves;
  mlp_forward_kernel<<<blocks < 4096 ? blocks : 4096, 64 * kMlpWaves, 0, stream>>>(theta, X, B, y);
  return hip_status(hipGetLastError());
}

size_t psdf_mlp_ws_bytes(int32_t B) {
  if (B <= 0) return 0;
  const int waves = grad_waves(B);
  const int blocks = (waves + kMlpWaves - 1) / kMlpWaves;
  return (size_t)blocks * kMlpWaves * kGradRow * sizeof(float);
}

static int mlp_step(float* theta, float* m, float* v, int32_t step, float lr, const float* X,
                    const float* T, int32_t B, float* grad, float* loss, void* ws, size_t ws_bytes,
                    hipStream_t stream) {
  if (B <= 0) return set_error(PSDF_EINVAL, "B = %d", B);
  if (!theta || !X || !T) return set_error(PSDF_EINVAL, "NULL argument");
  if (!ws || ws_bytes < psdf_mlp_ws_bytes(B))
    return set_error(PSDF_EWS, "workspace of %zu bytes, %zu needed", ws_bytes, psdf_mlp_ws_bytes(B));
  const int waves = grad_waves(B);
  const int blocks = (waves + kMlpWaves - 1) / kMlpWaves;
  const int all = blocks * kMlpWaves;
  const int groups = (B + 15) / 16;
  const int gpw = (groups + all - 1) / all;
  float* part = static_cast<float*>(ws);
  mlp_grad_kernel<<<blocks, 64 * kMlpWaves, 0, stream>>>(theta, X, T, B, gpw, part);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return hip_status(err);
  mlp_reduce_adam_kernel<<<(kGradRow + 63) / 64, 64 * kReduceWaves, 0, stream>>>(
      theta, m, v, part, all, B, step, lr, grad, loss);
  return hip_status(hipGetLastError());
}

int psdf_mlp_grad(const float* theta, const float* X, const float* T, int32_t B, float* grad,
                  void* ws, size_t ws_bytes, hipStream_t stream) {
  clear_error();
  if (!grad) return set_error(PSDF_EINVAL, "grad is NULL");
  return mlp_step(const_cast<float*>(theta), nullptr, nullptr, 1, 0.f, X, T, B, grad, nullptr, ws,
                  ws_bytes, stream);
}

int psdf_mlp_train_step(float* theta, float* m, float* v, int32_t step, float lr, const float* X,
                        const float* T, int32_t B, float* loss, void* ws, size_t ws_bytes,
                        hipStream_t stream) {
  clear_error();
  if (!m || !v || step < 1 || !(lr > 0.f)) return set_error(PSDF_EINVAL, "bad Adam state");
  return mlp_step(theta, m, v, step, lr, X, T, B, nullptr, loss, ws, ws_bytes, stream);
}

}  // extern "C"
