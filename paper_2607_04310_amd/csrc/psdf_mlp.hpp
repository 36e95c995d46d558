// Edge-screener MLP on the matrix cores (gfx950 MFMA, BF16 operands, FP32
// accumulation).  Network 4 -> 64 -> 64 -> 1 with ReLU; parameters in one
// FP32 vector: W1[64][4], b1[64], W2[64][64], b2[64], w3[64], b3.
//
// A wave evaluates 16 (stage, edge) pairs at a time in the transposed form
// (hidden units x pairs), so that each layer's output fragment, after bias,
// ReLU and rounding to BF16, is directly the next layer's B operand:
//   layer 1: H1^T = W1 X^T      v_mfma_f32_16x16x16_bf16, K = 4 features padded to 16
//   layer 2: H2^T = W2 H1^T     v_mfma_f32_16x16x32_bf16, K = 64 in two blocks
//   layer 3: y = w3 . relu(H2^T + b2) + b3   FP32 on the vector units
// Fragment layouts (lane l, g = l / 16, n = l % 16):
//   16x16x16: A[i = n][k = 4g + r], B[k = 4g + r][j = n], D[i = 4g + r][j = n]
//   16x16x32: A[i = n][k = 8g + r], B[k = 8g + r][j = n], D as above
// A D fragment holds units 16 mb + 4g + r of pair n; a layer-2 K block kb
// therefore uses the permuted unit order u(kb, g, r) = 32 kb + 4g + r
// (r < 4) or 32 kb + 16 + 4g + (r - 4) (r >= 4) in both operands, which
// leaves the sum unchanged.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace psdf {

constexpr int kH = 64;
constexpr int kIn = 4;
constexpr int kMlpParams = kH * kIn + kH + kH * kH + kH + kH + 1;   // 4545
constexpr int kOffW1 = 0, kOffB1 = kH * kIn, kOffW2 = kOffB1 + kH, kOffB2 = kOffW2 + kH * kH;
constexpr int kOffW3 = kOffB2 + kH, kOffB3 = kOffW3 + kH;
constexpr float kFeatureScale = 4.0f;   // features: robot-frame endpoints / 4 m

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef short bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// Round to BF16, nearest-even (finite inputs): the hardware conversion
// (v_cvt_pk_bf16_f32, two values per instruction).
__device__ __forceinline__ short to_bf16(float f) { return __builtin_bit_cast(short, (__bf16)f); }

__device__ __forceinline__ int perm_unit(int kb, int g, int r) {
  return 32 * kb + (r < 4 ? 4 * g + r : 16 + 4 * g + (r - 4));
}

// Loop-invariant weight fragments of one wave.
struct MlpFrag {
  bf16x4 a1[4];        // W1 blocks (units 16 mb + n, features 4g + r; zero for g > 0)
  bf16x8 a2[4][2];     // W2 blocks (rows 16 mb2 + n, permuted K)
  float b1[4][4];      // b1[16 mb + 4g + r]
  float b2[4][4];      // b2[16 mb2 + 4g + r]
  float w3[4][4];      // w3[16 mb2 + 4g + r]
  float b3;
};

__device__ __forceinline__ void mlp_load(const float* __restrict__ th, MlpFrag& f) {
  const int l = threadIdx.x & 63, g = l >> 4, n = l & 15;
#pragma unroll
  for (int mb = 0; mb < 4; ++mb) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int unit = 16 * mb + n;
      f.a1[mb][r] = g == 0 ? to_bf16(th[kOffW1 + unit * kIn + r]) : (short)0;
      f.b1[mb][r] = th[kOffB1 + 16 * mb + 4 * g + r];
      f.b2[mb][r] = th[kOffB2 + 16 * mb + 4 * g + r];
      f.w3[mb][r] = th[kOffW3 + 16 * mb + 4 * g + r];
    }
#pragma unroll
    for (int kb = 0; kb < 2; ++kb)
#pragma unroll
      for (int r = 0; r < 8; ++r)
        f.a2[mb][kb][r] = to_bf16(th[kOffW2 + (16 * mb + n) * kH + perm_unit(kb, g, r)]);
  }
  f.b3 = th[kOffB3];
}

// The fragments of all 64 lanes as a table of kFragWords 16-byte words per
// lane, word k of lane l at [k * 64 + l] (coalesced across the wave): built
// once per call by the horizon pass (its extra grid column), read with
// kFragWords vector loads.
constexpr int kFragWords = (sizeof(MlpFrag) + 15) / 16;

__device__ __forceinline__ void mlp_frag_store(const MlpFrag& f, uint4* __restrict__ table) {
  const int l = threadIdx.x & 63;
  uint4 w[kFragWords] = {};
  __builtin_memcpy(w, &f, sizeof(MlpFrag));
#pragma unroll
  for (int k = 0; k < kFragWords; ++k) table[k * 64 + l] = w[k];
}

__device__ __forceinline__ void mlp_frag_fetch(const uint4* __restrict__ table, MlpFrag& f) {
  const int l = threadIdx.x & 63;
  uint4 w[kFragWords];
#pragma unroll
  for (int k = 0; k < kFragWords; ++k) w[k] = table[k * 64 + l];
  __builtin_memcpy(&f, w, sizeof(MlpFrag));
}

// Forward intermediates of one 16-pair group (lane l: pair n = l % 16).
struct MlpAct {
  f32x4 h1pre[4];   // H1^T pre-activation, units 16 mb + 4g + r
  bf16x8 b2op[2];   // relu(H1^T) in BF16, layer-2 B operand per K block
  f32x4 h2pre[4];   // H2^T pre-activation (bias included)
  float y;          // output of pair n (all four lane groups agree)
};

// bx: the BF16 features of pair n in lanes g == 0, zero in the other lanes.
__device__ __forceinline__ void mlp_forward16_bf(const MlpFrag& f, bf16x4 bx, MlpAct& a) {
  short h1b[4][4];
#pragma unroll
  for (int mb = 0; mb < 4; ++mb) {
    f32x4 z = {0.f, 0.f, 0.f, 0.f};
    f32x4 d = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(f.a1[mb], bx, z, 0, 0, 0);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      d[r] += f.b1[mb][r];
      h1b[mb][r] = to_bf16(fmaxf(d[r], 0.f));
    }
    a.h1pre[mb] = d;
  }
#pragma unroll
  for (int kb = 0; kb < 2; ++kb)
#pragma unroll
    for (int r = 0; r < 8; ++r) a.b2op[kb][r] = r < 4 ? h1b[2 * kb][r] : h1b[2 * kb + 1][r - 4];
  float part = 0.f;
#pragma unroll
  for (int mb = 0; mb < 4; ++mb) {
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(f.a2[mb][0], a.b2op[0], acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(f.a2[mb][1], a.b2op[1], acc, 0, 0, 0);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      acc[r] += f.b2[mb][r];
      part = fmaf(f.w3[mb][r], fmaxf(acc[r], 0.f), part);
    }
    a.h2pre[mb] = acc;
  }
  part += __shfl_xor(part, 16);
  part += __shfl_xor(part, 32);
  a.y = part + f.b3;
}

// BF16 image of pair features x0..x3, as the network reads them.
__device__ __forceinline__ bf16x4 mlp_features(float x0, float x1, float x2, float x3) {
  bf16x4 bx;
  bx[0] = to_bf16(x0);
  bx[1] = to_bf16(x1);
  bx[2] = to_bf16(x2);
  bx[3] = to_bf16(x3);
  return bx;
}

// x0..x3: the features of pair n (read by lanes g == 0 only).
__device__ __forceinline__ void mlp_forward16(const MlpFrag& f, float x0, float x1, float x2,
                                              float x3, MlpAct& a) {
  const int g = (threadIdx.x & 63) >> 4;
  const bf16x4 zero = {0, 0, 0, 0};
  mlp_forward16_bf(f, g == 0 ? mlp_features(x0, x1, x2, x3) : zero, a);
}

}  // namespace psdf
