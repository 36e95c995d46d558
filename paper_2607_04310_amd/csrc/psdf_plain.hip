// Plain PSDF path for gfx950: psdf_eval, psdf_grad, psdf_bwd, psdf_encode_padded.
//
// Kernel sequence of one call (all on the caller's stream, no host sync):
// init_keys_kernel (keys[s] = empty), main_kernel (per-stage minimum of
// (sd, obstacle) by 64-bit atomicMin), epilogue_kernel (winner's adjoint and
// the outputs).  The kernels live in psdf_kernels.hpp.
#include <hip/hip_runtime.h>

#include <cmath>

#include "psdf.h"
#include "psdf_kernels.hpp"

namespace psdf {

__global__ void init_keys_kernel(uint64_t* __restrict__ keys, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) keys[i] = kEmptyKey;
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

hipError_t launch_plain(const FpConst& F, const float* poses, int N, const psdf_edges& e,
                        uint64_t* keys, const LaunchShape& ls, hipStream_t st) {
  init_keys_kernel<<<(N + 255) / 256, 256, 0, st>>>(keys, N);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess || e.M == 0) return err;
  timer_begin(st);
  err = PSDF_BY_MF(launch_main_mf, obst_class(e.mbar), ls, F, poses, N, e, keys, st);
  timer_end(st);
  return err;
}

hipError_t launch_epilogue(const FpConst& F, const float* poses, int N, const psdf_edges& e,
                           const uint64_t* keys, const float* gout, int mode, float* d, int* edge,
                           int* obst, float* grad, hipStream_t st) {
  return PSDF_BY_MF(launch_epi_mf, obst_class(e.mbar), F, poses, N, e, keys, gout, mode, d, edge,
                    obst, grad, st);
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

static int plain_common(const float* footprint, int32_t m, const float* poses, int32_t N,
                        const psdf_edges* edges, const psdf_params* params, FpConst& F,
                        psdf_edges& e) {
  int rc = prepare_footprint(footprint, m, params, &F);
  if (rc) return rc;
  rc = check_edges(edges, &e);
  if (rc) return rc;
  if (N < 0) return set_error(PSDF_EINVAL, "N = %d is negative", N);
  if (N > 0 && !poses) return set_error(PSDF_EINVAL, "poses is NULL");
  return PSDF_OK;
}

int psdf_eval(const float* footprint, int32_t m, const float* poses, int32_t N,
              const psdf_edges* edges, const psdf_params* params, float* d, int32_t* edge,
              int32_t* obst, uint64_t* keys, hipStream_t stream) {
  clear_error();
  FpConst F;
  psdf_edges e;
  int rc = plain_common(footprint, m, poses, N, edges, params, F, e);
  if (rc) return rc;
  if (N == 0) return PSDF_OK;
  if (!d || !edge || !obst || !keys) return set_error(PSDF_EINVAL, "an output pointer is NULL");
  LaunchShape ls = choose_shape(N, e.M);
  hipError_t err = launch_plain(F, poses, N, e, keys, ls, stream);
  if (err == hipSuccess)
    err = launch_epilogue(F, poses, N, e, keys, nullptr, 0, d, edge, obst, nullptr, stream);
  return hip_status(err);
}

int psdf_grad(const float* footprint, int32_t m, const float* poses, int32_t N,
              const psdf_edges* edges, const psdf_params* params, float* d, int32_t* edge,
              int32_t* obst, float* grad, uint64_t* keys, hipStream_t stream) {
  clear_error();
  FpConst F;
  psdf_edges e;
  int rc = plain_common(footprint, m, poses, N, edges, params, F, e);
  if (rc) return rc;
  if (N == 0) return PSDF_OK;
  if (!d || !edge || !obst || !grad || !keys)
    return set_error(PSDF_EINVAL, "an output pointer is NULL");
  LaunchShape ls = choose_shape(N, e.M);
  hipError_t err = launch_plain(F, poses, N, e, keys, ls, stream);
  if (err == hipSuccess)
    err = launch_epilogue(F, poses, N, e, keys, nullptr, 1, d, edge, obst, grad, stream);
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
  return hip_status(launch_epilogue(F, poses, N, e, keys, gout, 2, nullptr, nullptr, nullptr,
                                    gpose, stream));
}

size_t psdf_encode_ws_bytes(int32_t Mbar) { return Mbar > 0 ? (size_t)Mbar * sizeof(int) : 0; }

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
