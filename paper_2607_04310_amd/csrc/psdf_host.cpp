// Host-side validation, footprint preparation and launch heuristics.
#include "psdf_host.hpp"

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <map>
#include <mutex>
#include <tuple>
#include <utility>
#include <vector>

namespace psdf {

namespace {
thread_local std::string g_err;
}

const char* last_error() { return g_err.c_str(); }
void clear_error() { g_err.clear(); }

int set_error(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int hip_status(hipError_t err) {
  if (err == hipSuccess) return PSDF_OK;
  return set_error(PSDF_EHIP, "HIP error %d: %s", (int)err, hipGetErrorString(err));
}

int prepare_footprint(const float* xy, int m, const psdf_params* params, FpConst* F) {
  if (!xy) return set_error(PSDF_EINVAL, "footprint is NULL");
  if (m < 3 || m > kMaxFp)
    return set_error(PSDF_ENONCONVEX, "footprint has %d vertices, 3..%d allowed", m, kMaxFp);
  psdf_params p = {1e-12f, 1e-6f, 1000.0f};
  if (params) p = *params;
  if (!(p.eps >= 0.f) || !(p.eps_sat >= 0.f) || std::isnan(p.eta))
    return set_error(PSDF_EINVAL, "eps and eps_sat must be >= 0 and eta not NaN");
  double vx[kMaxFp], vy[kMaxFp];
  for (int l = 0; l < m; ++l) {
    vx[l] = xy[2 * l];
    vy[l] = xy[2 * l + 1];
    if (!std::isfinite(vx[l]) || !std::isfinite(vy[l]))
      return set_error(PSDF_EINVAL, "footprint vertex %d is not finite", l);
  }
  double area2 = 0.0;
  for (int l = 0; l < m; ++l) area2 += vx[l] * vy[(l + 1) % m] - vy[l] * vx[(l + 1) % m];
  const bool reversed = area2 < 0.0;
  if (reversed) {  // reorder counter-clockwise
    for (int l = 0; l < m / 2; ++l) {
      std::swap(vx[l], vx[m - 1 - l]);
      std::swap(vy[l], vy[m - 1 - l]);
    }
  }
  for (int l = 0; l < m; ++l) {
    const int b = (l + 1) % m;
    if (vx[b] == vx[l] && vy[b] == vy[l])
      return set_error(PSDF_EDEGENERATE, "footprint edge %d has zero length", l);
  }
  for (int l = 0; l < m; ++l) {
    const int a = l, b = (l + 1) % m, c = (l + 2) % m;
    const double ex = vx[b] - vx[a], ey = vy[b] - vy[a];
    const double cr = ex * (vy[c] - vy[b]) - ey * (vx[c] - vx[b]);
    if (!(cr > 0.0)) return set_error(PSDF_ENONCONVEX, "footprint is not strictly convex at vertex %d", b);
  }
  // Winding number 1: a strictly convex polygon turns once.
  double turn = 0.0;
  for (int l = 0; l < m; ++l) {
    const int a = l, b = (l + 1) % m, c = (l + 2) % m;
    const double a1 = std::atan2(vy[b] - vy[a], vx[b] - vx[a]);
    const double a2 = std::atan2(vy[c] - vy[b], vx[c] - vx[b]);
    double d = a2 - a1;
    while (d <= -M_PI) d += 2 * M_PI;
    while (d > M_PI) d -= 2 * M_PI;
    turn += d;
  }
  if (std::fabs(turn - 2 * M_PI) > 1e-6) return set_error(PSDF_ENONCONVEX, "footprint self-intersects");

  FpConst& f = *F;
  std::memset(&f, 0, sizeof f);
  f.m = m;
  f.reversed = reversed ? 1 : 0;
  f.eps = p.eps;
  f.eps_sat = p.eps_sat;
  f.eta = p.eta;
  f.hard = (p.eta <= 0.f || std::isinf(p.eta)) ? 1 : 0;
  for (int l = 0; l < m; ++l) {
    const int b = (l + 1) % m;
    const double ex = vx[b] - vx[l], ey = vy[b] - vy[l];
    const double len = std::sqrt(ex * ex + ey * ey);
    const double nx = ey / len, ny = -ex / len;   // outward normal of a CCW edge
    double lo = INFINITY, hi = -INFINITY;
    for (int k = 0; k < m; ++k) {
      const double q = vx[k] * nx + vy[k] * ny;
      lo = std::fmin(lo, q);
      hi = std::fmax(hi, q);
    }
    f.vx[l] = (float)vx[l];
    f.vy[l] = (float)vy[l];
    f.ex[l] = (float)ex;
    f.ey[l] = (float)ey;
    f.einv[l] = (float)(1.0 / (ex * ex + ey * ey + (double)p.eps));
    f.nx[l] = (float)nx;
    f.ny[l] = (float)ny;
    f.pa[l] = (float)lo;
    f.pb[l] = (float)hi;
    f.ux[l] = (float)(ex / len);
    f.uy[l] = (float)(ey / len);
    f.len[l] = (float)len;
    f.cu[l] = (float)((vx[l] * ex + vy[l] * ey) / len);
    f.cn[l] = (float)(vx[l] * nx + vy[l] * ny);
    f.oa[l] = (float)(lo - (vx[l] * nx + vy[l] * ny));
    f.ob[l] = (float)(hi - (vx[l] * nx + vy[l] * ny));
  }
  // certificate constants (see FpConst)
  double rmax = 0.0, max_ext = 0.0;
  for (int l = 0; l < m; ++l) {
    rmax = std::fmax(rmax, std::sqrt(vx[l] * vx[l] + vy[l] * vy[l]));
    const int a = l, b = (l + 1) % m, c = (l + 2) % m;
    const double e1x = vx[b] - vx[a], e1y = vy[b] - vy[a], e2x = vx[c] - vx[b], e2y = vy[c] - vy[b];
    const double ext = std::atan2(e1x * e2y - e1y * e2x, e1x * e2x + e1y * e2y);  // exterior angle
    max_ext = std::fmax(max_ext, ext);
  }
  const double kappa = std::cos(0.5 * max_ext);
  f.rmax = (float)(rmax * (1.0 + 1e-6) + 1e-6);
  f.tau_sep = kappa > 1e-3 ? (float)((double)p.eps_sat / kappa + 1e-3) : INFINITY;
  for (int l = m; l < kMaxFp; ++l) {  // padded slots repeat slot m - 1
    f.vx[l] = f.vx[m - 1]; f.vy[l] = f.vy[m - 1];
    f.ex[l] = f.ex[m - 1]; f.ey[l] = f.ey[m - 1];
    f.einv[l] = f.einv[m - 1];
    f.nx[l] = f.nx[m - 1]; f.ny[l] = f.ny[m - 1];
    f.pa[l] = f.pa[m - 1]; f.pb[l] = f.pb[m - 1];
    f.ux[l] = f.ux[m - 1]; f.uy[l] = f.uy[m - 1]; f.len[l] = f.len[m - 1];
    f.cu[l] = f.cu[m - 1]; f.cn[l] = f.cn[m - 1];
    f.oa[l] = f.oa[m - 1]; f.ob[l] = f.ob[m - 1];
  }
  return PSDF_OK;
}

int check_edges(const psdf_edges* in, psdf_edges* out) {
  if (!in) return set_error(PSDF_EINVAL, "edges is NULL");
  if (in->E < 0 || in->M < 0) return set_error(PSDF_EINVAL, "E = %d, M = %d", in->E, in->M);
  if (in->mbar < 1 || in->mbar > kMaxObst)
    return set_error(PSDF_ETOOBIG, "mbar = %d, 1..%d allowed", in->mbar, kMaxObst);
  if (in->E > 0 && (!in->ax || !in->ay || !in->bx || !in->by))
    return set_error(PSDF_EINVAL, "an edge array is NULL");
  if (in->M > 0 && !in->obst_off) return set_error(PSDF_EINVAL, "obst_off is NULL");
  *out = *in;
  return PSDF_OK;
}

LaunchShape choose_shape(int N, int M) {
  // Enough waves to cover 1024 SIMDs about four deep, then as many stages per
  // work-group as that allows (each reuse amortises the obstacle load).
  const int waves = (M + 63) / 64;
  LaunchShape ls{256, 1};
  if (M <= 1024) ls.blk = 64;
  const long target = 4096;
  int sb = 1;
  while (sb < kMaxStageBlock && (long)waves * ((N + 2 * sb - 1) / (2 * sb)) >= target) sb *= 2;
  ls.sb = sb;
  return ls;
}

namespace {
std::mutex g_shape_mu;
LaunchShape g_override{0, 0};
}  // namespace

LaunchShape tuned_shape(int m, int mbar, int N, int M) {
  (void)m;
  (void)mbar;
  std::lock_guard<std::mutex> lk(g_shape_mu);
  if (g_override.blk) return g_override;
  return choose_shape(N, M);
}

namespace {
struct Timer {
  std::mutex mu;
  std::vector<hipEvent_t> ev;   // start, stop pairs
  size_t used = 0;              // events recorded (even: between launches)
  bool open = false;
} g_timer;
}  // namespace

void timer_begin(hipStream_t st) {
  std::lock_guard<std::mutex> lk(g_timer.mu);
  if (g_timer.used + 2 > g_timer.ev.size()) return;
  if (hipEventRecord(g_timer.ev[g_timer.used], st) == hipSuccess) {
    ++g_timer.used;
    g_timer.open = true;
  }
}

bool timer_kernel_events(hipEvent_t* start, hipEvent_t* stop) {
  std::lock_guard<std::mutex> lk(g_timer.mu);
  if (g_timer.open || g_timer.used + 2 > g_timer.ev.size()) return false;
  *start = g_timer.ev[g_timer.used];
  *stop = g_timer.ev[g_timer.used + 1];
  g_timer.used += 2;
  return true;
}

void timer_end(hipStream_t st) {
  std::lock_guard<std::mutex> lk(g_timer.mu);
  if (!g_timer.open) return;
  g_timer.open = false;
  if (hipEventRecord(g_timer.ev[g_timer.used], st) == hipSuccess) ++g_timer.used;
  else --g_timer.used;
}

}  // namespace psdf

using namespace psdf;

extern "C" int psdf_set_launch_shape(int32_t blk, int32_t sb) {
  clear_error();
  if (blk == 0) {
    std::lock_guard<std::mutex> lk(g_shape_mu);
    g_override = LaunchShape{0, 0};
    return PSDF_OK;
  }
  if ((blk != 64 && blk != 256) || sb < 1 || sb > kMaxStageBlock)
    return set_error(PSDF_EINVAL, "launch shape blk=%d sb=%d (blk 64 or 256, sb 1..%d)", blk, sb,
                     kMaxStageBlock);
  std::lock_guard<std::mutex> lk(g_shape_mu);
  g_override = LaunchShape{blk, sb};
  return PSDF_OK;
}

extern "C" int psdf_timer_enable(int32_t capacity) {
  clear_error();
  std::lock_guard<std::mutex> lk(g_timer.mu);
  for (hipEvent_t e : g_timer.ev) (void)hipEventDestroy(e);
  g_timer.ev.clear();
  g_timer.used = 0;
  g_timer.open = false;
  if (capacity < 0) return set_error(PSDF_EINVAL, "capacity %d < 0", capacity);
  for (int i = 0; i < 2 * capacity; ++i) {
    hipEvent_t e;
    hipError_t err = hipEventCreate(&e);
    if (err != hipSuccess) return hip_status(err);
    g_timer.ev.push_back(e);
  }
  return PSDF_OK;
}

extern "C" int psdf_timer_read(double* total_ms, int64_t* launches) {
  clear_error();
  if (!total_ms || !launches) return set_error(PSDF_EINVAL, "NULL output");
  std::lock_guard<std::mutex> lk(g_timer.mu);
  double sum = 0.0;
  const size_t pairs = g_timer.used / 2;
  for (size_t i = 0; i < pairs; ++i) {
    hipError_t err = hipEventSynchronize(g_timer.ev[2 * i + 1]);
    if (err != hipSuccess) return hip_status(err);
    float ms = 0.f;
    err = hipEventElapsedTime(&ms, g_timer.ev[2 * i], g_timer.ev[2 * i + 1]);
    if (err != hipSuccess) return hip_status(err);
    sum += ms;
  }
  *total_ms = sum;
  *launches = (int64_t)pairs;
  g_timer.used = 0;
  return PSDF_OK;
}
