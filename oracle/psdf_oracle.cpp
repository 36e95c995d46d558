// FP64 CPU oracle of the Polygonal Signed Distance Function (PSDF).
//
// TEST INFRASTRUCTURE ONLY.  This file is the reference that the HIP path is
// checked against.  Only the test suite, the smoke check and the CPU-baseline
// leg of the benchmark may load it; the product path never calls it and shares
// no code, header or constant with it.
//
// It is written for reading, not speed: every step follows the paper's
// pipeline (Sec. IV-A "Architecture Overview", items 1-4) in the paper's order
// and notation, in double precision, on the FP32 inputs promoted to double.
//
//   1. coordinate transform   Sec. IV-A, eq. for A~, B~  (A~ = R(theta)^T (A - p))
//   2. point-segment pools    Sec. IV-B, eqs. for u, t, d(P,[A,B]), d_v, d_e, d_sep
//   3. SAT + soft-min depth   Sec. IV-C, eqs. for n', N^i, I_P0, I_i, delta, separated,
//                             and the log-sum-exp penetration depth
//   4. synthesis, min         Sec. IV-D, eqs. for sd and phi = min_i sd^i
//
// The gradient with respect to the pose (x, y, theta) is obtained by running
// the very same template code on a forward-mode dual number with three
// tangent directions.  Kinks follow the active-branch subgradient convention
// of Sec. IV-D: a min/max over bit-equal entries averages their tangents
// (the even split of a tensor min-reduction), ReLU'(0) = 0, max(delta,0)'
// at 0 is 0, and across obstacles the lowest index attaining the minimum wins.
//
// Readings where the paper is silent (all are runtime parameters or stated
// conventions; parity of their absolute values is unpinned):
//   * eps (Sec. IV-B, IV-C), eps_sat (Sec. IV-C) and eta (soft-min) values.
//   * eta <= 0 or eta = +inf selects the hard minimum (the eta -> inf limit).
//   * The obstacle vertex set is {A~_j} U {B~_j}: identical to {A~_j} for a
//     closed polygon, and it makes a one-edge "free segment" a two-vertex set.
//   * The log-sum-exp is evaluated in its max-shifted form (same value in exact
//     arithmetic); no clamp is applied to its sign.
//   * The footprint may be given in either orientation; it is reordered CCW.
//   * The reported edge of the winning obstacle is the one with the smallest
//     (pool distance, edge index), where the pool distance of edge j is the
//     min over the robot vertices to [A~_j,B~_j] and over A~_j, B~_j to the
//     robot edges.

#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <vector>
#include <algorithm>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

// ---------------------------------------------------------------- scalar types

// Forward-mode dual number: value and tangents along (x, y, theta).
struct Dual {
  double v;
  double g[3];
  Dual() : v(0) { g[0] = g[1] = g[2] = 0; }
  Dual(double x) : v(x) { g[0] = g[1] = g[2] = 0; }  // NOLINT: implicit constant
};
inline Dual operator+(const Dual& a, const Dual& b) { Dual r(a.v + b.v); for (int k = 0; k < 3; ++k) r.g[k] = a.g[k] + b.g[k]; return r; }
inline Dual operator-(const Dual& a, const Dual& b) { Dual r(a.v - b.v); for (int k = 0; k < 3; ++k) r.g[k] = a.g[k] - b.g[k]; return r; }
inline Dual operator-(const Dual& a) { Dual r(-a.v); for (int k = 0; k < 3; ++k) r.g[k] = -a.g[k]; return r; }
inline Dual operator*(const Dual& a, const Dual& b) { Dual r(a.v * b.v); for (int k = 0; k < 3; ++k) r.g[k] = a.g[k] * b.v + a.v * b.g[k]; return r; }
inline Dual operator/(const Dual& a, const Dual& b) { Dual r(a.v / b.v); for (int k = 0; k < 3; ++k) r.g[k] = (a.g[k] * b.v - a.v * b.g[k]) / (b.v * b.v); return r; }
inline Dual dsqrt(const Dual& a) { Dual r(std::sqrt(a.v)); for (int k = 0; k < 3; ++k) r.g[k] = a.g[k] / (2.0 * r.v); return r; }
inline Dual dexp(const Dual& a) { Dual r(std::exp(a.v)); for (int k = 0; k < 3; ++k) r.g[k] = a.g[k] * r.v; return r; }
inline Dual dlog(const Dual& a) { Dual r(std::log(a.v)); for (int k = 0; k < 3; ++k) r.g[k] = a.g[k] / a.v; return r; }
inline Dual dcos(const Dual& a) { Dual r(std::cos(a.v)); for (int k = 0; k < 3; ++k) r.g[k] = -std::sin(a.v) * a.g[k]; return r; }
inline Dual dsin(const Dual& a) { Dual r(std::sin(a.v)); for (int k = 0; k < 3; ++k) r.g[k] = std::cos(a.v) * a.g[k]; return r; }
inline double val(const Dual& a) { return a.v; }

inline double dsqrt(double a) { return std::sqrt(a); }
inline double dexp(double a) { return std::exp(a); }
inline double dlog(double a) { return std::log(a); }
inline double dcos(double a) { return std::cos(a); }
inline double dsin(double a) { return std::sin(a); }
inline double val(double a) { return a; }

// Active-branch scan (test support for the subgradient check of Sec. IV-D).
// While a scan is installed, every min / max whose extreme is attained by
// several entries (within `tol` of it) and every ReLU whose argument lies
// within `tol` of its kink passes on the tangent of ONE active branch,
// picked by the scan's next digit, instead of the even split; the number of
// active branches of each such kink and the weight the default convention
// gives each (even split over bit-equal entries, ReLU'(0) = 0) are
// recorded in evaluation order.  Which kinks occur, and their branch
// counts, depend on the values only, never on the digits, so every run
// meets the same kinks and all combinations can be visited.  Without a scan
// (the default) nothing changes.
struct TieScan {
  double tol = 0.0;
  std::vector<int> digit;                  // branch taken at each kink met so far
  std::vector<int> count;                  // active branches of each kink
  std::vector<std::vector<double>> weight; // each branch's weight in the default convention
  size_t pos = 0;
};
thread_local TieScan* g_scan = nullptr;
// With g_probe >= 0 the obstacle evaluation returns max(delta(n_q), 0) of
// axis q = g_probe in place of sd (test support: the soft-min and the hard
// minimum combine these per-axis terms).
thread_local int g_probe = -1;

int scan_choice(int n, const std::vector<double>& w) {
  TieScan& t = *g_scan;
  const size_t k = t.pos++;
  if (t.count.size() <= k) {
    t.count.push_back(n);
    t.weight.push_back(w);
  }
  return k < t.digit.size() ? t.digit[k] % n : 0;
}

// ReLU with ReLU'(0) = 0; NaN propagates (as in a tensor ReLU).
inline double relu(double a) { return (a > 0 || a != a) ? a : 0.0; }
inline Dual relu(const Dual& a) {
  if (a.v != a.v) return a;
  if (g_scan && std::fabs(a.v) <= g_scan->tol) {   // kink: the zero branch or the identity
    Dual r(a.v > 0 ? a.v : 0.0);
    if (scan_choice(2, {a.v > 0 ? 0.0 : 1.0, a.v > 0 ? 1.0 : 0.0}) == 1)
      for (int k = 0; k < 3; ++k) r.g[k] = a.g[k];
    return r;
  }
  return a.v > 0 ? a : Dual(0.0);
}

// Min / max over a list: the value is the extreme; the tangent is the mean of
// the tangents of all bit-equal extreme entries (even split at ties).  A NaN
// entry makes the result NaN (as in a tensor min/max reduction).
template <class T> T reduce_min(const std::vector<T>& xs);
template <class T> T reduce_max(const std::vector<T>& xs);

template <> double reduce_min<double>(const std::vector<double>& xs) {
  double m = std::numeric_limits<double>::infinity();
  for (double x : xs) { if (x != x) return x; m = std::min(m, x); }
  return m;
}
template <> double reduce_max<double>(const std::vector<double>& xs) {
  double m = -std::numeric_limits<double>::infinity();
  for (double x : xs) { if (x != x) return x; m = std::max(m, x); }
  return m;
}
template <class Cmp>
Dual reduce_split(const std::vector<Dual>& xs, Cmp better) {
  double m = xs[0].v;
  for (const Dual& x : xs) {
    if (x.v != x.v) return Dual(x.v);
    if (better(x.v, m)) m = x.v;
  }
  Dual r(m);
  if (g_scan) {   // one active entry, picked by the scan
    std::vector<size_t> act;
    std::vector<double> w;   // the even split's weight of each active entry
    int n_eq = 0;
    for (size_t i = 0; i < xs.size(); ++i)
      if (xs[i].v == m || std::fabs(xs[i].v - m) <= g_scan->tol) {
        act.push_back(i);
        w.push_back(xs[i].v == m ? 1.0 : 0.0);
        n_eq += xs[i].v == m;
      }
    for (double& x : w) x /= n_eq;
    const size_t c = act.size() > 1 ? (size_t)scan_choice((int)act.size(), w) : 0;
    for (int k = 0; k < 3; ++k) r.g[k] = xs[act[c]].g[k];
    return r;
  }
  int cnt = 0;
  for (const Dual& x : xs)
    if (x.v == m) { for (int k = 0; k < 3; ++k) r.g[k] += x.g[k]; ++cnt; }
  for (int k = 0; k < 3; ++k) r.g[k] /= cnt;
  return r;
}
template <> Dual reduce_min<Dual>(const std::vector<Dual>& xs) {
  return reduce_split(xs, [](double a, double b) { return a < b; });
}
template <> Dual reduce_max<Dual>(const std::vector<Dual>& xs) {
  return reduce_split(xs, [](double a, double b) { return a > b; });
}
template <class T> T min2(const T& a, const T& b) { return reduce_min<T>({a, b}); }

// ---------------------------------------------------------------- geometry

struct Vec { double x, y; };

// Footprint in the robot-local frame, CCW, with its outward unit edge normals.
struct Footprint {
  std::vector<Vec> v;   // V^0, CCW
  std::vector<Vec> n;   // n_l: outward unit normal of E_l = [v_l, v_{l+1}]
  bool reversed = false;  // the caller's order was clockwise (v[k] = caller[m-1-k])
};

Footprint make_footprint(const double* xy, int m) {
  Footprint f;
  for (int l = 0; l < m; ++l) f.v.push_back({xy[2 * l], xy[2 * l + 1]});
  double area2 = 0;  // twice the signed area (shoelace)
  for (int l = 0; l < m; ++l) {
    const Vec& a = f.v[l]; const Vec& b = f.v[(l + 1) % m];
    area2 += a.x * b.y - a.y * b.x;
  }
  if (area2 < 0) {  // the paper requires CCW
    std::reverse(f.v.begin(), f.v.end());
    f.reversed = true;
  }
  for (int l = 0; l < m; ++l) {
    const Vec& a = f.v[l]; const Vec& b = f.v[(l + 1) % m];
    double ex = b.x - a.x, ey = b.y - a.y, len = std::sqrt(ex * ex + ey * ey);
    // For a CCW polygon the outward normal of edge e is e rotated by -90 deg.
    f.n.push_back({ey / len, -ex / len});
  }
  return f;
}

template <class T> struct P2 { T x, y; };

// Branch-free point-to-segment distance, Sec. IV-B:
//   v = B - A,  u = (P - A).v / (|v|^2 + eps),  t = ReLU(u) - ReLU(u - 1),
//   Q = A + t v,  d = |P - Q|.
template <class T>
T seg_dist(const P2<T>& P, const P2<T>& A, const P2<T>& B, double eps) {
  T vx = B.x - A.x, vy = B.y - A.y;
  T u = ((P.x - A.x) * vx + (P.y - A.y) * vy) / (vx * vx + vy * vy + T(eps));
  T t = relu(u) - relu(u - T(1.0));
  T qx = A.x + t * vx, qy = A.y + t * vy;
  T rx = P.x - qx, ry = P.y - qy;
  return dsqrt(rx * rx + ry * ry);
}

struct Params { double eps, eps_sat, eta; };

template <class T>
struct ObstacleEval {
  T sd;                   // sd(P^0(x), P^i), Sec. IV-D
  bool separated;         // SAT flag, Sec. IV-C
  T d_sep;                // separation distance, Sec. IV-B
  std::vector<double> edge_pool;  // per-edge pool distance (for the reported edge)
};

// Signed distance between the footprint V0 (CCW, local frame) at pose
// (px, py, th) and obstacle i, whose edges are [A_j, B_j], j = 0..mi-1 (world
// frame).  Every input may carry tangents: the pose for the pose gradient,
// the endpoints and vertices for the geometry gradient.
template <class T>
ObstacleEval<T> eval_obstacle_geo(const std::vector<P2<T>>& V0, const T& px, const T& py,
                                  const T& th, const std::vector<P2<T>>& Aw,
                                  const std::vector<P2<T>>& Bw, const Params& prm) {
  const int m = (int)V0.size();
  const int mi = (int)Aw.size();
  ObstacleEval<T> out;

  // ---- Step 1: coordinate transform, A~ = R^T (A - p), B~ = R^T (B - p).
  // R(theta) = [[c, -s], [s, c]]  =>  R^T (dx, dy) = (c dx + s dy, -s dx + c dy).
  T c = dcos(th), s = dsin(th);
  std::vector<P2<T>> At(mi), Bt(mi);
  for (int j = 0; j < mi; ++j) {
    T dx = Aw[j].x - px, dy = Aw[j].y - py;
    At[j] = {c * dx + s * dy, T(0.0) - s * dx + c * dy};
    T ex = Bw[j].x - px, ey = Bw[j].y - py;
    Bt[j] = {c * ex + s * ey, T(0.0) - s * ex + c * ey};
  }

  // ---- Step 2: point-to-segment pools.
  // d_v^i: robot vertices to obstacle edges.
  std::vector<T> pool_v;
  std::vector<double> edge_pool(mi, std::numeric_limits<double>::infinity());
  for (int l = 0; l < m; ++l)
    for (int j = 0; j < mi; ++j) {
      T d = seg_dist(V0[l], At[j], Bt[j], prm.eps);
      pool_v.push_back(d);
      edge_pool[j] = std::min(edge_pool[j], val(d));
    }
  // V_obs^i = {A~_j} U {B~_j}; d_e^i: obstacle vertices to robot edges E_l.
  std::vector<P2<T>> Vobs;
  std::vector<int> Vobs_edge;
  for (int j = 0; j < mi; ++j) { Vobs.push_back(At[j]); Vobs_edge.push_back(j); }
  for (int j = 0; j < mi; ++j) { Vobs.push_back(Bt[j]); Vobs_edge.push_back(j); }
  std::vector<T> pool_e;
  for (size_t k = 0; k < Vobs.size(); ++k)
    for (int l = 0; l < m; ++l) {
      T d = seg_dist(Vobs[k], V0[l], V0[(l + 1) % m], prm.eps);
      pool_e.push_back(d);
      int j = Vobs_edge[k];
      edge_pool[j] = std::min(edge_pool[j], val(d));
    }
  T d_v = reduce_min(pool_v), d_e = reduce_min(pool_e);
  out.d_sep = min2(d_v, d_e);
  out.edge_pool = edge_pool;

  // ---- Step 3: SAT over the candidate axes N^i = {n_l} U {n'_j}.
  std::vector<P2<T>> axes;
  for (int l = 0; l < m; ++l) {
    // outward unit normal of the CCW footprint edge E_l: e_l rotated by -90 deg
    T ex = V0[(l + 1) % m].x - V0[l].x, ey = V0[(l + 1) % m].y - V0[l].y;
    T len = dsqrt(ex * ex + ey * ey);
    axes.push_back({ey / len, (T(0.0) - ex) / len});
  }
  for (int j = 0; j < mi; ++j) {
    T ux = Bt[j].x - At[j].x, uy = Bt[j].y - At[j].y;       // u_j = B~_j - A~_j
    T den = dsqrt(ux * ux + uy * uy) + T(prm.eps);          // |u_j| + eps
    axes.push_back({(T(0.0) - uy) / den, ux / den});        // rot90(u_j)/(|u_j|+eps)
  }
  std::vector<T> delta;
  bool separated = false;
  for (const P2<T>& n : axes) {
    std::vector<T> pr, po;
    for (int l = 0; l < m; ++l) pr.push_back(V0[l].x * n.x + V0[l].y * n.y);
    for (const P2<T>& w : Vobs) po.push_back(w.x * n.x + w.y * n.y);
    T aP = reduce_min(pr), bP = reduce_max(pr);   // I_P0(n)
    T ai = reduce_min(po), bi = reduce_max(po);   // I_i(n)
    T dl = min2(bi - aP, bP - ai);                // delta^i(n)
    delta.push_back(dl);
    if (val(dl) < -prm.eps_sat) separated = true; // separated^i
  }
  out.separated = separated;

  // Smooth penetration depth: -(1/eta) log sum exp(-eta * max(delta, 0)).
  std::vector<T> dplus;
  for (const T& dl : delta) dplus.push_back(relu(dl));
  if (g_probe >= 0) {   // test support: one axis's term alone
    out.sd = g_probe < (int)dplus.size() ? dplus[g_probe] : T(std::nan(""));
    return out;
  }
  T pen;
  const bool hard = !(prm.eta > 0) || std::isinf(prm.eta);
  if (hard) {
    pen = reduce_min(dplus);
  } else {
    double mu = val(reduce_min(dplus));   // shift constant: the value only
    T acc = T(0.0);
    for (const T& dp : dplus) acc = acc + dexp(T(-prm.eta) * (dp - T(mu)));
    pen = T(mu) - dlog(acc) / T(prm.eta);
  }

  // ---- Step 4: synthesis.
  out.sd = separated ? out.d_sep : T(0.0) - pen;
  return out;
}

// The same with constant geometry: the footprint F and obstacle edges as
// plain doubles; only the pose may carry tangents.
template <class T>
ObstacleEval<T> eval_obstacle(const Footprint& F, const T& px, const T& py, const T& th,
                              const double* ax, const double* ay, const double* bx,
                              const double* by, int mi, const Params& prm) {
  std::vector<P2<T>> V0(F.v.size()), Aw(mi), Bw(mi);
  for (size_t l = 0; l < F.v.size(); ++l) V0[l] = {T(F.v[l].x), T(F.v[l].y)};
  for (int j = 0; j < mi; ++j) {
    Aw[j] = {T(ax[j]), T(ay[j])};
    Bw[j] = {T(bx[j]), T(by[j])};
  }
  return eval_obstacle_geo<T>(V0, px, py, th, Aw, Bw, prm);
}

struct Edges {
  const double *ax, *ay, *bx, *by;
  const int32_t* off;
  int M;
};

struct StageResult {
  double phi;
  int obst, edge, penetrating;
  double grad[3];
};

StageResult eval_stage(const Footprint& F, const double* pose, const Edges& Ed, const Params& prm) {
  StageResult r;
  r.phi = std::numeric_limits<double>::infinity();
  r.obst = r.edge = -1;
  r.penetrating = 0;
  r.grad[0] = r.grad[1] = r.grad[2] = 0.0;
  bool any_nan = false;
  // phi = min_i sd^i; the lowest index attaining the minimum wins.
  for (int i = 0; i < Ed.M; ++i) {
    int e0 = Ed.off[i], mi = Ed.off[i + 1] - e0;
    if (mi <= 0) continue;
    ObstacleEval<double> ev = eval_obstacle<double>(F, pose[0], pose[1], pose[2], Ed.ax + e0,
                                                    Ed.ay + e0, Ed.bx + e0, Ed.by + e0, mi, prm);
    if (std::isnan(ev.sd)) { any_nan = true; break; }
    if (ev.sd < r.phi) {
      r.phi = ev.sd;
      r.obst = i;
      r.penetrating = ev.separated ? 0 : 1;
      int jb = 0;
      for (int j = 1; j < mi; ++j)
        if (ev.edge_pool[j] < ev.edge_pool[jb]) jb = j;
      r.edge = e0 + jb;
    }
  }
  if (any_nan) {
    r.phi = std::numeric_limits<double>::quiet_NaN();
    r.obst = r.edge = -1;
    r.grad[0] = r.grad[1] = r.grad[2] = std::numeric_limits<double>::quiet_NaN();
    return r;
  }
  if (r.obst < 0) return r;
  // Gradient through the winning obstacle only (active-branch subgradient).
  Dual px(pose[0]), py(pose[1]), th(pose[2]);
  px.g[0] = 1; py.g[1] = 1; th.g[2] = 1;
  int e0 = Ed.off[r.obst], mi = Ed.off[r.obst + 1] - e0;
  ObstacleEval<Dual> ev = eval_obstacle<Dual>(F, px, py, th, Ed.ax + e0, Ed.ay + e0,
                                              Ed.bx + e0, Ed.by + e0, mi, prm);
  for (int k = 0; k < 3; ++k) r.grad[k] = ev.sd.g[k];
  return r;
}

}  // namespace

extern "C" {

// Full PSDF for every stage pose: phi, winning obstacle / edge, gradient.
//   fp_xy   : m x 2 footprint vertices (local frame), either orientation
//   poses   : N x 3 (x, y, theta)
//   ax..by  : E edge endpoints (world frame); obstacle i owns [off[i], off[i+1])
//   eta     : soft-min sharpness; <= 0 or +inf selects the hard minimum
//   outputs : phi[N], obst[N], edge[N], grad[N x 3], pen[N] (1 if the winner
//             is in the non-separated branch)
//   nthreads: OpenMP threads over stages (<= 0: runtime default)
// Returns the number of threads used.
int oracle_psdf(const double* fp_xy, int m, const double* poses, int N, const double* ax,
                const double* ay, const double* bx, const double* by, const int32_t* off, int M,
                double eps, double eps_sat, double eta, double* phi, int32_t* obst,
                int32_t* edge, double* grad, int32_t* pen, int nthreads) {
  Footprint F = make_footprint(fp_xy, m);
  Edges Ed{ax, ay, bx, by, off, M};
  Params prm{eps, eps_sat, eta};
  int used = 1;
#ifdef _OPENMP
  if (nthreads <= 0) nthreads = omp_get_max_threads();
  used = nthreads;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
#endif
  for (int s = 0; s < N; ++s) {
    StageResult r = eval_stage(F, poses + 3 * s, Ed, prm);
    phi[s] = r.phi;
    obst[s] = r.obst;
    edge[s] = r.edge;
    pen[s] = r.penetrating;
    for (int k = 0; k < 3; ++k) grad[3 * s + k] = r.grad[k];
  }
  return used;
}

// Per-obstacle detail for one (stage, obstacle): sd, separated flag, d_sep,
// per-edge pool distance (mi entries) and d sd / d(x, y, theta).
void oracle_obstacle(const double* fp_xy, int m, const double* pose, const double* ax,
                     const double* ay, const double* bx, const double* by, int mi, double eps,
                     double eps_sat, double eta, double* sd, int32_t* separated, double* d_sep,
                     double* edge_pool, double* grad) {
  Footprint F = make_footprint(fp_xy, m);
  Params prm{eps, eps_sat, eta};
  Dual px(pose[0]), py(pose[1]), th(pose[2]);
  px.g[0] = 1; py.g[1] = 1; th.g[2] = 1;
  ObstacleEval<Dual> ev = eval_obstacle<Dual>(F, px, py, th, ax, ay, bx, by, mi, prm);
  *sd = ev.sd.v;
  *separated = ev.separated ? 1 : 0;
  *d_sep = ev.d_sep.v;
  for (int j = 0; j < mi; ++j) edge_pool[j] = ev.edge_pool[j];
  for (int k = 0; k < 3; ++k) grad[k] = ev.sd.g[k];
}

// Active-branch (selection) gradients of sd for one (stage, obstacle): the
// pose gradient obtained when each kink of the pipeline (a min / max
// attained by several entries within `tol`, a ReLU argument within `tol` of
// zero) takes one of its active branches (Sec. IV-D: any active branch
// gives a valid subgradient).  Kinks whose branch never changes the
// gradient (those in a part of the pipeline that sd does not use) are found
// by flipping each kink's branch at the first-branch combination and at 64
// pseudo-random ones, and are held at their first branch.  With probe = q
// >= 0 the enumerated quantity is axis q's term max(delta(n_q), 0) instead
// of sd (the penetration branch combines these terms).  Up to 65536
// combinations of the remaining kinks are all visited; beyond that,
// `samples` pseudo-random combinations are.  The distinct gradients (up to
// 1e-12 relative) go to out[k][3], at most max_out of them.  first[3]
// receives the gradient with the first active entry at every kink (in the
// pipeline's index order).  mean[3] receives the average over a complete
// enumeration weighted as the default convention weighs the branches (even
// split over bit-equal entries, ReLU'(0) = 0), which for tol = 0 is the
// gradient of oracle_obstacle (NaN when sampled).  *combos gets the number
// of combinations of the live kinks (capped at 2^62), *sampled 1 if they
// were sampled.  Returns the number of distinct gradients.
int oracle_obstacle_selections(const double* fp_xy, int m, const double* pose, const double* ax,
                               const double* ay, const double* bx, const double* by, int mi,
                               double eps, double eps_sat, double eta, double tol, int probe,
                               int max_out, int samples, double* out, double* first,
                               double* mean, int64_t* combos, int32_t* sampled) {
  Footprint F = make_footprint(fp_xy, m);
  g_probe = probe;
  Params prm{eps, eps_sat, eta};
  Dual px(pose[0]), py(pose[1]), th(pose[2]);
  px.g[0] = 1; py.g[1] = 1; th.g[2] = 1;
  TieScan scan;
  scan.tol = tol;
  g_scan = &scan;
  auto run = [&](const std::vector<int>& digit, double g[3]) {
    scan.digit = digit;
    scan.pos = 0;
    ObstacleEval<Dual> ev = eval_obstacle<Dual>(F, px, py, th, ax, ay, bx, by, mi, prm);
    for (int k = 0; k < 3; ++k) g[k] = ev.sd.g[k];
  };
  auto same = [](const double* a, const double* b) {
    double diff = 0, scale = 1;
    for (int k = 0; k < 3; ++k) {
      diff = std::max(diff, std::fabs(a[k] - b[k]));
      scale = std::max(scale, std::fabs(b[k]));
    }
    return diff <= 1e-12 * scale || (a[0] != a[0] && b[0] != b[0]);
  };
  uint64_t lcg = 0x9e3779b97f4a7c15ull;
  auto next = [&](uint64_t n) {
    lcg = lcg * 6364136223846793005ull + 1442695040888963407ull;
    return (int)((lcg >> 33) % n);
  };
  run({}, first);   // meets every kink and records its branches
  const std::vector<int> count = scan.count;
  const std::vector<std::vector<double>> weight = scan.weight;
  const size_t nk = count.size();
  std::vector<char> live(nk, 0);
  for (int trial = 0; trial <= 64; ++trial) {
    std::vector<int> base(nk, 0);
    if (trial > 0)
      for (size_t k = 0; k < nk; ++k) base[k] = next((uint64_t)count[k]);
    double gb[3];
    run(base, gb);
    for (size_t k = 0; k < nk; ++k) {
      if (live[k] || count[k] < 2) continue;
      for (int c = 0; c < count[k] && !live[k]; ++c) {
        if (c == base[k]) continue;
        std::vector<int> alt = base;
        alt[k] = c;
        double ga[3];
        run(alt, ga);
        if (!same(ga, gb)) live[k] = 1;
      }
    }
  }
  std::vector<size_t> idx;
  int64_t total = 1;
  for (size_t k = 0; k < nk; ++k)
    if (live[k]) {
      idx.push_back(k);
      total = total > ((int64_t)1 << 62) / count[k] ? ((int64_t)1 << 62) : total * count[k];
    }
  *combos = total;
  const bool full = total <= 65536;
  *sampled = full ? 0 : 1;
  const int64_t visits = full ? total : std::max(1, samples);
  std::vector<int> digit(nk, 0);
  double acc[3] = {0, 0, 0};
  int n = 0;
  for (int64_t it = 0; it < visits; ++it) {
    if (!full && it > 0)
      for (size_t k : idx) digit[k] = next((uint64_t)count[k]);
    double g[3];
    run(digit, g);
    double wgt = 1.0;
    for (size_t k : idx) wgt *= weight[k][digit[k]];
    for (int k = 0; k < 3; ++k) acc[k] += wgt == 0.0 ? 0.0 : wgt * g[k];
    bool seen = false;
    for (int q = 0; q < n && !seen; ++q) seen = same(g, out + 3 * q);
    if (!seen && n < max_out) {
      for (int k = 0; k < 3; ++k) out[3 * n + k] = g[k];
      ++n;
    }
    if (full)
      for (size_t d : idx) {   // next combination of the live kinks (odometer)
        if (++digit[d] < count[d]) break;
        digit[d] = 0;
      }
  }
  g_scan = nullptr;
  g_probe = -1;
  for (int k = 0; k < 3; ++k) mean[k] = full ? acc[k] : std::nan("");
  return n;
}

// The penetration branch's per-axis terms of one (stage, obstacle): K = m +
// mi values max(delta(n_q), 0) in the pipeline's axis order (robot normals,
// then obstacle normals) to dplus[K], and the separated flag.  Returns K.
int oracle_obstacle_axes(const double* fp_xy, int m, const double* pose, const double* ax,
                         const double* ay, const double* bx, const double* by, int mi,
                         double eps, double eps_sat, double eta, double* dplus,
                         int32_t* separated) {
  Footprint F = make_footprint(fp_xy, m);
  Params prm{eps, eps_sat, eta};
  ObstacleEval<double> ev = eval_obstacle<double>(F, pose[0], pose[1], pose[2], ax, ay, bx, by,
                                                  mi, prm);
  *separated = ev.separated ? 1 : 0;
  for (int q = 0; q < m + mi; ++q) {
    g_probe = q;
    dplus[q] = eval_obstacle<double>(F, pose[0], pose[1], pose[2], ax, ay, bx, by, mi, prm).sd;
  }
  g_probe = -1;
  return m + mi;
}

// d sd / d(geometry) for one (stage, obstacle), by forward mode over every
// geometry coordinate (three per pass): g_edges[mi][4] = d sd / d(A_x, A_y,
// B_x, B_y) of each world edge endpoint, g_fp[m][2] = d sd / d(vertex) of the
// footprint in the caller's vertex order.  Same kink conventions as the pose
// gradient (even split over bit-equal entries of a min / max).
void oracle_obstacle_geom_grad(const double* fp_xy, int m, const double* pose, const double* ax,
                               const double* ay, const double* bx, const double* by, int mi,
                               double eps, double eps_sat, double eta, double* g_edges,
                               double* g_fp) {
  Footprint F = make_footprint(fp_xy, m);
  Params prm{eps, eps_sat, eta};
  const int P = 4 * mi + 2 * m;   // parameters: endpoints, then CCW footprint vertices
  for (int p0 = 0; p0 < P; p0 += 3) {
    std::vector<P2<Dual>> V0(m), Aw(mi), Bw(mi);
    for (int l = 0; l < m; ++l) V0[l] = {Dual(F.v[l].x), Dual(F.v[l].y)};
    for (int j = 0; j < mi; ++j) {
      Aw[j] = {Dual(ax[j]), Dual(ay[j])};
      Bw[j] = {Dual(bx[j]), Dual(by[j])};
    }
    auto coord = [&](int q) -> Dual& {
      if (q < 4 * mi) {
        const int j = q / 4, r = q % 4;
        P2<Dual>& e = r < 2 ? Aw[j] : Bw[j];
        return (r % 2 == 0) ? e.x : e.y;
      }
      const int l = (q - 4 * mi) / 2;
      return (q - 4 * mi) % 2 == 0 ? V0[l].x : V0[l].y;
    };
    for (int k = 0; k < 3 && p0 + k < P; ++k) coord(p0 + k).g[k] = 1.0;
    ObstacleEval<Dual> ev = eval_obstacle_geo<Dual>(V0, Dual(pose[0]), Dual(pose[1]),
                                                    Dual(pose[2]), Aw, Bw, prm);
    for (int k = 0; k < 3 && p0 + k < P; ++k) {
      const int q = p0 + k;
      if (q < 4 * mi) {
        g_edges[q] = ev.sd.g[k];
      } else {
        const int l = (q - 4 * mi) / 2, r = (q - 4 * mi) % 2;
        const int caller = F.reversed ? m - 1 - l : l;
        g_fp[2 * caller + r] = ev.sd.g[k];
      }
    }
  }
}

// sd^i for every (stage, obstacle): out is N x M, row-major.  Empty obstacles
// give +inf.
void oracle_sd_matrix(const double* fp_xy, int m, const double* poses, int N, const double* ax,
                      const double* ay, const double* bx, const double* by, const int32_t* off,
                      int M, double eps, double eps_sat, double eta, double* out, int nthreads) {
  Footprint F = make_footprint(fp_xy, m);
  Params prm{eps, eps_sat, eta};
#ifdef _OPENMP
  if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
#endif
  for (int s = 0; s < N; ++s)
    for (int i = 0; i < M; ++i) {
      int e0 = off[i], mi = off[i + 1] - e0;
      const double* p = poses + 3 * s;
      out[(size_t)s * M + i] =
          mi <= 0 ? std::numeric_limits<double>::infinity()
                  : eval_obstacle<double>(F, p[0], p[1], p[2], ax + e0, ay + e0, bx + e0, by + e0,
                                          mi, prm).sd;
    }
}

}  // extern "C"
