// psdf_batch: plan, work-item list, hipGraph capture and autotuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "psdf.h"
#include "psdf_batch.hpp"
#include "psdf_host.hpp"
#include "psdf_screen.hpp"
#include "psdf_horizon.hpp"

namespace psdf {

struct Shape {
  int sb;       // stages per work item
  int nw;       // waves per work-group (obstacles per tile = 64 nw)
  int direct;   // 1: one work-group per item instead of a persistent grid
};

}  // namespace psdf

using namespace psdf;

struct psdf_batch_plan {
  int device = 0;
  int n_inst = 0;
  int mi_class = 4;
  int flags = 0;
  int total_stages = 0;
  std::vector<psdf_batch_desc> desc;
  std::vector<FpConst> fp;
  Shape shape{1, 4, 0};
  int n_items = 0;
  int cu = 256;
  // one persistent launch per footprint-size group (MF = 3..8 or 16)
  // lane: the stream the group's launch goes to (0: the caller's, l > 0:
  // side[l - 1]); groups of one lane run one after another
  struct Group { int mf, start, count, grid, lane; };
  std::vector<Group> groups;
  int n_lanes = 1;
  // device memory owned by the plan
  FpConst* d_fp = nullptr;
  BatchInst* d_inst = nullptr;
  BatchItem* d_items = nullptr;
  size_t items_cap = 0;
  uint64_t* d_partial = nullptr;   // partial keys, then aux words
  size_t partial_cap = 0;          // entries of each
  unsigned* d_ctrl = nullptr;        // item counter per group
  // screening: stage -> instance, stage rows grouped by footprint size,
  // failed lists and counters (three per group)
  int* d_stage_inst = nullptr;
  FinStage* d_fin = nullptr;      // per stage: the finish kernel's record (set per shape)
  int4* d_stage_list = nullptr;   // (stage row, instance, circ_off, M) per screened stage
  int* d_failed = nullptr;
  int* d_fdone = nullptr;         // per failed slot: tiles done (bound form)
  unsigned* d_sctrl = nullptr;
  float4* d_hlist = nullptr;  // horizon lists (circle, index), sum M
  uint4* d_frag = nullptr;    // the screener's lane fragments, kFragWords x 64
  int* d_hcount = nullptr;    // per instance
  uint32_t* d_hrest = nullptr;
  struct SGroup { int mf, start, count, max_tiles; };
  std::vector<SGroup> sgroups;
  int max_M = 0;
  size_t sum_M = 0;
  // bounding circles taken once per edge set (psdf_batch_stage), indexed
  // like the horizon lists, and the edge arrays they were taken from
  float4* d_circ = nullptr;
  unsigned char* d_rows = nullptr;   // staged obstacle rows (psdf_staged.hpp)
  bool circ_staged = false;
  const void* circ_src[5] = {};
  // graph
  hipStream_t cap_stream = nullptr;
  // footprint-size groups run concurrently on up to kLanes streams: the
  // caller's and side[0 .. kLanes - 2], forked from and joined back to the
  // caller's stream with events (ev[0] the fork, ev[l] lane l's end)
  hipStream_t side[6] = {};
  hipEvent_t ev[7] = {};
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<const void*> bound;
};

namespace psdf {
namespace {

std::mutex g_cache_mu;
std::map<std::string, Shape> g_cache;
bool g_cache_loaded = false;

std::string signature(const psdf_batch_plan& p) {
  // batch size signature: instance count, edge class and log2 buckets of the
  // stage count and of the stage x edge pairs
  double pairs = 0.0;
  for (const auto& d : p.desc) pairs += (double)d.N * d.E;
  char buf[128];
  snprintf(buf, sizeof buf, "batch:%d:%d:%d:%d", p.n_inst, p.mi_class,
           (int)std::lround(std::log2(std::max(1, p.total_stages))),
           (int)std::lround(std::log2(std::max(1.0, pairs))));
  return buf;
}

void cache_load_locked() {
  if (g_cache_loaded) return;
  g_cache_loaded = true;
  const char* path = std::getenv("PSDF_TUNE_CACHE");
  if (!path) return;
  FILE* f = std::fopen(path, "r");
  if (!f) return;
  char key[128];
  int sb, nw, direct;
  while (std::fscanf(f, "%127s %d %d %d", key, &sb, &nw, &direct) == 4)
    if (sb >= 1 && sb <= kMaxStageBlock && (nw == 1 || nw == 4) && (direct == 0 || direct == 1))
      g_cache[key] = Shape{sb, nw, direct};
  std::fclose(f);
}

void cache_store(const std::string& key, Shape s) {
  std::lock_guard<std::mutex> lk(g_cache_mu);
  cache_load_locked();
  g_cache[key] = s;
  if (const char* path = std::getenv("PSDF_TUNE_CACHE")) {
    if (FILE* f = std::fopen(path, "a")) {
      std::fprintf(f, "%s %d %d %d\n", key.c_str(), s.sb, s.nw, s.direct);
      std::fclose(f);
    }
  }
}

bool cache_find(const std::string& key, Shape* s) {
  std::lock_guard<std::mutex> lk(g_cache_mu);
  cache_load_locked();
  auto it = g_cache.find(key);
  if (it == g_cache.end()) return false;
  *s = it->second;
  return true;
}

constexpr int kGroupMF[] = {3, 4, 5, 6, 7, 8, 16};
constexpr int kGroups = 7;
// Streams one call's groups run on (the caller's and kLanes - 1 plan-owned).
constexpr int kLanes = 4;
static_assert(sizeof(psdf_batch_plan::side) / sizeof(hipStream_t) == kGroups - 1 &&
                  sizeof(psdf_batch_plan::ev) / sizeof(hipEvent_t) == kGroups,
              "one side stream per group after the first, one event per group");
int group_of(int m) { return m <= 8 ? m - 3 : 6; }

hipError_t launch_batch(int mf, int mi_class, int nw, int grid, const BatchArgs& a, hipStream_t st,
                        hipEvent_t ev0, hipEvent_t ev1) {
  switch (mf) {
    case 3: return launch_batch_mf<3>(mi_class, nw, grid, a, st, ev0, ev1);
    case 4: return launch_batch_mf<4>(mi_class, nw, grid, a, st, ev0, ev1);
    case 5: return launch_batch_mf<5>(mi_class, nw, grid, a, st, ev0, ev1);
    case 6: return launch_batch_mf<6>(mi_class, nw, grid, a, st, ev0, ev1);
    case 7: return launch_batch_mf<7>(mi_class, nw, grid, a, st, ev0, ev1);
    case 8: return launch_batch_mf<8>(mi_class, nw, grid, a, st, ev0, ev1);
    default: return launch_batch_mf<16>(mi_class, nw, grid, a, st, ev0, ev1);
  }
}

int occupancy(int mf, int mi_class, int nw) {
  int b = 0;
  hipError_t err;
  switch (mf) {
    case 3: err = batch_occupancy_mf<3>(mi_class, nw, &b); break;
    case 4: err = batch_occupancy_mf<4>(mi_class, nw, &b); break;
    case 5: err = batch_occupancy_mf<5>(mi_class, nw, &b); break;
    case 6: err = batch_occupancy_mf<6>(mi_class, nw, &b); break;
    case 7: err = batch_occupancy_mf<7>(mi_class, nw, &b); break;
    case 8: err = batch_occupancy_mf<8>(mi_class, nw, &b); break;
    default: err = batch_occupancy_mf<16>(mi_class, nw, &b); break;
  }
  return (err == hipSuccess && b > 0) ? b : 1;
}

void free_graph(psdf_batch_plan* p) {
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  p->exec = nullptr;
  p->graph = nullptr;
  p->bound.clear();
}

// Build the instance table and the item list for a shape; upload both.
int build_items(psdf_batch_plan* p, Shape sh) {
  const int tile = 64 * sh.nw;
  std::vector<BatchInst> inst(p->n_inst);
  std::vector<FinStage> fin(std::max(1, p->total_stages), FinStage{0, 0, 0, 0, 0, 0, 0, 0});
  std::vector<BatchItem> items;
  std::vector<double> cost;
  size_t part = 0, circ = 0;
  for (int k = 0; k < p->n_inst; ++k) {
    const psdf_batch_desc& d = p->desc[k];
    BatchInst& b = inst[k];
    b.pose_off = d.pose_off; b.N = d.N; b.edge_off = d.edge_off; b.E = d.E;
    b.obst_off = d.obst_off; b.M = d.M; b.m = p->fp[k].m;
    b.nt = (d.M + tile - 1) / tile;
    b.part_off = (int)part;
    b.circ_off = (int)circ;
    circ += d.M;
    // ceil(N / sb) stage blocks of equal length (within one stage), so no
    // block pays an item's setup for a short remainder
    const int nb = (d.N + sh.sb - 1) / sh.sb;
    for (int t = 0; t < d.N; ++t)
      fin[d.pose_off + t] = FinStage{k, b.part_off + t * b.nt, b.nt, d.obst_off, d.M, d.edge_off, d.E, 0};
    part += (size_t)d.N * b.nt;
    if (d.M == 0) continue;
    const double per_edge = (double)d.E / std::max(1, d.M);
    for (int bi = 0; bi < nb; ++bi) {
      const int s0 = (int)((long)bi * d.N / nb), ns = (int)((long)(bi + 1) * d.N / nb) - s0;
      for (int t = 0; t < b.nt; ++t) {
        const int o0 = t * tile, no = std::min(tile, d.M - o0);
        items.push_back(BatchItem{k, s0, ns, o0, no, t});
        cost.push_back((double)ns * no * per_edge);
      }
    }
  }
  // group by footprint size, longest processing time first within a group
  std::vector<int> order(items.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
  auto grp = [&](int i) { return group_of(p->fp[items[i].inst].m); };
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    const int ga = grp(a), gb = grp(b);
    return ga != gb ? ga < gb : cost[a] > cost[b];
  });
  std::vector<BatchItem> sorted(items.size());
  for (size_t i = 0; i < order.size(); ++i) sorted[i] = items[order[i]];

  if (part > p->partial_cap || sorted.size() > p->items_cap)
    return set_error(PSDF_EINVAL, "internal: plan capacity exceeded");
  hipError_t err = hipMemcpy(p->d_inst, inst.data(), inst.size() * sizeof(BatchInst),
                             hipMemcpyHostToDevice);
  if (err == hipSuccess)
    err = hipMemcpy(p->d_fin, fin.data(), fin.size() * sizeof(FinStage), hipMemcpyHostToDevice);
  if (err == hipSuccess && !sorted.empty())
    err = hipMemcpy(p->d_items, sorted.data(), sorted.size() * sizeof(BatchItem),
                    hipMemcpyHostToDevice);
  if (err != hipSuccess) return hip_status(err);
  p->shape = sh;
  p->n_items = (int)sorted.size();
  p->groups.clear();
  for (size_t i = 0; i < order.size();) {
    const int g = grp(order[i]);
    size_t j = i;
    while (j < order.size() && grp(order[j]) == g) ++j;
    const int mf = kGroupMF[g];
    const int per_cu = occupancy(mf, p->mi_class, sh.nw);
    const int count = (int)(j - i);
    const int grid = sh.direct ? count : std::max(1, std::min(count, per_cu * p->cu));
    p->groups.push_back({mf, (int)i, count, grid, 0});
    i = j;
  }
  // lanes: the groups, largest estimated work first, each to the lane with
  // the least work so far (at most kLanes: a process gets a few hardware
  // queues, and streams beyond them share a queue, which serialises their
  // launches behind one another's whole kernels)
  {
    std::vector<double> gcost(p->groups.size(), 0.0);
    for (size_t k = 0; k < p->groups.size(); ++k)
      for (int i = p->groups[k].start; i < p->groups[k].start + p->groups[k].count; ++i)
        gcost[k] += cost[order[i]];
    std::vector<int> by(p->groups.size());
    for (size_t k = 0; k < by.size(); ++k) by[k] = (int)k;
    std::stable_sort(by.begin(), by.end(), [&](int a, int b) { return gcost[a] > gcost[b]; });
    p->n_lanes = std::max(1, std::min((int)p->groups.size(), kLanes));
    std::vector<double> load(p->n_lanes, 0.0);
    std::vector<psdf_batch_plan::Group> lanes;
    for (int k : by) {
      const int l = (int)(std::min_element(load.begin(), load.end()) - load.begin());
      load[l] += gcost[k];
      psdf_batch_plan::Group g = p->groups[k];
      g.lane = l;
      lanes.push_back(g);
    }
    // launch order: lane by lane, each lane's groups largest first
    std::stable_sort(lanes.begin(), lanes.end(),
                     [](const psdf_batch_plan::Group& a, const psdf_batch_plan::Group& b) {
                       return a.lane < b.lane;
                     });
    p->groups = lanes;
  }
  free_graph(p);
  return PSDF_OK;
}

BatchArgs make_args(psdf_batch_plan* p, const float* poses, const float* ax, const float* ay,
                    const float* bx, const float* by, const int32_t* off, float* d, int32_t* edge,
                    int32_t* obst, float* grad, uint64_t* keys) {
  BatchArgs a;
  a.fps = p->d_fp; a.insts = p->d_inst; a.items = p->d_items; a.n_items = p->n_items;
  a.sb = p->shape.sb;
  a.direct = p->shape.direct;
  a.poses = poses; a.ax = ax; a.ay = ay; a.bx = bx; a.by = by; a.off = off;
  a.partial = p->d_partial; a.aux = p->d_partial + p->partial_cap;
  a.ctrl = p->d_ctrl;   // per-group slices set by enqueue
  a.d = d; a.edge = edge; a.obst = obst; a.grad = grad; a.keys = keys;
  return a;
}

// One wave per stage (global row g): the stage's winning key, from the
// minimum of its partial row (partial non-null: the winning column's aux
// word carries the winner's global edge range) or from keys[g] (the screened
// path: the range from the offsets); then the winner adjoint and the
// outputs.  A stage without a partial column (no obstacle) gets the empty
// key and the empty-set result.  Block 0 also clears ctrl[0..n_ctrl), the
// item (or screening) counters of the launches before it on the stream, and
// opens the n_inst horizon lists for the next screened call (count 0, bound
// +inf).
//
// The kernel is latency-bound (one wave per stage, a few waves per CU), so
// its loads are issued in as few dependent rounds as the data allows: the
// stage record, pose and key first; then the footprint, the partial row
// (up to four keys per lane in flight) or the obstacle's offsets; then the
// winning column's aux word (a partial row's keys are distinct, each
// column's obstacle indices being its own, so the column is unique); then
// the winner's edges.
constexpr int kFinKeys = 4;   // partial keys per lane per round

// One 64-lane work-group per stage: g = blockIdx.x, uniform.
__global__ __launch_bounds__(64) void batch_finish_kernel(
    const FpConst* __restrict__ fps, const FinStage* __restrict__ fin, int S,
    const float* __restrict__ poses, const float* __restrict__ ax, const float* __restrict__ ay,
    const float* __restrict__ bx, const float* __restrict__ by, const int* __restrict__ off,
    const uint64_t* __restrict__ partial, const uint64_t* __restrict__ aux,
    uint64_t* __restrict__ keys, float* __restrict__ d, int* __restrict__ edge,
    int* __restrict__ obst, float* __restrict__ grad, unsigned* __restrict__ ctrl, int n_ctrl,
    int* __restrict__ hcount, uint32_t* __restrict__ hrest, int n_inst) {
  __shared__ FpLds fl;
  __shared__ WinnerLds wl;
  const int lane = threadIdx.x;
  const int g = blockIdx.x;
  if (g < S) {
    // round 1: the record (written before the launch: scalar loads), pose, key
    typedef const __attribute__((address_space(4))) FinStage FinC;
    const FinStage& R = *(const FinStage*)((FinC*)fin + g);
    const float* p = poses + 3 * g;
    const float px = p[0], py = p[1], th = p[2];
    uint64_t key = partial ? kEmptyKey : keys[g];
    // round 2: footprint, partial keys or offsets
    const FpConst& F = fp_const(fps, R.inst);
    stage_footprint(fl, F);
    int e0 = 0, mi = 0;
    bool valid;
    if (partial) {
      const uint64_t* prow = partial + R.row;
      int col = 0;
      for (int j0 = 0; j0 < R.nt; j0 += 64 * kFinKeys) {
        uint64_t k[kFinKeys];
#pragma unroll
        for (int u = 0; u < kFinKeys; ++u) {
          const int j = j0 + 64 * u + lane;
          k[u] = j < R.nt ? prow[j] : kEmptyKey;
        }
#pragma unroll
        for (int u = 0; u < kFinKeys; ++u)
          if (k[u] < key) { key = k[u]; col = j0 + 64 * u + lane; }
      }
      const uint64_t kmin = wave_min_u64(key);
      const int first = __ffsll((unsigned long long)__ballot(key == kmin)) - 1;
      col = (int)lane_u32((uint32_t)col, first);
      key = kmin;
      // round 3: the winning column's aux word
      const uint64_t a = key != kEmptyKey ? aux[R.row + col] : 0ull;
      e0 = (int)(uint32_t)(a >> 32);
      mi = (int)(uint32_t)(a & 0xffffffffu);
      valid = key != kEmptyKey && (key >> 32) != 0 && mi >= 1 && mi <= kMaxObst;
    } else {
      valid = key_range(key, off, R.obst_off, R.M, R.edge_off, R.E, e0, mi);
    }
    float sn, cs;
    sincosf(th, &sn, &cs);
    wave_sync();
    // last round: the winner's edges
    write_stage(F, fl, wl, ax, ay, bx, by, key, valid, e0, mi, R.edge_off, cs, sn, px, py, g, keys,
                d, edge, obst, grad);
  }
  if (blockIdx.x == 0) {
    if ((int)threadIdx.x < n_ctrl) ctrl[threadIdx.x] = 0u;
    for (int i = threadIdx.x; i < n_inst; i += blockDim.x) {
      hcount[i] = 0;
      hrest[i] = 0xffffffffu;
    }
  }
}

int run(psdf_batch_plan* p, const float* poses, const float* ax, const float* ay,
        const float* bx, const float* by, const int32_t* off, float* d, int32_t* edge,
        int32_t* obst, float* grad, uint64_t* keys, hipStream_t stream, bool use_graph) {
  if (p->total_stages == 0) return PSDF_OK;
  const BatchArgs a = make_args(p, poses, ax, ay, bx, by, off, d, edge, obst, grad, keys);
  // timed: events recorded by each batch-kernel dispatch itself (eager
  // calls only; a captured graph is timed as a whole)
  auto enqueue = [&](hipStream_t st, bool timed) -> hipError_t {
    // the groups write disjoint partial rows and count their items on
    // counters of their own, so they run concurrently (their tails overlap)
    const int ng = (int)p->groups.size(), nl = p->n_lanes;
    hipError_t err = hipSuccess;
    if (nl > 1 && !p->side[nl - 2]) return hipErrorInvalidValue;   // created with the plan
    if (nl > 1) {
      err = hipEventRecord(p->ev[0], st);
      for (int l = 1; l < nl && err == hipSuccess; ++l)
        err = hipStreamWaitEvent(p->side[l - 1], p->ev[0], 0);
    }
    for (int k = 0; k < ng && err == hipSuccess; ++k) {
      const auto& g = p->groups[k];
      BatchArgs ga = a;
      ga.items = a.items + g.start;
      ga.n_items = g.count;
      ga.ctrl = a.ctrl + group_of(g.mf);
      hipStream_t gs = g.lane == 0 ? st : p->side[g.lane - 1];
      hipEvent_t ev0 = nullptr, ev1 = nullptr;
      if (!timed || !timer_kernel_events(&ev0, &ev1)) ev0 = ev1 = nullptr;
      err = launch_batch(g.mf, p->mi_class, p->shape.nw, g.grid, ga, gs, ev0, ev1);
    }
    for (int l = 1; l < nl && err == hipSuccess; ++l) {
      err = hipEventRecord(p->ev[l], p->side[l - 1]);
      if (err == hipSuccess) err = hipStreamWaitEvent(st, p->ev[l], 0);
    }
    if (err != hipSuccess) return err;
    batch_finish_kernel<<<p->total_stages, 64, 0, st>>>(
        p->d_fp, p->d_fin, p->total_stages, poses, ax, ay, bx, by, off, a.partial, a.aux, keys, d,
        edge, obst, grad, p->d_ctrl, kGroups, nullptr, nullptr, 0);
    return hipGetLastError();
  };
  if (!use_graph) return hip_status(enqueue(stream, true));
  const std::vector<const void*> ptrs = {poses, ax, ay, bx, by, off, d, edge, obst, grad, keys};
  if (!p->exec || p->bound != ptrs) {
    free_graph(p);
    hipError_t err = hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal);
    if (err != hipSuccess) return hip_status(err);
    err = enqueue(p->cap_stream, false);
    hipGraph_t g = nullptr;
    hipError_t err2 = hipStreamEndCapture(p->cap_stream, &g);
    if (err != hipSuccess) { if (g) (void)hipGraphDestroy(g); return hip_status(err); }
    if (err2 != hipSuccess) return hip_status(err2);
    p->graph = g;
    err = hipGraphInstantiate(&p->exec, g, nullptr, nullptr, 0);
    if (err != hipSuccess) { free_graph(p); return hip_status(err); }
    p->bound = ptrs;
  }
  timer_begin(stream);
  hipError_t err = hipGraphLaunch(p->exec, stream);
  timer_end(stream);
  return hip_status(err);
}

hipError_t launch_screen(int mf, int mi_class, int grid, const ScreenArgs& a, hipStream_t st) {
  switch (mf) {
    case 3: return launch_screen_mf<3>(mi_class, grid, a, st);
    case 4: return launch_screen_mf<4>(mi_class, grid, a, st);
    case 5: return launch_screen_mf<5>(mi_class, grid, a, st);
    case 6: return launch_screen_mf<6>(mi_class, grid, a, st);
    case 7: return launch_screen_mf<7>(mi_class, grid, a, st);
    case 8: return launch_screen_mf<8>(mi_class, grid, a, st);
    default: return launch_screen_mf<16>(mi_class, grid, a, st);
  }
}

hipError_t launch_screen_bound(int mf, int mi_class, int grid, const ScreenArgs& a,
                               hipStream_t st) {
  switch (mf) {
    case 3: return launch_screen_bound_mf<3>(mi_class, grid, a, st);
    case 4: return launch_screen_bound_mf<4>(mi_class, grid, a, st);
    case 5: return launch_screen_bound_mf<5>(mi_class, grid, a, st);
    case 6: return launch_screen_bound_mf<6>(mi_class, grid, a, st);
    case 7: return launch_screen_bound_mf<7>(mi_class, grid, a, st);
    case 8: return launch_screen_bound_mf<8>(mi_class, grid, a, st);
    default: return launch_screen_bound_mf<16>(mi_class, grid, a, st);
  }
}

hipError_t launch_fallback(int mf, int mi_class, int grid, int tiles, const ScreenArgs& a,
                           hipStream_t st) {
  switch (mf) {
    case 3: return launch_fallback_mf<3>(mi_class, grid, tiles, a, st);
    case 4: return launch_fallback_mf<4>(mi_class, grid, tiles, a, st);
    case 5: return launch_fallback_mf<5>(mi_class, grid, tiles, a, st);
    case 6: return launch_fallback_mf<6>(mi_class, grid, tiles, a, st);
    case 7: return launch_fallback_mf<7>(mi_class, grid, tiles, a, st);
    case 8: return launch_fallback_mf<8>(mi_class, grid, tiles, a, st);
    default: return launch_fallback_mf<16>(mi_class, grid, tiles, a, st);
  }
}

}  // namespace

hipError_t launch_labels(const FpConst* fps, const BatchInst* insts, const int* stage_inst,
                         const float* poses, const float* ax, const float* ay, const float* bx,
                         const float* by, const int* stage, const int* edge, int n, int S, float* X,
                         float* T, hipStream_t st);

}  // namespace psdf

extern "C" {

// The screened call of either form: the horizon pass, per footprint-size
// group the screening kernel (ranked top-K with the network or the edge
// distance, or the bound-threshold form) and the fallback of the stages
// that fail the certificate, then (ranked forms) the finish kernel.  The
// bound form has no finish launch: its screen kernel writes the outputs of
// the stages it certifies, the fallback those of the others, and the last
// fallback launch reopens the horizon lists.
static int screened_run(psdf_batch_plan* p, bool bound, const float* theta, int32_t pool,
                        int32_t topk, const float* poses, const float* ax, const float* ay,
                        const float* bx, const float* by, const int32_t* off, float* d,
                        int32_t* edge, int32_t* obst, float* grad, uint64_t* keys,
                        int32_t* stage_cand, int32_t* stage_cert, uint64_t* cand_keys,
                        hipStream_t stream) {
  clear_error();
  if (!p) return set_error(PSDF_EINVAL, "plan is NULL");
  if (!bound && (pool < 1 || pool > kPoolCap || topk < 1))
    return set_error(PSDF_EINVAL, "pool = %d (1..%d), topk = %d (>= 1)", pool, kPoolCap, topk);
  if (p->max_M > kScreenMaxM)
    return set_error(PSDF_ETOOBIG, "an instance has %d obstacles; screening supports %d", p->max_M,
                     kScreenMaxM);
  if (p->n_inst > 65535)
    return set_error(PSDF_ETOOBIG, "%d instances; screening supports 65535", p->n_inst);
  if (p->total_stages == 0) return PSDF_OK;
  if (!poses || !off || !d || !edge || !obst || !grad || !keys)
    return set_error(PSDF_EINVAL, "a pose, offset or output pointer is NULL");
  if (p->max_M > 0 && (!ax || !ay || !bx || !by)) return set_error(PSDF_EINVAL, "an edge array is NULL");
  if (bound) theta = nullptr;
  const float4* circ = nullptr;
  if (p->circ_staged) {
    const void* src[5] = {ax, ay, bx, by, off};
    for (int k = 0; k < 5; ++k)
      if (src[k] != p->circ_src[k])
        return set_error(PSDF_EINVAL,
                         "the edge arrays differ from the ones psdf_batch_stage took the circles "
                         "from (stage again, or psdf_batch_unstage)");
    circ = p->d_circ;
  }
  ScreenArgs a;
  a.rows = circ ? p->d_rows : nullptr;
  a.fps = p->d_fp; a.insts = p->d_inst; a.stage_inst = p->d_stage_inst;
  a.poses = poses; a.ax = ax; a.ay = ay; a.bx = bx; a.by = by; a.off = off;
  a.hlist = p->d_hlist; a.hcount = p->d_hcount; a.hrest = p->d_hrest;
  a.theta = theta; a.frag = p->d_frag; a.pool = pool; a.topk = topk; a.keys = keys;
  a.stage_cand = stage_cand; a.stage_cert = stage_cert; a.cand_keys = cand_keys;
  a.finish = bound ? 1 : 0;
  a.d = d; a.edge = edge; a.obst = obst; a.grad = grad;
  a.reset_n = 0; a.reset_hcount = p->d_hcount; a.reset_hrest = p->d_hrest;
  timer_begin(stream);
  hipError_t err = hipSuccess;
  if (p->n_inst > 0) {
    // column kHorizonSplit of the grid builds the network's fragment table
    const dim3 grid(kHorizonSplit + (theta ? 1 : 0), p->n_inst);
    if (p->mi_class == 4)
      horizon_kernel<4><<<grid, kScreenThreads, 0, stream>>>(
          p->d_fp, p->d_inst, poses, ax, ay, bx, by, off, circ, p->d_hlist, p->d_hcount,
          p->d_hrest, theta, p->d_frag, p->d_sctrl, 2 * kGroups);
    else if (p->mi_class == 8)
      horizon_kernel<8><<<grid, kScreenThreads, 0, stream>>>(
          p->d_fp, p->d_inst, poses, ax, ay, bx, by, off, circ, p->d_hlist, p->d_hcount,
          p->d_hrest, theta, p->d_frag, p->d_sctrl, 2 * kGroups);
    else
      horizon_kernel<16><<<grid, kScreenThreads, 0, stream>>>(
          p->d_fp, p->d_inst, poses, ax, ay, bx, by, off, circ, p->d_hlist, p->d_hcount,
          p->d_hrest, theta, p->d_frag, p->d_sctrl, 2 * kGroups);
    err = hipGetLastError();
  }
  for (size_t k = 0; k < p->sgroups.size(); ++k) {
    if (err != hipSuccess) break;
    const auto& g = p->sgroups[k];
    ScreenArgs ga = a;
    ga.stages = p->d_stage_list + g.start;
    ga.n_stages = g.count;
    ga.failed = p->d_failed + g.start;
    ga.fdone = p->d_fdone + g.start;
    ga.ctrl = p->d_sctrl + 2 * group_of(g.mf);
    if (bound && k + 1 == p->sgroups.size()) ga.reset_n = p->n_inst;
    err = bound ? launch_screen_bound(g.mf, p->mi_class, g.count, ga, stream)
                : launch_screen(g.mf, p->mi_class, g.count, ga, stream);
    if (err != hipSuccess) break;
    const int grid = std::max(1, std::min(g.count * g.max_tiles, 4 * p->cu));
    err = launch_fallback(g.mf, p->mi_class, grid, g.max_tiles, ga, stream);
    if (err != hipSuccess) break;
  }
  timer_end(stream);
  if (err == hipSuccess && !bound) {
    batch_finish_kernel<<<p->total_stages, 64, 0, stream>>>(
        p->d_fp, p->d_fin, p->total_stages, poses, ax, ay, bx, by, off, nullptr, nullptr, keys, d,
        edge, obst, grad, p->d_sctrl, 2 * kGroups, p->d_hcount, p->d_hrest, p->n_inst);
    err = hipGetLastError();
  }
  return hip_status(err);
}

int psdf_batch_screened(psdf_batch_plan* p, const float* theta, int32_t pool, int32_t topk,
                        const float* poses, const float* ax, const float* ay, const float* bx,
                        const float* by, const int32_t* off, float* d, int32_t* edge,
                        int32_t* obst, float* grad, uint64_t* keys, int32_t* stage_cand,
                        int32_t* stage_cert, uint64_t* cand_keys, hipStream_t stream) {
  return screened_run(p, false, theta, pool, topk, poses, ax, ay, bx, by, off, d, edge, obst,
                      grad, keys, stage_cand, stage_cert, cand_keys, stream);
}

int psdf_batch_screened_bound(psdf_batch_plan* p, const float* poses, const float* ax,
                              const float* ay, const float* bx, const float* by,
                              const int32_t* off, float* d, int32_t* edge, int32_t* obst,
                              float* grad, uint64_t* keys, int32_t* stage_cand,
                              int32_t* stage_cert, uint64_t* cand_keys, hipStream_t stream) {
  return screened_run(p, true, nullptr, 1, 1, poses, ax, ay, bx, by, off, d, edge, obst, grad,
                      keys, stage_cand, stage_cert, cand_keys, stream);
}

int psdf_batch_stage(psdf_batch_plan* p, const float* ax, const float* ay, const float* bx,
                     const float* by, const int32_t* off, hipStream_t stream) {
  clear_error();
  if (!p) return set_error(PSDF_EINVAL, "plan is NULL");
  if (p->max_M > kScreenMaxM)
    return set_error(PSDF_ETOOBIG, "an instance has %d obstacles; screening supports %d", p->max_M,
                     kScreenMaxM);
  if (p->n_inst > 65535)
    return set_error(PSDF_ETOOBIG, "%d instances; screening supports 65535", p->n_inst);
  if (p->sum_M > 0) {
    if (!off) return set_error(PSDF_EINVAL, "obst_off is NULL");
    if (!ax || !ay || !bx || !by) return set_error(PSDF_EINVAL, "an edge array is NULL");
    hipError_t err = hipSuccess;
    if (!p->d_circ) {
      err = hipMalloc(&p->d_circ, p->sum_M * sizeof(float4));
      if (err != hipSuccess) p->d_circ = nullptr;
    }
    if (err == hipSuccess && !p->d_rows) {
      err = hipMalloc(&p->d_rows, p->sum_M * (size_t)(40 * p->mi_class + 16));
      if (err != hipSuccess) p->d_rows = nullptr;
    }
    if (err != hipSuccess) return hip_status(err);
    const dim3 grid((p->max_M + 255) / 256, p->n_inst);
#define PSDF_STAGE_BATCH(MI)                                                               \
  stage_batch_kernel<MI><<<grid, 256, 0, stream>>>(p->d_fp, p->d_inst, ax, ay, bx, by, off, \
                                                   p->d_circ, p->d_rows)
    if (p->mi_class == 4) PSDF_STAGE_BATCH(4);
    else if (p->mi_class == 8) PSDF_STAGE_BATCH(8);
    else PSDF_STAGE_BATCH(16);
#undef PSDF_STAGE_BATCH
    err = hipGetLastError();
    if (err != hipSuccess) return hip_status(err);
  }
  p->circ_staged = true;
  const void* src[5] = {ax, ay, bx, by, off};
  for (int k = 0; k < 5; ++k) p->circ_src[k] = src[k];
  return PSDF_OK;
}

int psdf_batch_unstage(psdf_batch_plan* p) {
  clear_error();
  if (!p) return set_error(PSDF_EINVAL, "plan is NULL");
  p->circ_staged = false;
  return PSDF_OK;
}

int psdf_screen_labels(const psdf_batch_plan* p, const float* poses, const float* ax,
                       const float* ay, const float* bx, const float* by, const int32_t* stage,
                       const int32_t* edge, int32_t n, float* X, float* T, hipStream_t stream) {
  clear_error();
  if (!p) return set_error(PSDF_EINVAL, "plan is NULL");
  if (n < 0) return set_error(PSDF_EINVAL, "n = %d", n);
  if (n == 0) return PSDF_OK;
  if (!poses || !ax || !ay || !bx || !by || !stage || !edge || !X || !T)
    return set_error(PSDF_EINVAL, "NULL argument");
  return hip_status(launch_labels(p->d_fp, p->d_inst, p->d_stage_inst, poses, ax, ay, bx, by,
                                  stage, edge, n, p->total_stages, X, T, stream));
}


void psdf_batch_plan_destroy(psdf_batch_plan* p) {
  if (!p) return;
  int cur = 0;
  (void)hipGetDevice(&cur);
  (void)hipSetDevice(p->device);
  free_graph(p);
  if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
  for (hipStream_t s : p->side)
    if (s) (void)hipStreamDestroy(s);
  for (hipEvent_t e : p->ev)
    if (e) (void)hipEventDestroy(e);
  (void)hipFree(p->d_fp);
  (void)hipFree(p->d_inst);
  (void)hipFree(p->d_items);
  (void)hipFree(p->d_partial);
  (void)hipFree(p->d_ctrl);
  (void)hipFree(p->d_stage_inst);
  (void)hipFree(p->d_fin);
  (void)hipFree(p->d_stage_list);
  (void)hipFree(p->d_failed);
  (void)hipFree(p->d_fdone);
  (void)hipFree(p->d_sctrl);
  (void)hipFree(p->d_hlist);
  (void)hipFree(p->d_circ);
  (void)hipFree(p->d_rows);
  (void)hipFree(p->d_frag);
  (void)hipFree(p->d_hcount);
  (void)hipFree(p->d_hrest);
  (void)hipSetDevice(cur);
  delete p;
}

int psdf_batch_plan_create(psdf_batch_plan** out, const psdf_batch_desc* desc, int32_t n_inst,
                           const float* footprints, int32_t mbar, const psdf_params* params,
                           int32_t flags) {
  clear_error();
  if (!out) return set_error(PSDF_EINVAL, "plan is NULL");
  *out = nullptr;
  if (n_inst < 0 || (n_inst > 0 && (!desc || !footprints)))
    return set_error(PSDF_EINVAL, "n_inst = %d with a NULL descriptor or footprint array", n_inst);
  if (mbar < 1 || mbar > kMaxObst) return set_error(PSDF_ETOOBIG, "mbar = %d, 1..%d allowed", mbar, kMaxObst);
  psdf_batch_plan* p = new psdf_batch_plan();
  p->n_inst = n_inst;
  p->mi_class = obst_class(mbar);
  p->flags = flags;
  p->desc.assign(desc, desc + n_inst);
  p->fp.resize(n_inst);
  size_t part_max = 0, items_max = 0;
  long stages = 0;
  for (int k = 0; k < n_inst; ++k) {
    const psdf_batch_desc& d = desc[k];
    if (d.N < 0 || d.E < 0 || d.M < 0 || d.pose_off < 0 || d.edge_off < 0 || d.obst_off < 0 ||
        d.fp_off < 0) {
      delete p;
      return set_error(PSDF_EINVAL, "instance %d: negative size or offset", k);
    }
    int rc = prepare_footprint(footprints + 2 * (size_t)d.fp_off, d.m, params, &p->fp[k]);
    if (rc) {
      std::string msg = last_error();
      delete p;
      return set_error(rc, "instance %d: %s", k, msg.c_str());
    }
    stages += d.N;
    const size_t nt64 = (size_t)(d.M + 63) / 64;
    part_max += (size_t)d.N * nt64;
    items_max += (size_t)d.N * nt64;
  }
  if (stages > 0x7fffffffL) { delete p; return set_error(PSDF_ETOOBIG, "too many stages"); }
  // partial rows are addressed with 32-bit offsets (at most one 64-obstacle
  // tile per column)
  if (part_max > 0x7fffffffu) { delete p; return set_error(PSDF_ETOOBIG, "too many partial keys"); }
  // the instances' stage rows tile [0, sum N): each row belongs to exactly
  // one instance (in range and disjoint; the counts then cover every row)
  {
    std::vector<int> owner((size_t)stages, -1);
    for (int k = 0; k < n_inst; ++k) {
      const psdf_batch_desc& d = desc[k];
      if ((long)d.pose_off + d.N > stages) {
        delete p;
        return set_error(PSDF_EINVAL, "instance %d: stage rows [%d, %ld) beyond the %ld packed rows",
                         k, d.pose_off, (long)d.pose_off + d.N, stages);
      }
      for (int t = 0; t < d.N; ++t) {
        int& o = owner[(size_t)d.pose_off + t];
        if (o >= 0) {
          delete p;
          return set_error(PSDF_EINVAL, "instance %d: stage row %d also belongs to instance %d", k,
                           d.pose_off + t, o);
        }
        o = k;
      }
    }
  }
  p->total_stages = (int)stages;
  hipError_t err = hipGetDevice(&p->device);
  int cu = 0;
  if (err == hipSuccess) err = hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, p->device);
  p->cu = cu > 0 ? cu : 256;
  p->partial_cap = std::max<size_t>(1, part_max);
  p->items_cap = std::max<size_t>(1, items_max);
  if (err == hipSuccess) err = hipMalloc(&p->d_fp, std::max(1, n_inst) * sizeof(FpConst));
  if (err == hipSuccess) err = hipMalloc(&p->d_inst, std::max(1, n_inst) * sizeof(BatchInst));
  if (err == hipSuccess) err = hipMalloc(&p->d_items, p->items_cap * sizeof(BatchItem));
  if (err == hipSuccess) err = hipMalloc(&p->d_partial, 2 * p->partial_cap * sizeof(uint64_t));
  if (err == hipSuccess) err = hipMalloc(&p->d_ctrl, kGroups * sizeof(unsigned));
  if (err == hipSuccess) err = hipMemset(p->d_ctrl, 0, kGroups * sizeof(unsigned));
  if (err == hipSuccess && n_inst > 0)
    err = hipMemcpy(p->d_fp, p->fp.data(), n_inst * sizeof(FpConst), hipMemcpyHostToDevice);
  if (err == hipSuccess) err = hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking);
  // side streams and events for the concurrent footprint-size groups: one
  // stream per lane after the first, one event per lane
  {
    bool present[kGroups] = {};
    for (int k = 0; k < n_inst; ++k) present[group_of(p->fp[k].m)] = true;
    int ng = 0;
    for (bool b : present) ng += b ? 1 : 0;
    const int nl = std::min(ng, kLanes);
    for (int k = 0; k + 1 < nl && err == hipSuccess; ++k)
      err = hipStreamCreateWithFlags(&p->side[k], hipStreamNonBlocking);
    for (int k = 0; k < nl && nl > 1 && err == hipSuccess; ++k)
      err = hipEventCreateWithFlags(&p->ev[k], hipEventDisableTiming);
  }
  // screening tables
  if (err == hipSuccess) {
    const int S = std::max(1, p->total_stages);
    std::vector<int> stage_inst(S, 0), circ_off(std::max(1, n_inst), 0);
    std::vector<int4> list;
    list.reserve(S);
    int circ = 0;
    for (int k = 0; k < n_inst; ++k) {
      for (int t = 0; t < desc[k].N; ++t) stage_inst[desc[k].pose_off + t] = k;
      p->max_M = std::max(p->max_M, desc[k].M);
      circ_off[k] = circ;   // as build_items: the instances' M in order
      circ += desc[k].M;
    }
    for (int g = 0; g < kGroups; ++g) {
      const int start = (int)list.size();
      int max_tiles = 1;
      for (int k = 0; k < n_inst; ++k)
        if (group_of(p->fp[k].m) == g) {
          for (int t = 0; t < desc[k].N; ++t)
            list.push_back(make_int4(desc[k].pose_off + t, k, circ_off[k], desc[k].M));
          max_tiles = std::max(max_tiles, (desc[k].M + 255) / 256);
        }
      if ((int)list.size() > start)
        p->sgroups.push_back({kGroupMF[g], start, (int)list.size() - start, max_tiles});
    }
    size_t sumM = 0;
    for (int k = 0; k < n_inst; ++k) sumM += desc[k].M;
    p->sum_M = sumM;
    err = hipMalloc(&p->d_hlist, std::max<size_t>(1, sumM) * sizeof(float4));
    if (err == hipSuccess) err = hipMalloc(&p->d_frag, (size_t)kFragWords * 64 * sizeof(uint4));
    if (err == hipSuccess)
      err = hipMalloc(&p->d_hcount, std::max<size_t>(1, (size_t)n_inst) * sizeof(int));
    if (err == hipSuccess)
      err = hipMalloc(&p->d_hrest, std::max<size_t>(1, (size_t)n_inst) * sizeof(uint32_t));
    // horizon lists open (count 0, excluded bound +inf); every screened call
    // leaves them so
    if (err == hipSuccess)
      err = hipMemset(p->d_hcount, 0, std::max<size_t>(1, (size_t)n_inst) * sizeof(int));
    if (err == hipSuccess)
      err = hipMemset(p->d_hrest, 0xff, std::max<size_t>(1, (size_t)n_inst) * sizeof(uint32_t));
    if (err == hipSuccess) err = hipMalloc(&p->d_stage_inst, S * sizeof(int));
    if (err == hipSuccess) err = hipMalloc(&p->d_fin, S * sizeof(FinStage));
    if (err == hipSuccess) err = hipMalloc(&p->d_stage_list, S * sizeof(int4));
    if (err == hipSuccess) err = hipMalloc(&p->d_failed, S * sizeof(int));
    if (err == hipSuccess) err = hipMalloc(&p->d_fdone, S * sizeof(int));
    if (err == hipSuccess) err = hipMalloc(&p->d_sctrl, 2 * kGroups * sizeof(unsigned));
    if (err == hipSuccess) err = hipMemset(p->d_sctrl, 0, 2 * kGroups * sizeof(unsigned));
    if (err == hipSuccess)
      err = hipMemcpy(p->d_stage_inst, stage_inst.data(), S * sizeof(int), hipMemcpyHostToDevice);
    if (err == hipSuccess && !list.empty())
      err = hipMemcpy(p->d_stage_list, list.data(), list.size() * sizeof(int4), hipMemcpyHostToDevice);
  }
  if (err != hipSuccess) {
    int rc = hip_status(err);
    psdf_batch_plan_destroy(p);
    return rc;
  }
  Shape sh{32, 1, 1};
  if (!cache_find(signature(*p), &sh)) {
    // heuristic: one-wave work-groups, one per item (64-obstacle tiles,
    // dispatched directly), stage blocks of up to 32 stages cut evenly,
    // halved until the items cover the chip about eight deep.  On c5 (64 x
    // 50 stages x 16384 obstacles) that is 25-stage blocks, 32768 items:
    // 0.572 ms a call against 0.622 ms for 16-stage blocks of 256-obstacle
    // tiles on a persistent grid (sweep of stage block x tile x dispatch).
    auto items = [&](int sb) {
      double n = 0.0;
      for (const auto& d : p->desc) n += (double)((d.N + sb - 1) / sb) * ((d.M + 63) / 64);
      return n;
    };
    while (sh.sb > 1 && items(sh.sb) < 8.0 * p->cu) sh.sb /= 2;
  }
  int rc = build_items(p, sh);
  if (rc) { psdf_batch_plan_destroy(p); return rc; }
  *out = p;
  return PSDF_OK;
}

int psdf_batch(psdf_batch_plan* p, const float* poses, const float* ax, const float* ay,
               const float* bx, const float* by, const int32_t* off, float* d, int32_t* edge,
               int32_t* obst, float* grad, uint64_t* keys, hipStream_t stream) {
  clear_error();
  if (!p) return set_error(PSDF_EINVAL, "plan is NULL");
  if (p->total_stages > 0 && (!poses || !off || !d || !edge || !obst || !grad || !keys))
    return set_error(PSDF_EINVAL, "a pose, offset or output pointer is NULL");
  if (p->n_items > 0 && (!ax || !ay || !bx || !by)) return set_error(PSDF_EINVAL, "an edge array is NULL");
  return run(p, poses, ax, ay, bx, by, off, d, edge, obst, grad, keys, stream,
             (p->flags & PSDF_BATCH_GRAPH) != 0);
}

int psdf_batch_autotune(psdf_batch_plan* p, const float* poses, const float* ax, const float* ay,
                        const float* bx, const float* by, const int32_t* off, float* d,
                        int32_t* edge, int32_t* obst, float* grad, uint64_t* keys,
                        hipStream_t stream, float* best_ms) {
  clear_error();
  if (!p) return set_error(PSDF_EINVAL, "plan is NULL");
  if (!(p->flags & PSDF_BATCH_AUTOTUNE)) return set_error(PSDF_EINVAL, "plan built without PSDF_BATCH_AUTOTUNE");
  if (p->n_items == 0) return PSDF_OK;
  hipEvent_t e0, e1;
  hipError_t err = hipEventCreate(&e0);
  if (err == hipSuccess) err = hipEventCreate(&e1);
  if (err != hipSuccess) return hip_status(err);
  const int sbs[] = {1, 2, 4, 8, 16, 32, 64};
  constexpr int kSb = sizeof(sbs) / sizeof(sbs[0]);
  constexpr int kCand = 4 * kSb;   // stage block x work-group width x dispatch
  const int nws[] = {1, 4};
  auto shape_of = [&](int cand) {
    return Shape{sbs[cand % kSb], nws[(cand / kSb) % 2], cand / (2 * kSb)};
  };
  // Each candidate is timed as kBurst back-to-back calls between one event
  // pair (the steady state a caller's loop sees, not an isolated call),
  // after one untimed call; two rounds over all candidates, the better of
  // each candidate's two bursts counting, so that the clock's ramp under
  // load does not favour the candidates timed last.  Ten untimed calls of
  // the plan's shape warm the GPU first.
  constexpr int kBurst = 3, kRounds = 2;
  float t_best[kCand];
  for (float& t : t_best) t = INFINITY;
  int rc = PSDF_OK;
  for (int w = 0; w < 10 && rc == PSDF_OK; ++w)
    rc = run(p, poses, ax, ay, bx, by, off, d, edge, obst, grad, keys, stream, false);
  for (int round = 0; round < kRounds && rc == PSDF_OK; ++round)
    for (int cand = 0; cand < kCand && rc == PSDF_OK; ++cand) {
      rc = build_items(p, shape_of(cand));
      if (rc) break;
      rc = run(p, poses, ax, ay, bx, by, off, d, edge, obst, grad, keys, stream, false);
      if (rc) break;
      err = hipEventRecord(e0, stream);
      for (int k = 0; k < kBurst && err == hipSuccess && rc == PSDF_OK; ++k)
        rc = run(p, poses, ax, ay, bx, by, off, d, edge, obst, grad, keys, stream, false);
      if (rc) break;
      if (err == hipSuccess) err = hipEventRecord(e1, stream);
      if (err == hipSuccess) err = hipEventSynchronize(e1);
      float ms = 0.f;
      if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
      if (err != hipSuccess) { rc = hip_status(err); break; }
      t_best[cand] = std::min(t_best[cand], ms / kBurst);
    }
  float best = INFINITY;
  Shape best_sh = p->shape;
  for (int cand = 0; cand < kCand; ++cand)
    if (t_best[cand] < best) { best = t_best[cand]; best_sh = shape_of(cand); }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return rc;
  rc = build_items(p, best_sh);
  if (rc) return rc;
  cache_store(signature(*p), best_sh);
  rc = run(p, poses, ax, ay, bx, by, off, d, edge, obst, grad, keys, stream, false);
  if (best_ms) *best_ms = best;
  return rc;
}

int psdf_batch_set_shape(psdf_batch_plan* p, int32_t stages_per_item, int32_t obstacles_per_tile,
                         int32_t direct) {
  clear_error();
  if (!p) return set_error(PSDF_EINVAL, "plan is NULL");
  if (stages_per_item < 1 || stages_per_item > kMaxStageBlock ||
      (obstacles_per_tile != 64 && obstacles_per_tile != 256) || (direct != 0 && direct != 1))
    return set_error(PSDF_EINVAL, "shape sb=%d tile=%d direct=%d (sb 1..%d, tile 64 or 256, direct 0 or 1)",
                     stages_per_item, obstacles_per_tile, direct, kMaxStageBlock);
  return build_items(p, Shape{stages_per_item, obstacles_per_tile / 64, direct});
}

int psdf_batch_plan_info(const psdf_batch_plan* p, int32_t* stages_per_item,
                         int32_t* obstacles_per_tile, int32_t* n_items, int32_t* grid,
                         int32_t* direct) {
  clear_error();
  if (!p) return set_error(PSDF_EINVAL, "plan is NULL");
  if (stages_per_item) *stages_per_item = p->shape.sb;
  if (obstacles_per_tile) *obstacles_per_tile = 64 * p->shape.nw;
  if (n_items) *n_items = p->n_items;
  if (direct) *direct = p->shape.direct;
  if (grid) {
    int g = 0;
    for (const auto& gr : p->groups) g = std::max(g, gr.grid);
    *grid = g;
  }
  return PSDF_OK;
}

}  // extern "C"
