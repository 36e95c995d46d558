// Host model of the screening kernels' work-group index arithmetic, built
// with the address and undefined-behaviour sanitizers by
// tests/test_screen_index_model.py (test infrastructure only).
//
// It restates, for one 256-lane work-group executed phase by phase on the
// host, every LDS and list index that psdf_screen.hpp and psdf_batch.hip
// compute: the work-group reductions (block_reduce and block_scan_min,
// each call site on a slot region of its own, since no barrier follows
// their reads; block_threshold with its alternating halves of the reduction
// array), the pool and candidate compactions of screen_kernel, the seed and
// candidate compaction of screen_bound_kernel (list entries held in
// registers, then the tail re-read), and the horizon list append of
// horizon_kernel.  Every array has the kernel's size and checks its
// index; the sweep covers every pool size the ABI allows (1..512), top-K
// from 1 to past the pool's slot count, horizon lists of 0..2048 entries,
// the three edge classes, and key sets with ties, unused slots and -inf.
#include <algorithm>
#include <cassert>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <vector>

namespace {

constexpr int kThreads = 256, kWaves = 4;
constexpr int kStageKeys = 8, kHorizonCap = kThreads * kStageKeys;   // 2048
constexpr int kPoolCap = 512, kFeatSlots = 1024, kBoundCap = 512;
constexpr int kHorizonPool = 512, kHorizonSplit = 16, kHorizonKeys = 4;
constexpr uint32_t kUnused = 0xffffffffu;

long g_checks = 0;

[[noreturn]] void fail(const char* what, long i, long n) {
  std::fprintf(stderr, "index out of range: %s[%ld], size %ld\n", what, i, n);
  std::abort();
}

// An LDS / register array of the kernel's size with a checked index.
template <class T, int N>
struct Arr {
  T v[N];
  const char* name;
  explicit Arr(const char* nm) : name(nm) { std::memset(v, 0, sizeof v); }
  T& operator[](long i) {
    ++g_checks;
    if (i < 0 || i >= N) fail(name, i, N);
    return v[i];
  }
};

uint32_t orderable(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  if (f != f) return 0u;
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
float from_orderable(uint32_t k) {
  const uint32_t u = (k & 0x80000000u) ? (k & 0x7fffffffu) : ~k;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}

// ---- work-group reductions: one value per thread in, wave values written
// by lane 0 of each wave into the call site's slot region (the kernels'
// layout).  No barrier follows the reads, so every call site of a kernel
// must own its words: owner[] records which call site wrote each word in
// the current work-group and fails on a second one.
template <int N>
struct Slots {
  Arr<uint32_t, N> v{"reduction slots"};
  int owner[N];
  Slots() { for (int i = 0; i < N; ++i) owner[i] = -1; }
  uint32_t& put(int i, int site) {
    if (i < 0 || i >= N) fail("reduction slot", i, N);
    if (owner[i] != -1 && owner[i] != site) fail("slot word shared by two call sites", i, N);
    owner[i] = site;
    return v[i];
  }
};

// block_reduce<NM, NS>: minima of mn[i][t] and sums of sm[i][t] over the
// 256 threads, from slot words off + i * kWaves + wave
template <int NM, int NS, int N>
void block_reduce(const uint32_t (*mn)[kThreads], const int (*sm)[kThreads], Slots<N>& rs, int off,
                  int site, uint32_t* mn_out, int* sm_out) {
  for (int w = 0; w < kWaves; ++w) {
    for (int i = 0; i < NM; ++i) {
      uint32_t m = kUnused;
      for (int l = 0; l < 64; ++l) m = mn[i][64 * w + l] < m ? mn[i][64 * w + l] : m;
      rs.put(off + i * kWaves + w, site) = m;
    }
    for (int i = 0; i < NS; ++i) {
      int s = 0;
      for (int l = 0; l < 64; ++l) s += sm[i][64 * w + l];
      rs.put(off + (NM + i) * kWaves + w, site) = (uint32_t)s;
    }
  }
  for (int i = 0; i < NM; ++i) {
    uint32_t r = rs.v[off + i * kWaves];
    for (int w = 1; w < kWaves; ++w) r = rs.v[off + i * kWaves + w] < r ? rs.v[off + i * kWaves + w] : r;
    mn_out[i] = r;
  }
  for (int i = 0; i < NS; ++i) {
    int t = 0;
    for (int w = 0; w < kWaves; ++w) t += (int)rs.v[off + (NM + i) * kWaves + w];
    sm_out[i] = t;
  }
}

// block_scan_min: exclusive prefix per thread of v, its total, and the
// minimum of m; wave totals at off + wave, wave minima at off + kWaves + wave
template <int N>
void block_scan_min(const int* v, const uint32_t* m, Slots<N>& rs, int off, int site, int* prefix,
                    int* total, uint32_t* mn) {
  for (int w = 0; w < kWaves; ++w) {
    int s = 0;
    uint32_t x = kUnused;
    for (int l = 0; l < 64; ++l) {
      s += v[64 * w + l];
      x = m[64 * w + l] < x ? m[64 * w + l] : x;
    }
    rs.put(off + w, site) = (uint32_t)s;
    rs.put(off + kWaves + w, site) = x;
  }
  int tot = 0;
  uint32_t r = kUnused;
  for (int i = 0; i < kWaves; ++i) {
    tot += (int)rs.v[off + i];
    r = rs.v[off + kWaves + i] < r ? rs.v[off + kWaves + i] : r;
  }
  for (int t = 0; t < kThreads; ++t) {
    int base = 0;
    for (int i = 0; i < kWaves; ++i) base += i < (t >> 6) ? (int)rs.v[off + i] : 0;
    int x = 0;   // inclusive wave scan of lanes <= t
    for (int l = 64 * (t >> 6); l <= t; ++l) x += v[l];
    prefix[t] = base + x - v[t];
  }
  *total = tot;
  *mn = r;
}

// block_threshold: keys k[t][q], slots q < nq looked at
template <int KPT>
uint32_t block_threshold(const uint32_t (*k)[KPT], int nq, uint32_t lo, uint32_t hi, int lo_n,
                         int hi_n, Arr<int, kThreads>& red, int* rounds) {
  int half = 0;
  auto count = [&](uint32_t x) {
    for (int w = 0; w < kWaves; ++w) {
      int c = 0;
      for (int q = 0; q < KPT; ++q) {
        if (q >= nq) break;
        for (int l = 0; l < 64; ++l) {
          const uint32_t kk = k[64 * w + l][q];
          c += (kk <= x && kk != kUnused) ? 1 : 0;
        }
      }
      red[half * kWaves + w] = c;   // lane 0 of wave w
    }
    int t = 0;
    for (int i = 0; i < kWaves; ++i) t += red[half * kWaves + i];
    half ^= 1;
    return t;
  };
  uint32_t a = lo, b = hi, res = a;
  *rounds = 0;
  const int c0 = count(a);
  if (c0 < lo_n) {
    for (;;) {
      if (++*rounds > 200) { std::fprintf(stderr, "threshold search did not end\n"); std::abort(); }
      if (b - a <= 1u) { res = a; break; }
      uint32_t mid = orderable(0.5f * from_orderable(a) + 0.5f * from_orderable(b));
      if (!(mid > a && mid < b)) mid = a + (b - a) / 2u;
      const int c = count(mid);
      if (c > hi_n) b = mid;
      else if (c < lo_n) a = mid;
      else { res = mid; break; }
    }
  }
  return res;
}

template <int KPT>
int count_le(const uint32_t (*k)[KPT], int nq, uint32_t x) {
  int c = 0;
  for (int t = 0; t < kThreads; ++t)
    for (int q = 0; q < KPT && q < nq; ++q) c += (k[t][q] <= x && k[t][q] != kUnused) ? 1 : 0;
  return c;
}

// random orderable keys: a spread of distances, ties, -inf, NaN
uint32_t draw_key(std::mt19937& g, int mode) {
  std::uniform_real_distribution<float> U(-2.f, 40.f);
  switch (mode) {
    case 0: return orderable(U(g));
    case 1: return orderable((float)(g() % 7));                       // heavy ties
    case 2: return (g() % 5 == 0) ? orderable(-INFINITY) : orderable(U(g));
    case 3: return (g() % 11 == 0) ? 0u : orderable(U(g));            // NaN -> 0
    default: return orderable(1.0f);                                 // all equal
  }
}

// ---- one stage of screen_kernel (ranked top-K form): pool, scoring slots,
// top-K, candidates, certificate loops
template <int MI>
void screen_stage(std::mt19937& g, int n_h, int P, int K, int mode, bool mlp) {
  Arr<int, kThreads> scan("scan");
  Slots<10 * kWaves> rs;   // screen_kernel's rs
  Arr<int, kPoolCap> pool_o("pool_o");
  Arr<uint32_t, kPoolCap> pool_lb("pool_lb");
  Arr<float, kPoolCap * MI> score("score");
  Arr<uint32_t, kFeatSlots> feat("feat");
  Arr<uint8_t, kPoolCap> cand("cand");
  Arr<int, kPoolCap> cand_o("cand_o");
  std::vector<int> obst_edges(n_h + 1);
  for (auto& e : obst_edges) e = 1 + (int)(g() % MI);

  static uint32_t k[kThreads][kStageKeys];
  static int hidx[kThreads][kStageKeys];
  const int nq = (n_h + kThreads - 1) / kThreads;
  if (nq > kStageKeys) fail("stage key slot", nq, kStageKeys);
  for (int t = 0; t < kThreads; ++t)
    for (int q = 0; q < kStageKeys; ++q) {
      const int idx = t + kThreads * q;
      k[t][q] = kUnused;
      hidx[t][q] = 0;
      if (q < nq && idx < n_h) {
        k[t][q] = draw_key(g, mode);
        hidx[t][q] = idx;   // the list's local obstacle index (distinct)
      }
    }
  P = P < 1 ? 1 : (P > kPoolCap ? kPoolCap : P);
  static uint32_t mnv[2][kThreads];
  static int smv[1][kThreads];
  for (int t = 0; t < kThreads; ++t) {
    uint32_t vmin = kUnused, vmax = 0u;
    int used = 0;
    for (int q = 0; q < kStageKeys; ++q) {
      if (q >= nq) break;
      if (k[t][q] != kUnused) {
        vmin = k[t][q] < vmin ? k[t][q] : vmin;
        vmax = k[t][q] > vmax ? k[t][q] : vmax;
        ++used;
      }
    }
    mnv[0][t] = vmin; mnv[1][t] = ~vmax; smv[0][t] = used;
  }
  uint32_t mo[2];
  int so[1];
  block_reduce<2, 1>(mnv, smv, rs, 0, 0, mo, so);
  const uint32_t kmin = mo[0], kmax = ~mo[1];
  const int n_used = so[0];
  int rounds = 0;
  const uint32_t T = n_used > P ? block_threshold<kStageKeys>(k, nq, kmin, kmax, (3 * P) / 4, P,
                                                             scan, &rounds)
                                : 0xfffffffeu;
  const int cT = count_le<kStageKeys>(k, nq, T);
  if (n_used > P && cT > P && T != kmin) { std::fprintf(stderr, "pool threshold above P\n"); std::abort(); }
  int mine[kThreads], at[kThreads], pool_n = 0;
  uint32_t rest_t[kThreads], rest = 0;
  for (int t = 0; t < kThreads; ++t) {
    mine[t] = 0;
    rest_t[t] = kUnused;
    for (int q = 0; q < kStageKeys; ++q) {
      if (q >= nq) break;
      mine[t] += k[t][q] <= T && k[t][q] != kUnused;
      if (k[t][q] > T) rest_t[t] = k[t][q] < rest_t[t] ? k[t][q] : rest_t[t];
    }
  }
  block_scan_min(mine, rest_t, rs, 3 * kWaves, 1, at, &pool_n, &rest);
  if (pool_n != cT) { std::fprintf(stderr, "pool count\n"); std::abort(); }
  const bool overflow = pool_n > kPoolCap;
  if (!overflow)
    for (int t = 0; t < kThreads; ++t)
      for (int q = 0; q < kStageKeys; ++q)
        if (q < nq && k[t][q] <= T && k[t][q] != kUnused) {
          pool_o[at[t]] = hidx[t][q];
          pool_lb[at[t]] = k[t][q];
          ++at[t];
        }
  if (overflow || pool_n == 0) return;

  // ---- scoring slots
  const int slots = pool_n * MI;
  for (int t = 0; t < kThreads; ++t)
    for (int e = t; e < kPoolCap * MI; e += kThreads) score[e] = INFINITY;
  if (mlp) {
    for (int c0 = 0; c0 < slots; c0 += kFeatSlots) {
      const int cn = kFeatSlots < slots - c0 ? kFeatSlots : slots - c0;
      for (int t = 0; t < kThreads; ++t)
        for (int e = t; e < cn; e += kThreads) {
          const int q = (c0 + e) / MI, j = (c0 + e) - q * MI;
          const int o = pool_o[q];
          if (j < obst_edges[o]) {
            feat[e] = (uint32_t)(o * MI + j);
            score[c0 + e] = 0.f;
          }
        }
      for (int t = 0; t < kThreads; ++t) {
        const int w = t >> 6, n = t & 15, gq = (t & 63) >> 4;
        for (int base = w * 16; base < cn; base += 16 * kWaves) {
          const int e = base + n;
          const bool live = e < cn && score[c0 + e] != INFINITY;
          if (gq == 0 && live) {
            (void)feat[e];
            score[c0 + e] = (float)(g() % 1000) / 100.f;
          }
        }
      }
    }
  } else {
    for (int t = 0; t < kThreads; ++t)
      for (int e = t; e < slots; e += kThreads) {
        const int q = e / MI, j = e - q * MI;
        const int o = pool_o[q];
        if (j < obst_edges[o]) score[e] = (float)(g() % 1000) / 100.f;
      }
  }

  // ---- top-K edges -> candidates
  constexpr int SPT = kPoolCap * MI / kThreads;
  static uint32_t sk[kThreads][SPT];
  int live[kThreads];
  for (int t = 0; t < kThreads; ++t) {
    live[t] = 0;
    uint32_t smn = kUnused, smx = 0u;
    for (int q = 0; q < SPT; ++q) {
      const int e = t * SPT + q;
      const float v = score[e];
      sk[t][q] = (e < slots && v != INFINITY) ? orderable(v) : kUnused;
      live[t] += sk[t][q] != kUnused;
      if (sk[t][q] != kUnused) {
        smn = sk[t][q] < smn ? sk[t][q] : smn;
        smx = sk[t][q] > smx ? sk[t][q] : smx;
      }
    }
    mnv[0][t] = smn; mnv[1][t] = ~smx; smv[0][t] = live[t];
  }
  block_reduce<2, 1>(mnv, smv, rs, 5 * kWaves, 2, mo, so);
  const uint32_t smin = mo[0], smax = ~mo[1];
  const int n_live = so[0];
  const int KK = K < 1 ? 1 : K;
  const uint32_t S = n_live > KK ? block_threshold<SPT>(sk, SPT, smin, smax, (7 * KK) / 8, KK, scan,
                                                        &rounds)
                                 : 0xfffffffeu;
  for (int t = 0; t < kThreads; ++t)
    for (int q = t; q < pool_n; q += kThreads) cand[q] = 0;
  for (int t = 0; t < kThreads; ++t)
    for (int q = 0; q < SPT; ++q)
      if (sk[t][q] <= S && sk[t][q] != kUnused) cand[(t * SPT + q) / MI] = 1;
  int cnt[kThreads], c_at[kThreads], n_cand = 0;
  uint32_t excl_t[kThreads], excl = 0;
  const int per = (pool_n + kThreads - 1) / kThreads;
  for (int t = 0; t < kThreads; ++t) {
    cnt[t] = 0;
    excl_t[t] = rest;
    for (int q = t * per; q < (pool_n < (t + 1) * per ? pool_n : (t + 1) * per); ++q) {
      if (pool_lb[q] <= orderable(-INFINITY)) cand[q] = 1;
      cnt[t] += cand[q];
      if (!cand[q]) excl_t[t] = pool_lb[q] < excl_t[t] ? pool_lb[q] : excl_t[t];
    }
  }
  block_scan_min(cnt, excl_t, rs, 8 * kWaves, 3, c_at, &n_cand, &excl);
  uint32_t excl_ref = rest;   // every non-candidate pool member, each once
  for (int q = 0; q < pool_n; ++q)
    if (!cand[q]) excl_ref = pool_lb[q] < excl_ref ? pool_lb[q] : excl_ref;
  if (excl != excl_ref) { std::fprintf(stderr, "excluded bound\n"); std::abort(); }
  if (n_cand > pool_n) { std::fprintf(stderr, "more candidates than pool\n"); std::abort(); }
  for (int t = 0; t < kThreads; ++t)
    for (int q = t * per; q < (pool_n < (t + 1) * per ? pool_n : (t + 1) * per); ++q)
      if (cand[q]) cand_o[c_at[t]++] = pool_o[q];
  for (int c0 = 0; c0 < n_cand; c0 += kThreads)
    for (int t = 0; t < kThreads; ++t)
      if (c0 + t < n_cand) (void)cand_o[c0 + t];
  for (int t = 0; t < kThreads; ++t)
    for (int q = t; q < pool_n; q += kThreads) {
      if (cand[q]) continue;
      (void)pool_lb[q];
      (void)pool_o[q];
    }
}

// ---- one stage of screen_bound_kernel (one wave): seed, bar, candidate
// compaction by ballots into the LDS list.  Lane l holds list entries
// q * 64 + l, q < kBoundRegs, in registers (key rk, obstacle ro); entries
// from kBoundRegs * 64 on are read again in each pass.
constexpr int kBoundRegs = 8;
void bound_stage(std::mt19937& g, int n_h, int mode) {
  Arr<int, kBoundCap> cand_o("cand_o");
  std::vector<uint32_t> key(n_h);
  std::vector<int> obst(n_h);
  std::vector<int> perm(16384);
  for (int i = 0; i < 16384; ++i) perm[i] = i;
  std::shuffle(perm.begin(), perm.end(), g);
  for (int i = 0; i < n_h; ++i) {
    key[i] = draw_key(g, mode);
    obst[i] = perm[i];   // the list holds each obstacle (< 16384) once
  }
  static uint32_t rk[kBoundRegs][64];
  static int ro[kBoundRegs][64];
  // pass 1: wave minimum of (key << 32 | slot << 16 | obstacle)
  uint64_t lane_lo[64];
  for (int l = 0; l < 64; ++l) {
    lane_lo[l] = ~0ull;
    for (int q = 0; q < kBoundRegs; ++q) {
      const int idx = q * 64 + l;
      rk[q][l] = idx < n_h ? key[idx] : kUnused;
      ro[q][l] = idx < n_h ? obst[idx] : 0;
      if (idx < n_h) {
        const uint64_t v = ((uint64_t)rk[q][l] << 32) | ((uint32_t)idx << 16) | (uint32_t)ro[q][l];
        lane_lo[l] = v < lane_lo[l] ? v : lane_lo[l];
      }
    }
    for (int idx = kBoundRegs * 64 + l; idx < n_h; idx += 64) {
      const uint64_t v = ((uint64_t)key[idx] << 32) | ((uint32_t)idx << 16) | (uint32_t)obst[idx];
      lane_lo[l] = v < lane_lo[l] ? v : lane_lo[l];
    }
  }
  uint64_t lo = ~0ull;
  for (int l = 0; l < 64; ++l) lo = lane_lo[l] < lo ? lane_lo[l] : lo;
  int seed_o = -1;
  uint32_t tkey = orderable(INFINITY);
  if (lo != ~0ull) {
    const int slot = (int)((uint32_t)lo >> 16);
    if (slot < 0 || slot >= n_h) fail("seed slot", slot, n_h);
    seed_o = (int)(lo & 0xffffu);
    if (seed_o != obst[slot]) { std::fprintf(stderr, "seed obstacle\n"); std::abort(); }
    for (int i = 0; i < n_h; ++i)
      if (key[i] < key[slot] || (key[i] == key[slot] && i < slot)) {
        std::fprintf(stderr, "seed is not the first minimum\n");
        std::abort();
      }
    tkey = orderable(std::fmax(from_orderable(key[slot]) + (float)(g() % 100) / 50.f, 1e-3f));
  }
  // pass 2: the register chunks, then the tail chunks; ballot, prefix of
  // the lanes below
  int n_cand = 0, written = 0;
  std::vector<int> order;   // list slots in the order they are compacted
  auto chunk = [&](int i0, bool regs) {
    uint64_t m = 0;
    bool take[64];
    int o[64];
    for (int l = 0; l < 64; ++l) {
      const int idx = i0 + l;
      if (regs) {
        const int q = i0 / 64;
        if (q < 0 || q >= kBoundRegs) fail("register chunk", q, kBoundRegs);
        o[l] = ro[q][l];
        take[l] = idx < n_h && rk[q][l] <= tkey && o[l] != seed_o;
      } else {
        o[l] = idx < n_h ? obst[idx] : -1;
        take[l] = idx < n_h && key[idx] <= tkey && o[l] != seed_o;
      }
      if (take[l]) m |= 1ull << l;
    }
    for (int l = 0; l < 64; ++l) {
      const uint64_t below = (1ull << l) - 1ull;
      const int at = n_cand + __builtin_popcountll(m & below);
      if (take[l] && at < kBoundCap) { cand_o[at] = o[l]; ++written; order.push_back(i0 + l); }
    }
    n_cand += __builtin_popcountll(m);
  };
  for (int q = 0; q < kBoundRegs; ++q) chunk(q * 64, true);
  for (int i0 = kBoundRegs * 64; i0 < n_h; i0 += 64) chunk(i0, false);
  int ref = 0;
  for (int i = 0; i < n_h; ++i) ref += key[i] <= tkey && obst[i] != seed_o;
  if (ref != n_cand) { std::fprintf(stderr, "candidate count\n"); std::abort(); }
  const bool overflow = n_cand > kBoundCap;
  if (!overflow && written != n_cand) { std::fprintf(stderr, "candidates written\n"); std::abort(); }
  for (size_t i = 1; i < order.size(); ++i)
    if (order[i] <= order[i - 1]) { std::fprintf(stderr, "candidates out of list order\n"); std::abort(); }
  // exact evaluation: a quad of lanes per candidate while they fit two
  // passes (four-edge class on staged rows), else a lane per candidate
  if (!overflow && n_cand <= 32)
    for (int c0 = 0; c0 < n_cand; c0 += 16)
      for (int l = 0; l < 64; ++l)
        if (c0 + (l >> 2) < n_cand) (void)cand_o[c0 + (l >> 2)];
  if (!overflow)
    for (int c0 = 0; c0 < n_cand; c0 += 64)
      for (int l = 0; l < 64; ++l)
        if (c0 + l < n_cand) (void)cand_o[c0 + l];
}

// ---- horizon_kernel: every block of an instance appends its lowest keys
// start: the instance's count on entry (0 after a complete call; a call
// that stopped before reopening the lists can leave -1 or a count)
void horizon_instance(std::mt19937& g, int M, int mode, int start = 0) {
  std::vector<int> appended(M, 0);
  int hcount = start;
  const int chunk = (M + kHorizonSplit - 1) / kHorizonSplit;
  if (chunk > kThreads * kHorizonKeys) fail("horizon chunk", chunk, kThreads * kHorizonKeys);
  Arr<int, kThreads> scan("scan");
  std::vector<int> order(kHorizonSplit);
  for (int i = 0; i < kHorizonSplit; ++i) order[i] = i;
  std::shuffle(order.begin(), order.end(), g);   // blocks run in any order
  for (int part : order) {
    const int o0 = part * chunk, o1 = M < o0 + chunk ? M : o0 + chunk;
    if (o0 >= o1) continue;
    Slots<12 * kWaves> rs;   // horizon_kernel's rs, fresh per work-group
    static uint32_t k[kThreads][kHorizonKeys];
    static uint32_t mnv[4][kThreads];
    static int smv[1][kThreads];
    uint32_t mo[4];
    int so[1];
    // the stage positions' box and count of non-finite ones, then R
    for (int t = 0; t < kThreads; ++t) {
      for (int i = 0; i < 4; ++i) mnv[i][t] = (uint32_t)(g() | 0x80000000u);
      smv[0][t] = 0;
    }
    block_reduce<4, 1>(mnv, smv, rs, 0, 0, mo, so);
    block_reduce<1, 1>(mnv, smv, rs, 5 * kWaves, 1, mo, so);
    for (int t = 0; t < kThreads; ++t) {
      uint32_t mn = kUnused, mx = 0u;
      int used = 0;
      for (int q = 0; q < kHorizonKeys; ++q) {
        const int o = o0 + t + kThreads * q;
        k[t][q] = o < o1 ? draw_key(g, mode) : kUnused;
        if (k[t][q] != kUnused) {
          mn = k[t][q] < mn ? k[t][q] : mn;
          mx = k[t][q] > mx ? k[t][q] : mx;
          ++used;
        }
      }
      mnv[0][t] = mn; mnv[1][t] = ~mx; smv[0][t] = used;
    }
    block_reduce<2, 1>(mnv, smv, rs, 7 * kWaves, 2, mo, so);
    const uint32_t kmin = mo[0], kmax = ~mo[1];
    const int n_used = so[0];
    constexpr int P = kHorizonPool / kHorizonSplit;
    int rounds = 0;
    const uint32_t T = n_used > P ? block_threshold<kHorizonKeys>(k, kHorizonKeys, kmin, kmax, P / 2,
                                                                  P, scan, &rounds)
                                  : 0xfffffffeu;
    int mine[kThreads], at[kThreads], total = 0;
    uint32_t rest_t[kThreads], rest = 0;
    for (int t = 0; t < kThreads; ++t) {
      mine[t] = 0;
      rest_t[t] = kUnused;
      for (int q = 0; q < kHorizonKeys; ++q) {
        if (k[t][q] == kUnused) continue;
        if (k[t][q] <= T) ++mine[t];
        else rest_t[t] = k[t][q] < rest_t[t] ? k[t][q] : rest_t[t];
      }
    }
    block_scan_min(mine, rest_t, rs, 10 * kWaves, 3, at, &total, &rest);
    if (total != count_le<kHorizonKeys>(k, kHorizonKeys, T)) {
      std::fprintf(stderr, "horizon count\n");
      std::abort();
    }
    const int base = hcount;   // atomicAdd on the instance's count
    hcount += total;
    for (int t = 0; t < kThreads; ++t)
      for (int q = 0; q < kHorizonKeys; ++q)
        if (k[t][q] != kUnused && k[t][q] <= T) {
          const int slot = base + at[t]++;
          if (slot < 0 || slot >= M) {   // the kernel writes no slot outside [0, M)
            if (start == 0) fail("hlist (instance's M slots)", slot, M);
            continue;
          }
          ++g_checks;
          const int o = o0 + t + kThreads * q;
          if (appended[o]++) { std::fprintf(stderr, "obstacle appended twice\n"); std::abort(); }
        }
  }
}

}  // namespace

int main() {
  std::mt19937 g(12345);
  long stages = 0;
  const int edge_h[] = {0, 1, 63, 64, 255, 256, 257, 511, 1024, 2047, 2048};
  const int edge_p[] = {1, 2, 3, 127, 128, 255, 256, 511, 512};
  for (int mode = 0; mode < 5; ++mode) {
    for (int n_h : edge_h)
      for (int P : edge_p)
        for (int K : {1, 7, 256, 2048, 8192}) {
          const bool mlp = (n_h + P + K + mode) % 2 == 0;
          screen_stage<4>(g, n_h, P, K, mode, mlp);
          screen_stage<8>(g, n_h, P, K, mode, !mlp);
          screen_stage<16>(g, n_h, P, K, mode, mlp);
          stages += 3;
        }
    for (int trial = 0; trial < 400; ++trial) {
      const int n_h = (int)(g() % (kHorizonCap + 1));
      const int P = 1 + (int)(g() % kPoolCap);
      const int K = 1 + (int)(g() % 8192);
      screen_stage<4>(g, n_h, P, K, mode, trial % 2);
      screen_stage<16>(g, n_h, P, K, mode, trial % 3 == 0);
      stages += 2;
    }
    for (int n_h : edge_h) { bound_stage(g, n_h, mode); ++stages; }
    for (int trial = 0; trial < 400; ++trial) {
      bound_stage(g, (int)(g() % (kHorizonCap + 1)), mode);
      ++stages;
    }
    for (int M : {1, 15, 16, 17, 512, 4096, 16383, 16384}) {
      horizon_instance(g, M, mode);
      for (int start : {-1, M / 2, M}) horizon_instance(g, M, mode, start);
    }
  }
  std::printf("ok %ld stages, %ld checked indices\n", stages, g_checks);
  return 0;
}
