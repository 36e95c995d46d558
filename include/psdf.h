/*
 * psdf.h - C ABI of the MI355X (gfx950) Polygonal Signed Distance Function library.
 *
 * The PSDF phi(x, E) is the minimum over obstacles i of the signed distance
 * sd(P0(x), P^i) between a convex polygonal robot footprint P0 placed at pose
 * x = (p, theta) and obstacle i, given by its boundary edges (Sec. III-B,
 * eq. for phi).  Per stage pose and obstacle the library evaluates the
 * paper's four-stage pipeline (Sec. IV-A, items 1-4):
 *   1. edges to the robot-local frame, A~ = R(theta)^T (A - p)      (Sec. IV-A)
 *   2. branch-free point-to-segment pools d_v, d_e and d_sep          (Sec. IV-B)
 *   3. separating-axis test over robot and obstacle edge normals and
 *      the log-sum-exp soft-min penetration depth                     (Sec. IV-C)
 *   4. sd = d_sep if separated else -depth; phi = min over obstacles  (Sec. IV-D)
 * and, for the gradient, the reverse-mode adjoint of the winning obstacle's
 * pipeline with respect to (x, y, theta) (the active-branch subgradient of
 * Sec. IV-D; Alg. 1, PSDF_Backward).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Pointers documented "device" are HIP device pointers owned by the caller;
 *    the library never frees, retains or reallocates them.  Pointers
 *    documented "host" are read during the call only.
 *  - Every call only enqueues work on `stream` (NULL = the legacy default
 *    stream) and returns; outputs are valid once that stream has reached the
 *    enqueued work.  The library never synchronises the device or the stream.
 *  - Return value: PSDF_OK (0) on success, a negative PSDF_E* code otherwise;
 *    psdf_last_error() then holds a message (thread-local).  On error nothing
 *    has been enqueued.  No C++ exception crosses the ABI.
 *  - Units: metres and radians.  Poses are (x, y, theta) rows, float32.
 *  - Footprint: m in [3, PSDF_MAX_FP_VERTS] vertices in the robot-local frame,
 *    a strictly convex polygon (Assumption 1).  Either orientation is accepted;
 *    the library reorders it counter-clockwise, so vertex indices never appear
 *    in the outputs.
 *  - Edge set (Sec. III-A, the disjoint union of obstacle boundary edges):
 *    structure of arrays ax, ay, bx, by (float32[E], world frame) and CSR
 *    offsets obst_off (int32[M+1], device): obstacle i owns the edges
 *    [obst_off[i], obst_off[i+1]).  A closed polygon lists its edges in
 *    boundary order with B_j == A_{j+1} (bitwise); an obstacle of one edge is
 *    a free segment.  mbar is a host-side bound on the edges per obstacle (the
 *    paper's padded width m-bar, Sec. IV-A), 1 <= mbar <= PSDF_MAX_OBST_EDGES.
 *    Offsets are not scanned on the host: an obstacle whose edge count is
 *    negative or above mbar, or whose range leaves [0, E], makes every stage's
 *    result NaN (edge = obst = -1).  Obstacles with zero edges are ignored
 *    (the paper's S = 0 padding).
 *  - Outputs per stage s: d[s] = phi, obst[s] = winning obstacle (lowest index
 *    on ties), edge[s] = global index of the winner's edge with the smallest
 *    point-segment pool distance (lowest index on ties), grad[3s..3s+2] =
 *    dphi/d(x, y, theta).  An empty edge set gives d = +inf, obst = edge = -1,
 *    grad = 0; a non-finite pose gives d = NaN, obst = edge = -1, grad = NaN.
 *  - keys (device uint64[N]) is scratch for the per-stage minimum and, on
 *    return, holds the winner of each stage: (orderable(sd) << 32) | obstacle.
 *    psdf_bwd consumes it.
 */
#ifndef PSDF_H
#define PSDF_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PSDF_MAX_FP_VERTS 16
#define PSDF_MAX_OBST_EDGES 16

enum {
  PSDF_OK = 0,
  PSDF_EINVAL = -1,      /* null pointer, negative size, bad parameter */
  PSDF_ENONCONVEX = -2,  /* footprint not strictly convex, or m out of range */
  PSDF_EDEGENERATE = -3, /* zero-length footprint edge */
  PSDF_ETOOBIG = -4,     /* mbar above PSDF_MAX_OBST_EDGES, or a size above a limit */
  PSDF_EWS = -5,         /* workspace too small */
  PSDF_EHIP = -6         /* HIP runtime error (message in psdf_last_error) */
};

/* Constants of the method that the paper leaves open (Sec. IV-B: eps in the
 * projection factor and in the obstacle normals; Sec. IV-C: eps_sat of the
 * separating-axis test and the soft-min sharpness eta).  eta <= 0 or +inf
 * selects the hard minimum, the eta -> inf limit. */
typedef struct {
  float eps;     /* default 1e-12 */
  float eps_sat; /* default 1e-6 m */
  float eta;     /* default 1000 1/m */
} psdf_params;

/* Edge set of one environment (see the conventions above). */
typedef struct {
  const float* ax; /* device float32[E] */
  const float* ay;
  const float* bx;
  const float* by;
  const int32_t* obst_off; /* device int32[M+1] */
  int32_t E;
  int32_t M;
  int32_t mbar;
} psdf_edges;

/* Message of the last failed call on this thread ("" if none). */
const char* psdf_last_error(void);

/* Library version string. */
const char* psdf_version(void);

/* psdf_eval - phi, winning obstacle and edge for N stage poses (Sec. IV-A..D;
 * Alg. 1, PSDF_Forward).
 *   footprint  host float32[m][2]
 *   poses      device float32[N][3]
 *   edges      host struct describing device arrays
 *   params     host; NULL selects the defaults
 *   d, edge, obst, keys   device outputs of length N (see conventions) */
int psdf_eval(const float* footprint, int32_t m, const float* poses, int32_t N,
              const psdf_edges* edges, const psdf_params* params, float* d, int32_t* edge,
              int32_t* obst, uint64_t* keys, hipStream_t stream);

/* psdf_grad - psdf_eval plus grad (device float32[N][3]) = dphi/d(x, y, theta)
 * of each stage, the reverse-mode adjoint through the winning obstacle
 * (Sec. IV-D active-branch subgradient; Alg. 1, PSDF_Backward). */
int psdf_grad(const float* footprint, int32_t m, const float* poses, int32_t N,
              const psdf_edges* edges, const psdf_params* params, float* d, int32_t* edge,
              int32_t* obst, float* grad, uint64_t* keys, hipStream_t stream);

/* psdf_bwd - vector-Jacobian product of phi with respect to the poses:
 * gpose[s] = gout[s] * dphi_s/d(x, y, theta) (Alg. 1, PSDF_Backward), from the
 * winners that a previous psdf_eval/psdf_grad left in keys (device
 * uint64[N], read only).  The footprint, poses, edges and params must be the
 * ones of that call.  gout device float32[N]; gpose device float32[N][3]
 * (overwritten).  A stage with a non-finite gout or winner gives NaN. */
int psdf_bwd(const float* footprint, int32_t m, const float* poses, int32_t N,
             const psdf_edges* edges, const psdf_params* params, const uint64_t* keys,
             const float* gout, float* gpose, hipStream_t stream);

/* psdf_encode_padded - EncodeEdges of Alg. 1 for the paper's padded tensors
 * (Sec. IV-A): A, B device float32[Mbar][mbar][2] and the validity mask S
 * device uint8[Mbar][mbar] become the CSR edge arrays.  Valid entries keep
 * their order; obstacle i of the output is padded row i (rows without a valid
 * entry become empty obstacles).  Outputs (device): ax, ay, bx, by with room
 * for Mbar * mbar entries, obst_off int32[Mbar + 1] (obst_off[Mbar] = E).
 * ws: device scratch of psdf_encode_ws_bytes(Mbar) bytes. */
size_t psdf_encode_ws_bytes(int32_t Mbar);
int psdf_encode_padded(const float* A, const float* B, const uint8_t* S, int32_t Mbar,
                       int32_t mbar, float* ax, float* ay, float* bx, float* by,
                       int32_t* obst_off, void* ws, size_t ws_bytes, hipStream_t stream);

/* Kernel timer, an instrumentation aid for benchmarks.  With capacity > 0,
 * each launch of the dominant kernel of an entry point (the per-stage minimum
 * kernel of psdf_eval / psdf_grad) is bracketed by a pair of HIP events
 * recorded on the launch stream, for up to `capacity` launches.
 * psdf_timer_read waits for those events, returns their summed duration in
 * milliseconds and the number of timed launches, and starts a new count.
 * capacity 0 turns the timer off and releases its events.  Not thread-safe
 * with respect to concurrent launches from several host threads. */
int psdf_timer_enable(int32_t capacity);
int psdf_timer_read(double* total_ms, int64_t* launches);

#ifdef __cplusplus
}
#endif
#endif /* PSDF_H */
