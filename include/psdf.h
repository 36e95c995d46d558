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
 *    Offsets are not scanned on the host.  An obstacle whose edge count is
 *    negative or above the edge class of mbar (mbar rounded up to 4, 8 or
 *    16), whose range leaves [0, E], or with a non-finite coordinate makes
 *    every stage's result NaN (edge = obst = -1); a count above mbar itself
 *    is outside the contract.  psdf_validate_edges scans a device edge set
 *    for all of these.  Obstacles with zero edges are ignored (the paper's
 *    S = 0 padding).
 *  - Outputs per stage s: d[s] = phi, obst[s] = winning obstacle (lowest index
 *    on ties), edge[s] = global index of the winner's edge with the smallest
 *    point-segment pool distance (lowest index on ties), grad[3s..3s+2] =
 *    dphi/d(x, y, theta).  An empty edge set gives d = +inf, obst = edge = -1,
 *    grad = 0; a non-finite pose gives d = NaN, obst = edge = -1, grad = NaN.
 *  - keys (device uint64[N]) receives the winner of each stage:
 *    (orderable(sd) << 32) | obstacle, where orderable maps floats to
 *    unsigned integers in the same order (NaN lowest).  psdf_bwd consumes it.
 *  - ws (device, caller-owned, 16-byte aligned) is scratch of at least
 *    psdf_workspace_bytes(N, M) bytes: the per-work-group partial minima
 *    and the winners' edge ranges, as 16-byte pairs.  Its content on entry
 *    does not matter.  A misaligned ws gives PSDF_EINVAL.
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

/* Staged constants of an edge set (filled by psdf_stage_edges, below). */
typedef struct {
  void* table;      /* device, caller-owned, psdf_staged_bytes(M, mbar) bytes */
  size_t bytes;     /* its size */
  int32_t E, M;     /* the edge set it was made for */
  int32_t mi_class; /* edge class of that set's mbar: 4, 8 or 16 */
  float eps;        /* params->eps it was made with */
  const void* src[5]; /* that set's ax, ay, bx, by, obst_off */
} psdf_staged;

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
  const psdf_staged* staged; /* host, optional (NULL): see psdf_stage_edges */
} psdf_edges;

/* Message of the last failed call on this thread ("" if none). */
const char* psdf_last_error(void);

/* Library version string. */
const char* psdf_version(void);

/* Bytes of the ws argument of psdf_eval / psdf_grad for N stages and M
 * obstacles (0 when N or M is 0). */
size_t psdf_workspace_bytes(int32_t N, int32_t M);

/* psdf_eval - phi, winning obstacle and edge for N stage poses (Sec. IV-A..D;
 * Alg. 1, PSDF_Forward).
 *   footprint  host float32[m][2]
 *   poses      device float32[N][3]
 *   edges      host struct describing device arrays
 *   params     host; NULL selects the defaults
 *   d, edge, obst, keys   device outputs of length N (see conventions)
 *   ws, ws_bytes          device scratch (see conventions) */
int psdf_eval(const float* footprint, int32_t m, const float* poses, int32_t N,
              const psdf_edges* edges, const psdf_params* params, float* d, int32_t* edge,
              int32_t* obst, uint64_t* keys, void* ws, size_t ws_bytes, hipStream_t stream);

/* psdf_grad - psdf_eval plus grad (device float32[N][3]) = dphi/d(x, y, theta)
 * of each stage, the reverse-mode adjoint through the winning obstacle
 * (Sec. IV-D active-branch subgradient; Alg. 1, PSDF_Backward). */
int psdf_grad(const float* footprint, int32_t m, const float* poses, int32_t N,
              const psdf_edges* edges, const psdf_params* params, float* d, int32_t* edge,
              int32_t* obst, float* grad, uint64_t* keys, void* ws, size_t ws_bytes,
              hipStream_t stream);

/* psdf_grad_noalloc - psdf_grad for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  Same arguments, outputs and errors as psdf_grad,
 * without ws / ws_bytes: the per-work-group partial minima go to a
 * library-owned device buffer of PSDF_NOALLOC_WS_BYTES per GPU (a static
 * device array, held by each GPU the library runs on until the process
 * ends).  A problem whose psdf_workspace_bytes(N, M) exceeds that size
 * returns PSDF_ETOOBIG before anything is enqueued (4 MiB holds, e.g.,
 * N = 64 stages against 262144 obstacles).  The call allocates nothing: no
 * hipMalloc, hipFree or allocating library routine.  Every call on one GPU
 * uses that GPU's one buffer, so calls that overlap in time on one GPU
 * (several streams or host threads) race and must be serialised by the
 * caller; consecutive calls on one stream are safe (each call writes every
 * partial it reads). */
#define PSDF_NOALLOC_WS_BYTES (4u << 20)
int psdf_grad_noalloc(const float* footprint, int32_t m, const float* poses, int32_t N,
                      const psdf_edges* edges, const psdf_params* params, float* d,
                      int32_t* edge, int32_t* obst, float* grad, uint64_t* keys,
                      hipStream_t stream);

/* psdf_constraints - the stage-wise parameters of the linearised safety
 * constraint h(x) = phi(x) - d_min >= 0 that an SQP step hands to its QP
 * (Sec. V: first-order expansion of h about the nominal poses, with
 * J_g = -grad_x h, so that J_g dx <= h; Alg. 1, the export step).
 * hj: device float32[N][4], row s = (phi_s - d_min, -dphi/dx, -dphi/dy,
 * -dphi/dtheta), overwritten.  keys: device uint64[N] (the winners, for a
 * later psdf_bwd).  ws: as for psdf_grad.  hj_host (may be NULL): host
 * float32[N][4] that receives a copy of hj, enqueued on `stream` after the
 * kernels; it should be pinned (hipHostMalloc) for the copy to be
 * asynchronous, and it holds the data once the stream has synchronised.
 * d_min must be finite (PSDF_EINVAL).  An empty edge set gives
 * (+inf, -0, -0, -0); a non-finite pose a row of NaN. */
int psdf_constraints(const float* footprint, int32_t m, const float* poses, int32_t N,
                     const psdf_edges* edges, const psdf_params* params, float d_min, float* hj,
                     float* hj_host, uint64_t* keys, void* ws, size_t ws_bytes,
                     hipStream_t stream);

/* psdf_time_stage_min - measurement aid: enqueues `reps` (1..100000)
 * launches of psdf_eval's per-stage-minimum kernel (the same launch shape)
 * on `stream`, each with an event pair that the dispatch records at its own
 * start and end, waits for them, and stores the mean kernel duration in *ms
 * (host): the kernel's own time, whatever the host's enqueue rate.  Writes
 * only the workspace (sized as for psdf_eval). */
int psdf_time_stage_min(const float* footprint, int32_t m, const float* poses, int32_t N,
                        const psdf_edges* edges, const psdf_params* params, void* ws,
                        size_t ws_bytes, int32_t reps, hipStream_t stream, float* ms);

/* psdf_bwd - vector-Jacobian product of phi with respect to the poses:
 * gpose[s] = gout[s] * dphi_s/d(x, y, theta) (Alg. 1, PSDF_Backward), from the
 * winners that a previous psdf_eval/psdf_grad left in keys (device
 * uint64[N], read only).  The footprint, poses, edges and params must be the
 * ones of that call.  gout device float32[N]; gpose device float32[N][3]
 * (overwritten).  A stage with a non-finite gout or winner gives NaN. */
int psdf_bwd(const float* footprint, int32_t m, const float* poses, int32_t N,
             const psdf_edges* edges, const psdf_params* params, const uint64_t* keys,
             const float* gout, float* gpose, hipStream_t stream);

/* psdf_bwd_geometry - vector-Jacobian product of phi with respect to the
 * geometry: gedges[e] = sum_s gout[s] * dphi_s / d(A_x, A_y, B_x, B_y) of
 * edge e (world frame), gfp[k] = sum_s gout[s] * dphi_s / d(vertex k) of the
 * footprint (its own frame, the caller's vertex order), through each stage's
 * winning obstacle with the active-branch subgradient (Sec. IV-D applied to
 * every input of the pipeline of Sec. IV-A..IV-C).  keys: the winners of a
 * previous psdf_eval/psdf_grad on the same inputs.  gedges: device
 * float32[E][4], gfp: device float32[m][2], both overwritten (zero where no
 * winner depends on them).  A polygon vertex shared by two edges (B_j ==
 * A_{j+1}) may see its gradient split between the two copies in any way;
 * their sum is the vertex's gradient.  Stages add in an unspecified order
 * (FP32 atomics), so the last bits may vary between runs.  A stage with a
 * NaN winner adds NaN to every footprint vertex; a non-finite gout[s] adds
 * NaN to its winner's edges and the footprint. */
int psdf_bwd_geometry(const float* footprint, int32_t m, const float* poses, int32_t N,
                      const psdf_edges* edges, const psdf_params* params, const uint64_t* keys,
                      const float* gout, float* gedges, float* gfp, hipStream_t stream);

/* psdf_sd_matrix - every obstacle's signed distance at every stage, before
 * the minimum over obstacles (Sec. IV-D: sd^i, whose minimum is phi), for
 * callers that constrain several obstacles per stage.  sd: device
 * float32[N][M], stage-major (sd[s * M + i]), overwritten.  An empty
 * obstacle gives +inf, a non-finite pose or an invalid obstacle NaN.  The
 * row minimum and its lowest index equal psdf_eval's d and obst bit for bit.
 * Needs no workspace; the main plain-path launch grid bounds apply
 * (PSDF_ETOOBIG beyond 262140 stages). */
int psdf_sd_matrix(const float* footprint, int32_t m, const float* poses, int32_t N,
                   const psdf_edges* edges, const psdf_params* params, float* sd,
                   hipStream_t stream);

/* psdf_staged_bytes - size of a staged table for M obstacles under the bound
 * mbar: (40 * edge class + 16) bytes per obstacle, M rounded up to 64 (0
 * when M <= 0, M > 2^28 or mbar outside 1..PSDF_MAX_OBST_EDGES). */
size_t psdf_staged_bytes(int32_t M, int32_t mbar);

/* psdf_stage_edges - the pose-independent part of the evaluation, done once
 * per edge set instead of in every call: EncodeEdges of Alg. 1, which runs
 * only when the environment changes while the per-stage evaluation runs at
 * every control step.  For each obstacle it stores, laid out for coalesced
 * loads, the edge start points, the unit edge directions u_j = (B_j - A_j) /
 * (|B_j - A_j| + eps) that give the obstacle normals n'_j = rot90(u_j)
 * (Sec. IV-C), the edge lengths of the point-segment pools (Sec. IV-B), the
 * obstacle's own interval on each of its axes (Sec. IV-C: it does not depend
 * on the pose), its extra V_obs points (open chains), and its closed and
 * invalid flags.
 *   edges   the edge set (edges->staged is ignored)
 *   params  NULL selects the defaults; only eps enters the table
 *   table   device, 16-byte aligned, at least psdf_staged_bytes(M, mbar)
 *           bytes, caller-owned; overwritten on `stream`
 *   out     host; receives (table, bytes, E, M, edge class, eps, the five
 *           array pointers)
 * M above 2^28 gives PSDF_ETOOBIG, a table below the size PSDF_EWS.
 * Point edges->staged at *out for the calls that should use it: psdf_eval,
 * psdf_grad, psdf_grad_noalloc, psdf_constraints and psdf_time_stage_min then
 * read each obstacle from the table in their per-stage minimum kernel, with
 * results bit for bit those of the same call without it (the one-launch form
 * for at most 256 obstacles of at most four edges, and every other entry
 * point, do not use it).  Given a table made for other arrays, another E, M,
 * edge class or eps, or smaller than needed, those calls and psdf_bwd / psdf_sd_matrix
 * return PSDF_EINVAL (psdf_bwd_geometry and psdf_validate_edges ignore the
 * field).  The
 * table describes the edge arrays' contents at staging time: after changing
 * them, stage again before the next call (a stale table gives the old
 * obstacles' distances).  The edge arrays themselves stay in use (the winner
 * adjoint reads them). */
int psdf_stage_edges(const psdf_edges* edges, const psdf_params* params, void* table,
                     size_t table_bytes, psdf_staged* out, hipStream_t stream);

/* psdf_validate_edges - debug scan of a device edge set (the staging step of
 * Sec. IV-A / Alg. 1 EncodeEdges, checked): counts the obstacles outside the
 * edge-set contract above (edge count negative or above mbar, range outside
 * [0, E], a non-finite coordinate) and finds the lowest such index.
 * result: device int32[2], overwritten with (count, lowest index), the index
 * being M when every obstacle is valid.  Enqueued on `stream` (two kernels);
 * reads each obstacle's offsets, and its edges only when its range is valid. */
int psdf_validate_edges(const psdf_edges* edges, int32_t* result, hipStream_t stream);

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

/* ------------------------------------------------------------------------
 * Uneven batches: many independent instances (robots or candidate horizons),
 * each with its own footprint, horizon and edge set, evaluated by persistent
 * launches (one per footprint size present; work items = instance x stage
 * block x obstacle tile, pulled from a device counter, longest first) that
 * also run each stage's winner adjoint.  Every instance is the plain problem of psdf_grad
 * (Sec. IV-A..D); the batch only changes how the work is scheduled.
 *
 * Packed inputs (device, caller-owned): poses float32[sum N][3]; edge
 * columns ax, ay, bx, by float32[sum E]; obstacle offsets int32[sum (M + 1)]
 * with each instance's offsets relative to its own first edge (they start at
 * 0).  Outputs (device, length sum N, rows in the packed pose order): d,
 * edge (index within the instance's edges), obst (index within the
 * instance's obstacles), grad [sum N][3], keys.  The stages of an instance
 * without obstacles (M = 0) get the result of an empty edge set: d = +inf,
 * edge = obst = -1, zero gradient, key 0xffffffffffffffff.  Edge columns
 * may be NULL when no instance has an obstacle.
 * ------------------------------------------------------------------------ */
typedef struct {
  int32_t fp_off;   /* first vertex of this instance's footprint in the host footprint array */
  int32_t m;        /* its vertex count, 3..16 */
  int32_t pose_off; /* first stage row in the packed poses */
  int32_t N;        /* stages */
  int32_t edge_off; /* first edge in the packed edge columns */
  int32_t E;        /* edges */
  int32_t obst_off; /* first entry of its offsets in the packed offset array */
  int32_t M;        /* obstacles (M + 1 offsets) */
} psdf_batch_desc;

typedef struct psdf_batch_plan psdf_batch_plan;

enum {
  PSDF_BATCH_GRAPH = 1,    /* replay a captured hipGraph (captured on first run) */
  PSDF_BATCH_AUTOTUNE = 2  /* psdf_batch_autotune may pick the launch shape */
};

/* Build a plan.  desc: host array of n_inst descriptors; footprints: host
 * float32[][2] indexed by desc[k].fp_off; mbar: bound on the edges per
 * obstacle over all instances (1..16).  Validates every footprint
 * (PSDF_ENONCONVEX / PSDF_EDEGENERATE name the instance in the message) and
 * that the instances' stage rows [pose_off, pose_off + N) tile the packed
 * rows [0, sum N) (else PSDF_EINVAL),
 * allocates the plan's device tables and scratch (freed by
 * psdf_batch_plan_destroy) on the current device.  Calls that use one plan
 * must not overlap in time (the plan's scratch is shared). */
int psdf_batch_plan_create(psdf_batch_plan** plan, const psdf_batch_desc* desc, int32_t n_inst,
                           const float* footprints, int32_t mbar, const psdf_params* params,
                           int32_t flags);
void psdf_batch_plan_destroy(psdf_batch_plan* plan);

/* Evaluate every instance: d, edge, obst, grad and keys as described above.
 * The launches of the different footprint sizes run concurrently: they fork
 * from `stream` onto up to three plan-owned side streams with events and
 * join back before the final kernel, so the call still completes in
 * `stream` order.  With PSDF_BATCH_GRAPH the first call (and any call whose
 * pointers differ from the captured ones) captures the launch into a
 * hipGraph on a plan-owned stream; later calls replay it on `stream`.  Input
 * contents may change between replays.  The final kernel also clears the
 * plan's work counters for the next call: if a call returns an error after
 * it has enqueued work, destroy the plan rather than call it again. */
int psdf_batch(psdf_batch_plan* plan, const float* poses, const float* ax, const float* ay,
               const float* bx, const float* by, const int32_t* obst_off, float* d,
               int32_t* edge, int32_t* obst, float* grad, uint64_t* keys, hipStream_t stream);

/* Autotune the plan's launch shape on real inputs (same arguments as
 * psdf_batch): times each candidate (stages per work item 1, 2, 4, ..., 64 x
 * obstacles per tile 64 or 256 x persistent grid or one work-group per
 * item) on `stream` as a burst of back-to-back calls, in two rounds over
 * all candidates after ten warm-up calls (the better burst counts),
 * synchronising it, keeps the fastest in the plan and in a
 * process-wide cache keyed by the batch's size signature (later plans of the
 * same signature start from it; with PSDF_TUNE_CACHE set to a file path the
 * cache is also read from and appended to that file).  Outputs are left
 * holding a valid result.  best_ms (host, may be NULL) gets the best time. */
int psdf_batch_autotune(psdf_batch_plan* plan, const float* poses, const float* ax,
                        const float* ay, const float* bx, const float* by,
                        const int32_t* obst_off, float* d, int32_t* edge, int32_t* obst,
                        float* grad, uint64_t* keys, hipStream_t stream, float* best_ms);

/* Set the plan's launch shape explicitly (for sweeps and for reproducing a
 * tuned shape): stages_per_item 1..64 (each instance's horizon is cut into
 * ceil(N / stages_per_item) blocks of equal length), obstacles_per_tile 64
 * or 256, direct 0 (persistent grid) or 1 (one work-group per item).  A
 * captured graph is dropped and captured again on the next call.  Results
 * do not depend on the shape. */
int psdf_batch_set_shape(psdf_batch_plan* plan, int32_t stages_per_item,
                         int32_t obstacles_per_tile, int32_t direct);

/* The plan's current shape, work-item count, the largest grid of its
 * launches (one per footprint-size group) and whether items are dispatched
 * one per work-group (direct = 1) or pulled by a persistent grid (host
 * outputs, may be NULL). */
int psdf_batch_plan_info(const psdf_batch_plan* plan, int32_t* stages_per_item,
                         int32_t* obstacles_per_tile, int32_t* n_items, int32_t* grid,
                         int32_t* direct);

/* Certified screened evaluation of a batch (same outputs as psdf_batch, bit
 * for bit).  Per stage: a conservative lower bound LB_i <= sd_i for every
 * obstacle (distance from the pose origin to the obstacle's bounding circle,
 * which a first kernel computes per call unless psdf_batch_stage took them
 * once, minus the footprint's radius
 * about that origin, minus 1e-3 m), a pool of about `pool` lowest-LB
 * obstacles (1..512) whose bounds are tightened to the distance to the
 * polygon itself (-inf if the origin is inside), a ranking of
 * the pool's edges by the screener MLP (theta: device float32[PSDF_MLP_PARAMS],
 * see below) or, with theta = NULL, by the edge's distance to the pose origin,
 * exact evaluation of the obstacles owning the `topk` best edges, and the
 * certificate min over every other obstacle of LB_i > max(phi_K, tau), where
 * phi_K is the candidates' minimum and tau the distance above which the axis
 * test separates two convex sets for this footprint.  Stages that fail the
 * certificate are evaluated in full.  Assumes convex obstacles (Assumption 1)
 * and at most 16384 obstacles per instance and 65535 instances
 * (PSDF_ETOOBIG otherwise).
 * Optional device outputs (length sum N, may be NULL): stage_cand = obstacles
 * evaluated exactly by the screen, stage_cert = 1 if certified, cand_keys =
 * the candidates' minimum key before any fallback.
 * The plan keeps per-instance screening lists that every call opens and
 * closes on the stream; a screened call that returns an error after it has
 * enqueued work may leave them open, so destroy such a plan rather than
 * call it again (the kernels stay within the plan's buffers either way). */
int psdf_batch_screened(psdf_batch_plan* plan, const float* theta, int32_t pool, int32_t topk,
                        const float* poses, const float* ax, const float* ay, const float* bx,
                        const float* by, const int32_t* obst_off, float* d, int32_t* edge,
                        int32_t* obst, float* grad, uint64_t* keys, int32_t* stage_cand,
                        int32_t* stage_cert, uint64_t* cand_keys, hipStream_t stream);

/* Certified screened evaluation without a ranking (same outputs as
 * psdf_batch, bit for bit).  Per stage, with the lower bounds LB_i of
 * psdf_batch_screened: the obstacle with the smallest bound (the seed) is
 * evaluated exactly; its sd bounds phi from above (phi is the minimum over
 * obstacles, Sec. IV-D), so the bar T = max(sd_seed, tau) is at least
 * max(phi, tau), and every obstacle with LB_i <= T is evaluated exactly.
 * The obstacles left out then satisfy the certificate LB_i > max(phi_K,
 * tau) by construction.  A stage still takes the full evaluation when more
 * than 512 obstacles have LB_i <= T, when the bound of the obstacles outside
 * its instance's horizon list is not above T, or when that list is unusable.
 * Same assumptions, limits and optional outputs as psdf_batch_screened
 * (stage_cand counts the seed). */
int psdf_batch_screened_bound(psdf_batch_plan* plan, const float* poses, const float* ax,
                              const float* ay, const float* bx, const float* by,
                              const int32_t* obst_off, float* d, int32_t* edge, int32_t* obst,
                              float* grad, uint64_t* keys, int32_t* stage_cand,
                              int32_t* stage_cert, uint64_t* cand_keys, hipStream_t stream);

/* psdf_batch_stage - the pose-independent part of the screened forms, taken
 * once per edge set instead of in every screened call (Alg. 1 re-encodes the
 * environment only when it changes): every obstacle's bounding circle, and
 * its row of constants for the exact evaluations (unit edge directions,
 * lengths, own-axis intervals of Sec. IV-C, flags).  Until
 * psdf_batch_unstage, psdf_batch_screened and psdf_batch_screened_bound read
 * them, with outputs bit for bit those of the unstaged call; they return
 * PSDF_EINVAL when called with edge or offset pointers other than the ones
 * staged.  The circles describe the arrays' contents at staging time: after
 * changing them in place, stage again (a stale circle can make the
 * certificate exclude the true winner).  The first call allocates device
 * memory held by the plan: 16 bytes per obstacle for the circles and
 * 40 * edge class + 16 bytes for the rows; each call enqueues one kernel on
 * `stream`.  Same limits as psdf_batch_screened. */
int psdf_batch_stage(psdf_batch_plan* plan, const float* ax, const float* ay, const float* bx,
                     const float* by, const int32_t* obst_off, hipStream_t stream);

/* psdf_batch_unstage - screened calls derive the circles from the edges
 * again (the staged circles stay allocated until the plan is destroyed). */
int psdf_batch_unstage(psdf_batch_plan* plan);

/* ------------------------------------------------------------------------
 * Edge-screener MLP: 4 -> 64 -> 64 -> 1 with ReLU on per-(stage, edge)
 * features (the edge's endpoints in the robot frame, divided by 4 m).
 * Parameters: device float32[PSDF_MLP_PARAMS] = W1[64][4], b1[64],
 * W2[64][64], b2[64], w3[64], b3.  The kernels round the matrix operands to
 * BF16 and accumulate in FP32 on the matrix cores.
 * ------------------------------------------------------------------------ */
#define PSDF_MLP_PARAMS 4545

/* y[i] = MLP(X[i]) for B feature rows X (device float32[B][4]). */
int psdf_mlp_forward(const float* theta, const float* X, int32_t B, float* y, hipStream_t stream);

/* Workspace bytes of psdf_mlp_grad / psdf_mlp_train_step for B rows. */
size_t psdf_mlp_ws_bytes(int32_t B);

/* Gradient of the mean squared error mean_i (MLP(X_i) - T_i)^2 with respect
 * to theta: grad device float32[PSDF_MLP_PARAMS + 1], the last entry is the
 * loss.  Deterministic (fixed reduction order). */
int psdf_mlp_grad(const float* theta, const float* X, const float* T, int32_t B, float* grad,
                  void* ws, size_t ws_bytes, hipStream_t stream);

/* One training step: the gradient as above, then Adam (beta1 0.9, beta2
 * 0.999, eps 1e-8, step >= 1, learning rate lr) on theta with moments m, v
 * (device float32[PSDF_MLP_PARAMS], zero before step 1); loss (device float,
 * may be NULL) receives the batch loss before the update. */
int psdf_mlp_train_step(float* theta, float* m, float* v, int32_t step, float lr, const float* X,
                        const float* T, int32_t B, float* loss, void* ws, size_t ws_bytes,
                        hipStream_t stream);

/* Training pairs: for n sampled (stage row, edge index within that stage's
 * instance) pairs of a batch, X[i] (device float32[n][4]) = the edge's
 * robot-frame endpoints / 4 m and T[i] = its pool distance: the minimum over
 * the robot vertices to the edge and over its two endpoints to the robot
 * edges (Sec. IV-B), clipped to [0, 5] m.  Out-of-range pairs give NaN. */
int psdf_screen_labels(const psdf_batch_plan* plan, const float* poses, const float* ax,
                       const float* ay, const float* bx, const float* by, const int32_t* stage,
                       const int32_t* edge, int32_t n, float* X, float* T, hipStream_t stream);

/* Launch shape of the per-stage minimum kernel: blk obstacles per work-group
 * (64 or 256) and sb stages per work-group (1..64).  A non-zero blk overrides
 * every later call in the process (for sweeps); blk = 0 restores the
 * automatic choice (a heuristic on N and M).  Results do not depend on the
 * shape (the minimum and its tie rule are exact). */
int psdf_set_launch_shape(int32_t blk, int32_t sb);

/* Kernel timer, an instrumentation aid for benchmarks.  With capacity > 0,
 * each launch of the dominant kernel of an entry point is bracketed by a
 * pair of HIP events recorded on its launch stream, for up to `capacity`
 * launches: the per-stage minimum kernel of psdf_eval / psdf_grad and the
 * persistent batch kernel of each footprint-size group of an eager
 * psdf_batch call (events recorded by the dispatch itself), the graph
 * replay of a graph psdf_batch call, the screening kernels of
 * psdf_batch_screened / psdf_batch_screened_bound.
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
