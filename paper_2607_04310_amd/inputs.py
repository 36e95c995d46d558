"""Seeded synthetic workloads (footprints, stage poses, obstacle edge sets).

This module only draws inputs; it holds none of the PSDF arithmetic.  Both the
HIP path's tests/benchmark and the CPU oracle's tests take their inputs from
here.  Every array is float32 (int32 for offsets), the precision the kernels
consume; the oracle promotes the same arrays to float64.

Edge sets are CSR: ``edges`` is (E, 4) with rows (ax, ay, bx, by) in world
metres, and obstacle i owns rows [obst_off[i], obst_off[i+1]).  Rectangles are
emitted as 4 edges in counter-clockwise order (B_j == A_{j+1} bit-exactly);
free segments are 1-edge obstacles.

Workloads (the paper's Table I uses "randomly generated" obstacle sets and
poses; these stand in for it):

* ``c1``  rectangle footprint 0.6 x 0.4 m; N = 20 poses, x, y ~ U[-5, 5],
  theta ~ U[-pi, pi]; 64 rectangles, sides U[0.2, 1.0], centres U[-5, 5]^2,
  rotations U[-pi, pi] (E = 256).
* ``c2``  hexagonal footprint (circumradius 0.5 m, vertex radii jittered
  +-10 %); N = 50 poses along a random smooth path (Gaussian steps sigma =
  0.1 m, theta from the heading); 4096 rectangles, sides U[0.1, 0.8], in a
  40 x 40 m square (E = 16384).
* ``c3``  c1's shapes plus upstream gradients g ~ N(0, 1) per stage.
* ``c4``  512 independent instances with random convex footprints of 3-8
  vertices, horizons N ~ U{10..80}, edge counts log-uniform in [64, 32768]:
  rectangles plus free segments of length U[0.1, 2].
* ``c5``  64 instances, hexagonal footprint, N = 50, 16384 rectangles whose
  centres follow a 32-component Gaussian mixture (sigma = 2 m) in a 60 x 60 m
  square (E = 65536).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

BASE_SEED = 20261200


def rng_for(cfg: int, instance: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(BASE_SEED + cfg + 1000 * instance))


@dataclass
class Instance:
    footprint: np.ndarray   # (m, 2) float32, CCW, robot-local frame
    poses: np.ndarray       # (N, 3) float32 (x, y, theta)
    edges: np.ndarray       # (E, 4) float32 (ax, ay, bx, by)
    obst_off: np.ndarray    # (M + 1,) int32
    mbar: int               # max edges per obstacle
    meta: dict = field(default_factory=dict)

    @property
    def N(self):
        return int(self.poses.shape[0])

    @property
    def E(self):
        return int(self.edges.shape[0])

    @property
    def M(self):
        return int(self.obst_off.shape[0] - 1)


def rect_footprint(w=0.6, h=0.4):
    a, b = w / 2, h / 2
    return np.array([[-a, -b], [a, -b], [a, b], [-a, b]], dtype=np.float32)


def hexagon_footprint(rng, radius=0.5, jitter=0.1):
    ang = np.deg2rad(60.0 * np.arange(6))
    rad = radius * (1.0 + rng.uniform(-jitter, jitter, size=6))
    return np.stack([rad * np.cos(ang), rad * np.sin(ang)], axis=1).astype(np.float32)


def _hull_ccw(points):
    """Andrew's monotone chain; returns hull vertices counter-clockwise."""
    pts = sorted(map(tuple, np.asarray(points, dtype=np.float64)))

    def cross(o, a, b):
        return (a[0] - o[0]) * (b[1] - o[1]) - (a[1] - o[1]) * (b[0] - o[0])

    lower, upper = [], []
    for p in pts:
        while len(lower) >= 2 and cross(lower[-2], lower[-1], p) <= 0:
            lower.pop()
        lower.append(p)
    for p in reversed(pts):
        while len(upper) >= 2 and cross(upper[-2], upper[-1], p) <= 0:
            upper.pop()
        upper.append(p)
    return np.array(lower[:-1] + upper[:-1])


def random_convex_footprint(rng, m):
    """m vertices taken, in hull order, from the convex hull of 64 points ~ U[-0.5, 0.5]^2."""
    while True:
        hull = _hull_ccw(rng.uniform(-0.5, 0.5, size=(64, 2)))
        if len(hull) >= m:
            break
    idx = np.sort(rng.choice(len(hull), size=m, replace=False))
    return hull[idx].astype(np.float32)


def uniform_poses(rng, n, lo=-5.0, hi=5.0):
    xy = rng.uniform(lo, hi, size=(n, 2))
    th = rng.uniform(-np.pi, np.pi, size=(n, 1))
    return np.concatenate([xy, th], axis=1).astype(np.float32)


def path_poses(rng, n, lo, hi, sigma=0.1):
    """Random smooth path: p_0 ~ U[lo, hi]^2, p_{s+1} = p_s + N(0, sigma^2 I),
    theta_s = heading of the step leaving p_s (the last stage keeps the last heading)."""
    p0 = rng.uniform(lo, hi, size=2)
    steps = rng.normal(0.0, sigma, size=(n, 2))
    pts = p0 + np.concatenate([np.zeros((1, 2)), np.cumsum(steps[:-1], axis=0)], axis=0)
    heading = np.arctan2(steps[:, 1], steps[:, 0])
    return np.concatenate([pts, heading[:, None]], axis=1).astype(np.float32)


def rect_edges(centres, sides, angles):
    """(R*4, 4) CCW edges of rectangles; corners computed in float64, rounded
    to float32 once so that B_j == A_{j+1} bit-exactly."""
    R = len(centres)
    hx, hy = sides[:, 0] / 2, sides[:, 1] / 2
    local = np.stack([np.stack([-hx, -hy], 1), np.stack([hx, -hy], 1),
                      np.stack([hx, hy], 1), np.stack([-hx, hy], 1)], axis=1)  # (R, 4, 2)
    c, s = np.cos(angles)[:, None], np.sin(angles)[:, None]
    wx = centres[:, None, 0] + c * local[..., 0] - s * local[..., 1]
    wy = centres[:, None, 1] + s * local[..., 0] + c * local[..., 1]
    corners = np.stack([wx, wy], axis=-1).astype(np.float32)         # (R, 4, 2)
    nxt = np.roll(corners, -1, axis=1)
    return np.concatenate([corners, nxt], axis=-1).reshape(R * 4, 4)


def segment_edges(centres, lengths, angles):
    d = np.stack([np.cos(angles), np.sin(angles)], 1) * (lengths[:, None] / 2)
    a = (centres - d).astype(np.float32)
    b = (centres + d).astype(np.float32)
    return np.concatenate([a, b], axis=1)


def random_rects(rng, R, side_lo, side_hi, lo, hi):
    centres = rng.uniform(lo, hi, size=(R, 2))
    sides = rng.uniform(side_lo, side_hi, size=(R, 2))
    angles = rng.uniform(-np.pi, np.pi, size=R)
    return rect_edges(centres, sides, angles)


def csr_offsets(sizes):
    return np.concatenate([[0], np.cumsum(sizes)]).astype(np.int32)


def c1(seed_instance: int = 0) -> Instance:
    rng = rng_for(1, seed_instance)
    fp = rect_footprint()
    poses = uniform_poses(rng, 20)
    edges = random_rects(rng, 64, 0.2, 1.0, -5.0, 5.0)
    return Instance(fp, poses, edges, csr_offsets([4] * 64), 4, dict(workload="c1"))


def table_i(M: int, B: int, seed_instance: int = 0) -> Instance:
    """The query shapes of the paper's Table I: B random poses against M random
    obstacles (c1's footprint, rectangles and square)."""
    rng = rng_for(7, 1000 * M + B + 100000 * seed_instance)
    fp = rect_footprint()
    poses = uniform_poses(rng, B)
    edges = random_rects(rng, M, 0.2, 1.0, -5.0, 5.0)
    return Instance(fp, poses, edges, csr_offsets([4] * M), 4, dict(workload=f"table_i M={M} B={B}"))


def c2(seed_instance: int = 0) -> Instance:
    rng = rng_for(2, seed_instance)
    fp = hexagon_footprint(rng)
    poses = path_poses(rng, 50, -20.0, 20.0)
    edges = random_rects(rng, 4096, 0.1, 0.8, -20.0, 20.0)
    return Instance(fp, poses, edges, csr_offsets([4] * 4096), 4, dict(workload="c2"))


def c3(seed_instance: int = 0) -> Instance:
    inst = c1(seed_instance)
    rng = rng_for(3, seed_instance)
    inst.meta = dict(workload="c3", gout=rng.normal(0.0, 1.0, size=inst.N).astype(np.float32))
    return inst


def c2_batch(n_instances: int = 256):
    """c2 at throughput size: n independent c2 draws (seeds 0..n-1), one batch."""
    return [c2(k) for k in range(n_instances)]


def single_pose(n_rects: int, seed: int = 0) -> Instance:
    """One stage pose at the centre of n_rects c2-style rectangles spread at c2's
    density (4096 per 40 x 40 m): the edge-streaming end of the workload
    (every edge is read once per call)."""
    rng = rng_for(7, seed)
    fp = hexagon_footprint(rng_for(2, 0))
    side = 40.0 * float(np.sqrt(n_rects / 4096.0))
    edges = random_rects(rng, n_rects, 0.1, 0.8, -side / 2, side / 2)
    poses = np.array([[0.0, 0.0, float(rng.uniform(-np.pi, np.pi))]], dtype=np.float32)
    return Instance(fp, poses, edges, csr_offsets([4] * n_rects), 4,
                    dict(workload="single_pose", rects=n_rects))


def moving_obstacles(seed: int = 0, N: int = 30, R: int = 200, dt: float = 0.1,
                     half: float = 6.0):
    """A horizon whose edge set changes per stage: R rectangles (centres in
    [-half, half]^2) moving at constant velocities (|v| <= 1 m/s) seen at
    t = s * dt for stage s, and a c2-style path of N poses through them
    (within [-half / 2, half / 2]^2).  Returns (footprint, poses, [edges of
    stage s], [offsets of stage s])."""
    rng = rng_for(8, seed)
    fp = hexagon_footprint(rng)
    poses = path_poses(rng, N, -half / 2, half / 2)
    centres = rng.uniform(-half, half, size=(R, 2))
    sides = rng.uniform(0.1, 0.8, size=(R, 2))
    angles = rng.uniform(-np.pi, np.pi, size=R)
    vel = rng.uniform(-0.7, 0.7, size=(R, 2))
    spin = rng.uniform(-0.5, 0.5, size=R)
    stage_edges, stage_off = [], []
    for s in range(N):
        t = s * dt
        stage_edges.append(rect_edges(centres + t * vel, sides, angles + t * spin))
        stage_off.append(csr_offsets([4] * R))
    return fp, poses, stage_edges, stage_off


def c4_instance(k: int) -> Instance:
    rng = rng_for(4, k)
    m = int(rng.integers(3, 9))
    fp = random_convex_footprint(rng, m)
    N = int(rng.integers(10, 81))
    E = int(round(np.exp(rng.uniform(np.log(64), np.log(32768)))))
    R = int(np.floor(0.75 * E / 4))
    S = E - 4 * R
    side = float(np.sqrt(max(R, 1) / 0.64))
    lo, hi = -side / 2, side / 2
    rect = random_rects(rng, R, 0.1, 0.8, lo, hi)
    seg = segment_edges(rng.uniform(lo, hi, size=(S, 2)), rng.uniform(0.1, 2.0, size=S),
                        rng.uniform(-np.pi, np.pi, size=S))
    edges = np.concatenate([rect, seg], axis=0).astype(np.float32)
    poses = path_poses(rng, N, lo, hi)
    off = csr_offsets([4] * R + [1] * S)
    return Instance(fp, poses, edges, off, 4, dict(workload="c4", k=k))


def c4(n_instances: int = 512):
    return [c4_instance(k) for k in range(n_instances)]


def gmm_rects(rng, R, n_comp, sigma, lo, hi, side_lo=0.1, side_hi=0.8):
    means = rng.uniform(lo, hi, size=(n_comp, 2))
    centres = np.empty((0, 2))
    while len(centres) < R:
        comp = rng.integers(0, n_comp, size=R)
        draw = means[comp] + rng.normal(0.0, sigma, size=(R, 2))
        ok = np.all((draw >= lo) & (draw <= hi), axis=1)
        centres = np.concatenate([centres, draw[ok]], axis=0)
    centres = centres[:R]
    sides = rng.uniform(side_lo, side_hi, size=(R, 2))
    angles = rng.uniform(-np.pi, np.pi, size=R)
    return rect_edges(centres, sides, angles)


def c5_instance(k: int, fp=None, cfg: int = 5) -> Instance:
    rng = rng_for(cfg, k)
    if fp is None:
        fp = hexagon_footprint(rng_for(2, 0))
    edges = gmm_rects(rng, 16384, 32, 2.0, -30.0, 30.0)
    poses = path_poses(rng, 50, -30.0, 30.0)
    return Instance(fp, poses, edges, csr_offsets([4] * 16384), 4, dict(workload="c5", k=k))


def c5(n_instances: int = 64, cfg: int = 5):
    fp = hexagon_footprint(rng_for(2, 0))
    return [c5_instance(k, fp, cfg) for k in range(n_instances)]


# Contact placements of an axis-aligned rectangle against an axis-aligned
# rectangular footprint: (name, side, gap) with gap > 0 a clearance, 0
# touching and < 0 an overlap, on the footprint's right / top face, or at its
# top-right corner (diagonal offset: vertex to vertex when gap >= 0).
CONTACTS = ([(f"face_{side}_{name}", side, g)
             for side in ("right", "top")
             for name, g in (("far", 0.25), ("near", 1.0 / 1024), ("touch", 0.0),
                             ("shallow", -1.0 / 2048), ("mid", -1.0 / 16), ("deep", -0.15))]
            + [(f"corner_{name}", "corner", g)
               for name, g in (("far", 0.25), ("touch", 0.0), ("shallow", -1.0 / 2048),
                               ("deep", -1.0 / 16))])


def aligned_contacts(seed: int = 0, rotate=None) -> Instance:
    """Scenes of exact contact geometry (tie-rich): footprint 0.625 x 0.375 m,
    one stage per placement of CONTACTS (heading 0, stages 16 m apart), each
    against its own axis-aligned rectangle (sides 0.5 x 0.75 m) placed at that
    gap from the footprint's face or corner and slid along the face by a
    seeded dyadic offset (flush, inside or overhanging).  Every coordinate is
    a multiple of 2^-11 m, so the contact ties are exact in float32 and
    float64.  rotate = (angle, tx, ty) applies one rigid motion to every pose
    and edge (the ties then hold only to rounding)."""
    rng = rng_for(40, seed)
    fp = np.array([[-0.3125, -0.1875], [0.3125, -0.1875], [0.3125, 0.1875], [-0.3125, 0.1875]],
                  dtype=np.float32)
    hw, hh = 0.3125, 0.1875          # footprint half extents
    ow, oh = 0.25, 0.375             # obstacle half extents
    poses, edges = [], []
    for k, (_, side, gap) in enumerate(CONTACTS):
        px, py = 16.0 * (k % 4) - 24.0, 16.0 * (k // 4) - 24.0
        slide = float(rng.integers(-512, 513)) / 2048.0     # along the face, |slide| <= 0.25
        if side == "right":
            cx, cy = px + hw + gap + ow, py + slide
        elif side == "top":
            cx, cy = px + slide, py + hh + gap + oh
        else:
            cx, cy = px + hw + gap + ow, py + hh + gap + oh
        poses.append((px, py, 0.0))
        x0, x1, y0, y1 = cx - ow, cx + ow, cy - oh, cy + oh
        corners = [(x0, y0), (x1, y0), (x1, y1), (x0, y1)]
        for j in range(4):
            a, b = corners[j], corners[(j + 1) % 4]
            edges.append((a[0], a[1], b[0], b[1]))
    poses = np.array(poses, dtype=np.float64)
    edges = np.array(edges, dtype=np.float64)
    if rotate is not None:
        ang, tx, ty = rotate
        c, s = np.cos(ang), np.sin(ang)

        def move(x, y):
            return c * x - s * y + tx, s * x + c * y + ty
        poses[:, 0], poses[:, 1] = move(poses[:, 0], poses[:, 1])
        poses[:, 2] += ang
        edges[:, 0], edges[:, 1] = move(edges[:, 0], edges[:, 1])
        edges[:, 2], edges[:, 3] = move(edges[:, 2], edges[:, 3])
    edges = edges.astype(np.float32)
    edges[:, 2:] = np.roll(edges[:, :2].reshape(-1, 4, 2), -1, axis=1).reshape(-1, 2)
    n = len(CONTACTS)
    return Instance(fp, poses.astype(np.float32), edges, csr_offsets([4] * n), 4,
                    dict(workload="aligned_contacts", contacts=[c[0] for c in CONTACTS]))


def random_small(rng, n_obst=8, n_poses=16, lo=-2.0, hi=2.0, fp_m=None, segments=0):
    """Small mixed workloads for parity sweeps: random convex footprint,
    rectangles and free segments near the poses (so that many stages penetrate)."""
    m = int(fp_m) if fp_m is not None else int(rng.integers(3, 9))
    fp = random_convex_footprint(rng, m)
    rect = random_rects(rng, n_obst, 0.1, 1.0, lo, hi)
    seg = segment_edges(rng.uniform(lo, hi, size=(segments, 2)), rng.uniform(0.1, 2.0, segments),
                        rng.uniform(-np.pi, np.pi, segments))
    edges = np.concatenate([rect, seg], axis=0).astype(np.float32)
    poses = uniform_poses(rng, n_poses, lo, hi)
    off = csr_offsets([4] * n_obst + [1] * segments)
    return Instance(fp, poses, edges, off, 4, dict(workload="random_small"))


# ---------------------------------------------------------------- screener

MLP_HIDDEN = 64
MLP_INPUTS = 4
MLP_PARAMS = MLP_HIDDEN * MLP_INPUTS + MLP_HIDDEN + MLP_HIDDEN * MLP_HIDDEN + 2 * MLP_HIDDEN + 1


def mlp_init_params(seed: int = 0) -> np.ndarray:
    """Initial screener weights, He-style normal draws (float32), in the layout
    W1[64][4], b1[64], W2[64][64], b2[64], w3[64], b3."""
    rng = np.random.default_rng(seed)
    H, I = MLP_HIDDEN, MLP_INPUTS
    W1 = rng.normal(0, np.sqrt(2.0 / I), (H, I))
    W2 = rng.normal(0, np.sqrt(2.0 / H), (H, H))
    w3 = rng.normal(0, np.sqrt(1.0 / H), H)
    return np.concatenate([W1.ravel(), np.zeros(H), W2.ravel(), np.zeros(H), w3, [0.0]]).astype(np.float32)


def screener_training_pairs(instances, near=1024, far=1024, seed=0):
    """(stage row, local edge) pairs for screener training over a packed list
    of instances: per stage, the `near` edges whose midpoints are closest to
    the pose position and `far` edges drawn uniformly from the rest."""
    rng = np.random.default_rng(seed)
    stages, edges = [], []
    row = 0
    for inst in instances:
        mid = 0.5 * (inst.edges[:, :2] + inst.edges[:, 2:]).astype(np.float64)
        E = len(mid)
        for s in range(inst.N):
            d2 = ((mid - inst.poses[s, :2].astype(np.float64)) ** 2).sum(1)
            k = min(near, E)
            close = np.argpartition(d2, k - 1)[:k] if k < E else np.arange(E)
            rest = np.setdiff1d(np.arange(E), close, assume_unique=False)
            pick = rng.choice(rest, size=min(far, len(rest)), replace=False) if len(rest) else rest
            sel = np.concatenate([close, pick]).astype(np.int32)
            stages.append(np.full(len(sel), row + s, np.int32))
            edges.append(sel)
        row += inst.N
    return np.concatenate(stages), np.concatenate(edges)
