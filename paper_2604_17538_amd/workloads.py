"""Seeded synthetic inputs for the contact-manifold workloads.

This module only draws random numbers: point clouds of convex pieces, explicit
box geometry, poses, cotangents and directions.  It holds none of the method's
arithmetic (no hull, no SDF, no contact, no blending), so both the HIP path and
the FP64 oracle consume exactly the same inputs.

The paper evaluates on armadillo/cup meshes and random configurations
(Sec. V.3-V.4); those assets are not available, so these generators stand in for
them with unions of convex pieces of comparable primitive counts.

Recipes (all draws from ``numpy.random.Generator(PCG64(seed))`` in the order
written below):

* ellipsoid points: ``a * normalize(N(0, I3))``; radial noise multiplies by
  ``1 + U[-noise, noise]``;
* log-uniform integer in [lo, hi]: ``floor(exp(U[ln lo, ln(hi + 1))))``;
* poses: ``T_A`` is the identity, ``q_B = normalize(N(0, I4))``,
  ``dir = normalize(N(0, I3))``, ``t_B = dist * dir`` with
  ``dist = (r_A + r_B) * U[0.6, 1.05]`` where ``r_X`` is the largest point norm of
  object X in its own frame.

Every coordinate, pose and direction is rounded to the nearest FP32 value after
it is drawn (rounding draws nothing, so the sequences are unchanged): the FP32
kernels and the FP64 oracle then see exactly the same inputs.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np

SEED_BASE = 17538


@dataclasses.dataclass
class PointObject:
    """An object given as point clouds, one per convex piece (object frame)."""
    offsets: np.ndarray  # int64 [n_pieces + 1], indices into points
    points: np.ndarray   # float64 [n_points, 3]

    @property
    def n_pieces(self) -> int:
        return len(self.offsets) - 1

    def piece(self, k: int) -> np.ndarray:
        return self.points[self.offsets[k]:self.offsets[k + 1]]

    def radius(self) -> float:
        return float(np.sqrt((self.points ** 2).sum(1)).max())


@dataclasses.dataclass
class RawObject:
    """An object given explicitly: planes (n, h), vertices and edges per piece."""
    plane_off: np.ndarray  # int64 [n_pieces + 1]
    planes: np.ndarray     # float64 [P, 4]  (n_x, n_y, n_z, h), inside: n.x + h <= 0
    vert_off: np.ndarray   # int64 [n_pieces + 1]
    verts: np.ndarray      # float64 [V, 3]
    edge_off: np.ndarray   # int64 [n_pieces + 1]
    edges: np.ndarray      # int32 [E, 2], piece-local vertex indices

    @property
    def n_pieces(self) -> int:
        return len(self.plane_off) - 1

    def radius(self) -> float:
        return float(np.sqrt((self.verts ** 2).sum(1)).max())


@dataclasses.dataclass
class Workload:
    name: str
    objects: list                 # PointObject | RawObject
    qa: np.ndarray                # int32 [n] object index of A
    qb: np.ndarray                # int32 [n] object index of B
    poses: np.ndarray             # float64 [n, 14]: qa(w,x,y,z) ta(3) qb(w,x,y,z) tb(3)
    L_ref: float                  # length scale of the workload (m)
    cot_seed: Optional[int] = None

    @property
    def n(self) -> int:
        return len(self.qa)


def unit_box(side: float = 1.0) -> RawObject:
    """Axis-aligned box [-side/2, side/2]^3: 8 vertices, 12 edges, 6 planes."""
    b = 0.5 * side
    planes = np.array([[1, 0, 0, -b], [-1, 0, 0, -b], [0, 1, 0, -b],
                       [0, -1, 0, -b], [0, 0, 1, -b], [0, 0, -1, -b]], np.float64)
    verts = np.array([[sx * b, sy * b, sz * b] for sx in (-1, 1) for sy in (-1, 1)
                      for sz in (-1, 1)], np.float64)
    edges = []
    for i in range(8):
        for j in range(i + 1, 8):
            if np.count_nonzero(verts[i] != verts[j]) == 1:
                edges.append((i, j))
    edges = np.array(edges, np.int32)
    z = np.array([0, 0], np.int64)
    return RawObject(np.array([0, 6], np.int64), planes, np.array([0, 8], np.int64), verts,
                     np.array([0, len(edges)], np.int64), edges)


def _f32(x):
    """Nearest FP32-representable value, kept as float64."""
    return np.asarray(x, np.float64).astype(np.float32).astype(np.float64)


def _unit_gauss(rng, n, d):
    x = rng.standard_normal((n, d))
    return x / np.linalg.norm(x, axis=1, keepdims=True)


def ellipsoid_points(rng, n, axes, noise=0.0):
    p = np.asarray(axes)[None, :] * _unit_gauss(rng, n, 3)
    if noise > 0:
        p = p * (1.0 + rng.uniform(-noise, noise, size=(n, 1)))
    return _f32(p)


def log_uniform_int(rng, lo, hi, size=None):
    return np.floor(np.exp(rng.uniform(np.log(lo), np.log(hi + 1), size=size))).astype(np.int64)


def random_poses(rng, radii_a, radii_b, lo=0.6, hi=1.05):
    """T_A = identity, q_B uniform on SO(3), t_B at distance (r_A + r_B) * U[lo, hi]."""
    n = len(radii_a)
    poses = np.zeros((n, 14))
    poses[:, 0] = 1.0
    qb = _unit_gauss(rng, n, 4)
    d = _unit_gauss(rng, n, 3)
    dist = (np.asarray(radii_a) + np.asarray(radii_b)) * rng.uniform(lo, hi, size=n)
    poses[:, 7:11] = qb
    poses[:, 11:14] = d * dist[:, None]
    return _f32(poses)


def multi_piece_object(rng, n_pieces, counts, axes_lo=0.02, axes_hi=0.2, centre=0.1,
                       noise=0.0) -> PointObject:
    pts, off = [], [0]
    for k in range(n_pieces):
        axes = rng.uniform(axes_lo, axes_hi, size=3)
        c = rng.uniform(-centre, centre, size=3)
        p = _f32(ellipsoid_points(rng, int(counts[k]), axes, noise) + c[None, :])
        pts.append(p)
        off.append(off[-1] + len(p))
    return PointObject(np.array(off, np.int64), np.concatenate(pts, 0))


def config0(seed: int = SEED_BASE + 0, n_poses: int = 256) -> Workload:
    """Two unit boxes (explicit geometry) + two hulls of 64 ellipsoid points."""
    rng = np.random.Generator(np.random.PCG64(seed))
    box = unit_box(1.0)
    e1 = PointObject(np.array([0, 64], np.int64),
                     ellipsoid_points(rng, 64, rng.uniform(0.5, 1.0, size=3)))
    e2 = PointObject(np.array([0, 64], np.int64),
                     ellipsoid_points(rng, 64, rng.uniform(0.5, 1.0, size=3)))
    objects = [box, box, e1, e2]
    p_box = random_poses(rng, [box.radius()] * n_poses, [box.radius()] * n_poses)
    p_ell = random_poses(rng, [e1.radius()] * n_poses, [e2.radius()] * n_poses)
    qa = np.array([0] * n_poses + [2] * n_poses, np.int32)
    qb = np.array([1] * n_poses + [3] * n_poses, np.int32)
    return Workload("c0", objects, qa, qb, np.concatenate([p_box, p_ell]), 1.0)


def config1(seed: int = SEED_BASE + 1, n_envs: int = 4096) -> Workload:
    """n_envs pairs of 8-piece objects; pieces are hulls of U{32..128} noisy ellipsoid points."""
    rng = np.random.Generator(np.random.PCG64(seed))
    objects = []
    for _ in range(2 * n_envs):
        counts = rng.integers(32, 129, size=8)
        objects.append(multi_piece_object(rng, 8, counts, noise=0.05))
    radii = np.array([o.radius() for o in objects])
    qa = np.arange(0, 2 * n_envs, 2, dtype=np.int32)
    qb = qa + 1
    poses = random_poses(rng, radii[qa], radii[qb])
    return Workload("c1", objects, qa, qb, poses, 0.1)


def _c2_object(rng, vlo=8, vhi=512, plo=1, phi=32):
    n_pieces = int(log_uniform_int(rng, plo, phi))
    counts = log_uniform_int(rng, vlo, vhi, size=n_pieces)
    return multi_piece_object(rng, n_pieces, counts, noise=0.0)


def config2(seed: int = SEED_BASE + 2, n_pairs: int = 16384) -> Workload:
    """Pairs with log-uniform piece counts [1,32] and vertex counts [8,512]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    objects = [_c2_object(rng) for _ in range(2 * n_pairs)]
    radii = np.array([o.radius() for o in objects])
    qa = np.arange(0, 2 * n_pairs, 2, dtype=np.int32)
    qb = qa + 1
    poses = random_poses(rng, radii[qa], radii[qb])
    return Workload("c2", objects, qa, qb, poses, 0.1, cot_seed=seed + 1000)


def config4(seed: int = SEED_BASE + 4, n_envs: int = 65536, library: Optional[int] = None) -> Workload:
    """Pairs of 32-piece objects with log-uniform [64,1024] points per piece.

    ``library`` draws the objects from a library of that many distinct objects
    (pair objects picked uniformly) instead of 2 * n_envs distinct ones.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    n_obj = 2 * n_envs if library is None else library
    objects = [_c2_object(rng, 64, 1024, 32, 32) for _ in range(n_obj)]
    radii = np.array([o.radius() for o in objects])
    if library is None:
        qa = np.arange(0, 2 * n_envs, 2, dtype=np.int32)
        qb = qa + 1
    else:
        qa = rng.integers(0, n_obj, size=n_envs).astype(np.int32)
        qb = rng.integers(0, n_obj, size=n_envs).astype(np.int32)
    poses = random_poses(rng, radii[qa], radii[qb])
    return Workload("c4", objects, qa, qb, poses, 0.1, cot_seed=seed + 1000)


def cotangents(seed: int, n_groups: int) -> np.ndarray:
    """Cotangent c ~ N(0, 1) for every group output (12 per group)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return _f32(rng.standard_normal((n_groups, 12)))


def directions(seed: int, n: int) -> np.ndarray:
    """Unit Gaussian direction in R^12 per pair-query."""
    rng = np.random.Generator(np.random.PCG64(seed + 1))
    return _f32(_unit_gauss(rng, n, 12))


@dataclasses.dataclass
class ServingTrace:
    """Poisson request stream over a library of objects."""
    arrival_s: np.ndarray      # float64 [R] arrival times
    n_pairs: np.ndarray        # int32 [R] pairs per request (U{1..64})
    want_grad: np.ndarray      # bool [R] (30 % forward+gradient)
    pair_a: List[np.ndarray]   # per request: object indices A
    pair_b: List[np.ndarray]
    poses: List[np.ndarray]    # per request: [n_pairs, 14]


def serving_trace(library: list, rate_hz: float, duration_s: float,
                  seed: int = SEED_BASE + 3, max_pairs: int = 64,
                  grad_fraction: float = 0.3) -> ServingTrace:
    rng = np.random.Generator(np.random.PCG64(seed))
    radii = np.array([o.radius() for o in library])
    t, arr = 0.0, []
    while True:
        t += rng.exponential(1.0 / rate_hz)
        if t >= duration_s:
            break
        arr.append(t)
    R = len(arr)
    n_pairs = rng.integers(1, max_pairs + 1, size=R).astype(np.int32)
    want_grad = rng.uniform(size=R) < grad_fraction
    pa, pb, ps = [], [], []
    for r in range(R):
        a = rng.integers(0, len(library), size=n_pairs[r]).astype(np.int32)
        b = rng.integers(0, len(library), size=n_pairs[r]).astype(np.int32)
        pa.append(a)
        pb.append(b)
        ps.append(random_poses(rng, radii[a], radii[b]))
    return ServingTrace(np.array(arr), n_pairs, want_grad, pa, pb, ps)


def library_objects(n: int = 2048, seed: int = SEED_BASE + 3) -> list:
    rng = np.random.Generator(np.random.PCG64(seed + 7))
    return [_c2_object(rng) for _ in range(n)]


# ------------------------------------------------------- primitive objects --
# Objects whose SDF side is a list of primitives (Sec. III-A: superquadrics
# intersected with half-spaces (PSQ), swept along quadratic splines (XPSQ),
# folded by union / subtraction / intersection) and whose mesh side is convex
# pieces: hulls of points drawn on the primitives' surfaces.  The records are the
# 32-double layout of cm_object_set_prims; every value is FP32-representable.
@dataclasses.dataclass
class PrimObject(PointObject):
    prim_rec: np.ndarray = None        # float64 [n, 32]
    prim_plane_off: np.ndarray = None  # int64 [n + 1]
    prim_planes: np.ndarray = None     # float64 [P, 4]


def prim_record(kind, op=0, c=(0, 0, 0), p=None, quat=(1, 0, 0, 0), a0=(1, 1, 1), e0=(1, 1), a1=None, e1=None):
    r = np.zeros(32)
    r[0], r[1] = kind, op
    if p is None:
        r[2:5] = c
    else:
        r[2:11] = np.asarray(p, np.float64).ravel()
    r[11:15] = quat
    r[15:18], r[18:20] = a0, e0
    r[20:23] = a0 if a1 is None else a1
    r[23:25] = e0 if e1 is None else e1
    return _f32(r)


def _spow(v, k):
    return np.sign(v) * np.abs(v) ** k


def sq_surface_points(rng, n, a, e):
    """Points of the superquadric f = 1 by its parametric form (angles uniform)."""
    eta = rng.uniform(-np.pi / 2, np.pi / 2, n)
    om = rng.uniform(-np.pi, np.pi, n)
    return np.stack([a[0] * _spow(np.cos(eta), e[0]) * _spow(np.cos(om), e[1]),
                     a[1] * _spow(np.cos(eta), e[0]) * _spow(np.sin(om), e[1]),
                     a[2] * _spow(np.sin(eta), e[0])], 1)


def _quat_R(q):
    w, x, y, z = np.asarray(q, np.float64) / np.linalg.norm(q)
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def _sweep_points(rng, P, a0, e0, a1, e1, t_lo, t_hi, n):
    """Points on the superquadrics placed along the spline P (3 control points)
    between t_lo and t_hi, each in the spline's Frenet frame [N, b, T]."""
    P = np.asarray(P, np.float64)
    A, B = P[0] - 2 * P[1] + P[2], 2 * (P[1] - P[0])
    b = np.cross(B, A)
    b /= np.linalg.norm(b)
    t = rng.uniform(t_lo, t_hi, n)
    t[:2] = (t_lo, t_hi)
    out = []
    for tk in t:
        T = 2 * A * tk + B
        T /= np.linalg.norm(T)
        N = np.cross(b, T)
        a = np.asarray(a0) + tk * (np.asarray(a1) - np.asarray(a0))
        e = np.asarray(e0) + tk * (np.asarray(e1) - np.asarray(e0))
        s = sq_surface_points(rng, 6, a, e)
        pt = (1 - tk) ** 2 * P[0] + 2 * tk * (1 - tk) * P[1] + tk ** 2 * P[2]
        out.append(pt + s[:, :1] * N + s[:, 1:2] * b + s[:, 2:3] * T)
    return np.concatenate(out, 0)


def prim_object(rng, kind: int) -> PrimObject:
    """One of four primitive objects, its sizes jittered by U[0.8, 1.2]:
    0 cup (cylinder minus a raised cylinder, plus a handle: a rounded box swept
    along a spline), 1 tube (a sphere swept along a random curved spline),
    2 dome (an ellipsoid cut by a half-space), 3 rounded box (a superquadric of
    exponents 0.3 at a random rotation)."""
    j = lambda: rng.uniform(0.8, 1.2)
    recs, planes, plane_off, pieces = [], [], [0], []
    if kind == 0:
        r, h, w = 0.05 * j(), 0.06 * j(), 0.007 * j()
        recs.append(prim_record(0, 0, c=(0, 0, 0), a0=(r, r, h), e0=(0.1, 1.0)))
        recs.append(prim_record(0, 1, c=(0, 0, 1.5 * w), a0=(r - w, r - w, h), e0=(0.1, 1.0)))
        P = [(0.9 * r, 0, 0.55 * h), (1.9 * r, 0, 0.0), (0.9 * r, 0, -0.55 * h)]
        ah = (w * 1.2, w * 1.6, w * 1.2)
        recs.append(prim_record(1, 0, p=P, a0=ah, e0=(0.3, 0.3)))
        plane_off += [0, 0, 0]
        pieces.append(sq_surface_points(rng, 160, (r, r, h), (0.1, 1.0)))
        for lo, hi in ((0.0, 0.5), (0.5, 1.0)):
            pieces.append(_sweep_points(rng, P, ah, (0.3, 0.3), ah, (0.3, 0.3), lo, hi, 12))
    elif kind == 1:
        rad = 0.015 * j()
        P = [(-0.06 * j(), 0, 0), (0.0, 0.05 * j(), 0.02 * rng.uniform(-1, 1)), (0.06 * j(), 0, 0.01 * rng.uniform(-1, 1))]
        recs.append(prim_record(1, 0, p=P, a0=(rad, rad, rad), e0=(1.0, 1.0), a1=(0.7 * rad, 0.7 * rad, 0.7 * rad)))
        plane_off.append(0)
        a1 = (0.7 * rad,) * 3
        for lo, hi in ((0.0, 1 / 3), (1 / 3, 2 / 3), (2 / 3, 1.0)):
            pieces.append(_sweep_points(rng, P, (rad,) * 3, (1.0, 1.0), a1, (1.0, 1.0), lo, hi, 14))
    elif kind == 2:
        a = (0.05 * j(), 0.04 * j(), 0.05 * j())
        cut = 0.3 * a[2]
        recs.append(prim_record(0, 0, c=(0, 0, 0), a0=a, e0=(1.0, 1.0)))
        planes.append((0.0, 0.0, 1.0, -cut))  # z <= cut
        plane_off.append(1)
        s = sq_surface_points(rng, 300, a, (1.0, 1.0))
        s = s[s[:, 2] <= cut]
        rr = np.sqrt(np.maximum(0.0, 1 - (cut / a[2]) ** 2))
        th = rng.uniform(0, 2 * np.pi, 40)
        disk = np.stack([a[0] * rr * np.cos(th), a[1] * rr * np.sin(th), np.full(40, cut)], 1)
        pieces.append(np.concatenate([s, disk], 0))
    else:
        a = (0.04 * j(), 0.03 * j(), 0.02 * j())
        q = _unit_gauss(rng, 1, 4)[0]
        recs.append(prim_record(0, 0, c=(0, 0, 0), quat=q, a0=a, e0=(0.3, 0.3)))
        plane_off.append(0)
        pieces.append(sq_surface_points(rng, 200, a, (0.3, 0.3)) @ _quat_R(_f32(q)).T)
    off = np.cumsum([0] + [len(p) for p in pieces]).astype(np.int64)
    return PrimObject(off, _f32(np.concatenate(pieces, 0)), np.array(recs), np.array(plane_off, np.int64),
                      _f32(np.array(planes, np.float64).reshape(-1, 4)))


def config_prims(seed: int = SEED_BASE + 5, n_pairs: int = 256) -> Workload:
    """Pairs of primitive objects (cup, tube, dome, rounded box, drawn uniformly),
    posed as the other workloads but closer, t_B at (r_A + r_B) U[0.35, 0.75]:
    the shapes are thin (handles, tubes), and at the usual distances few of
    their pieces come within d_max."""
    rng = np.random.Generator(np.random.PCG64(seed))
    kinds = rng.integers(0, 4, size=2 * n_pairs)
    objects = [prim_object(rng, int(k)) for k in kinds]
    radii = np.array([o.radius() for o in objects])
    qa = np.arange(0, 2 * n_pairs, 2, dtype=np.int32)
    qb = qa + 1
    poses = random_poses(rng, radii[qa], radii[qb], lo=0.35, hi=0.75)
    return Workload("prims", objects, qa, qb, poses, 0.1, cot_seed=seed + 1000)
