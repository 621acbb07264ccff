"""Oracle-side collision geometry of a convex piece, from its point cloud.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  Independent of the HIP
path's own hull builder: the hull itself is qhull (``scipy.spatial.ConvexHull``,
used as a library primitive), and the rest is written out plainly here.

A convex piece is the intersection of the half-spaces of its hull facets
(PSQ without the superquadric term; Sec. III-A.3).  Its collision mesh is the
set of hull vertices and the feature edges of the hull, i.e. the edges between
two facets on different planes (Sec. IV-A: vertices and edges of the mesh).
Triangulated facets that lie on one plane are merged so that no plane appears
twice in the smooth intersection (each duplicate would add tau*log(2)).
"""
from __future__ import annotations

import numpy as np
from scipy.spatial import ConvexHull

MERGE_TOL = 1e-9


def piece_geometry(points: np.ndarray):
    """Return (planes [P,4], verts [V,3], edges [E,2]) of the hull of `points`.

    planes hold (n, h) with unit outward n and n.x + h <= 0 inside.  Vertex order
    is the order of the input points; edges hold indices into `verts`.
    """
    pts = np.asarray(points, np.float64)
    hull = ConvexHull(pts)
    eq = hull.equations            # unit outward normal, offset
    simp = hull.simplices
    nb = hull.neighbors
    F = len(simp)
    scale = max(1.0, float(np.abs(pts).max()))
    # union-find over adjacent facets lying on the same plane
    parent = list(range(F))

    def find(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a

    def same_plane(f, g):
        return (np.linalg.norm(eq[f, :3] - eq[g, :3]) < MERGE_TOL
                and abs(eq[f, 3] - eq[g, 3]) < MERGE_TOL * scale)

    for f in range(F):
        for k in range(3):
            g = nb[f, k]
            if same_plane(f, g):
                ra, rb = find(f), find(g)
                if ra != rb:
                    parent[max(ra, rb)] = min(ra, rb)
    roots = sorted({find(f) for f in range(F)})
    planes = []
    for r in roots:
        members = [f for f in range(F) if find(f) == r]
        n = eq[members, :3].mean(0)
        n = n / np.linalg.norm(n)
        vids = np.unique(simp[members].ravel())
        h = -float((pts[vids] @ n).max())
        planes.append([n[0], n[1], n[2], h])
    # feature edges: between facets of different planes
    edges = set()
    for f in range(F):
        for k in range(3):
            g = nb[f, k]
            if find(f) != find(g):
                a, b = simp[f, (k + 1) % 3], simp[f, (k + 2) % 3]
                edges.add((min(a, b), max(a, b)))
    used = sorted({int(v) for e in edges for v in e} | set(int(v) for v in hull.vertices))
    remap = {v: i for i, v in enumerate(used)}
    verts = pts[used]
    E = np.array(sorted((remap[a], remap[b]) for a, b in edges), np.int32).reshape(-1, 2)
    return np.array(planes, np.float64), verts, E


def piece_triangles(points: np.ndarray) -> np.ndarray:
    """Boundary triangles [T, 9] of the hull of `points` (qhull's facets), for the
    ground truth of the spline SDF."""
    pts = np.asarray(points, np.float64)
    hull = ConvexHull(pts)
    return pts[hull.simplices].reshape(-1, 9)


def raw_piece_triangles(planes: np.ndarray, verts: np.ndarray, tol: float = 1e-9) -> np.ndarray:
    """Boundary triangles [T, 9] of a piece given explicitly by planes and
    vertices: per plane, its vertices (within tol of it) ordered by angle about
    their mean and joined as a fan."""
    tris = []
    scale = max(1.0, float(np.abs(verts).max()))
    for n0, n1, n2, h in planes:
        n = np.array([n0, n1, n2]) / np.linalg.norm([n0, n1, n2])
        hh = h / np.linalg.norm([n0, n1, n2])
        on = verts[np.abs(verts @ n + hh) < tol * scale]
        if len(on) < 3:
            continue
        c = on.mean(0)
        u = on[0] - c
        u /= np.linalg.norm(u)
        v = np.cross(n, u)
        order = np.argsort(np.arctan2((on - c) @ v, (on - c) @ u))
        ring = on[order]
        for k in range(1, len(ring) - 1):
            tris.append(np.concatenate([ring[0], ring[k], ring[k + 1]]))
    return np.array(tris, np.float64).reshape(-1, 9)


def object_geometry(offsets, points):
    """Per-piece hull geometry of an object given as point clouds.

    Returns (plane_off, planes, vert_off, verts, edge_off, edges) with piece-local
    edge indices, the layout the oracle's C++ core takes.
    """
    po, vo, eo = [0], [0], [0]
    P, V, E = [], [], []
    for k in range(len(offsets) - 1):
        pl, vs, es = piece_geometry(points[offsets[k]:offsets[k + 1]])
        P.append(pl); V.append(vs); E.append(es)
        po.append(po[-1] + len(pl)); vo.append(vo[-1] + len(vs)); eo.append(eo[-1] + len(es))
    return (np.array(po, np.int64), np.concatenate(P), np.array(vo, np.int64),
            np.concatenate(V), np.array(eo, np.int64), np.concatenate(E).astype(np.int32))
