"""Pins of the oracle's edge assignment (Sec. IV-D.1: an edge belongs to every
convex piece it intersects), CPU only: a hand-counted case (a thin bar
through a cube: exactly the bar's four long edges cross the cube, none of the
cube's edges cross the bar), dense sampling along every edge of random
overlapping pieces (an edge is assigned to a piece iff some sample lies inside
it, away from the tolerance), and single pieces (nothing to assign)."""
import numpy as np

import oracle as O
from paper_2604_17538_amd import workloads as W


def _box(lo, hi):
    s = np.array(np.meshgrid(*[[0, 1]] * 3, indexing="ij")).reshape(3, -1).T
    return np.asarray(lo) + s * (np.asarray(hi) - np.asarray(lo))


def test_bar_through_cube(oracle_mod):
    pts = np.concatenate([_box([0, 0, 0], [1, 1, 1]), _box([-1, 0.4, 0.4], [2, 0.6, 0.6])])
    o = O.from_points(np.array([0, 8, 16]), pts)
    counts = o.assign_edges()
    assert counts.tolist() == [4, 0]
    assert o.n_contacts() == len(o.verts) + len(o.edges) + 4


def test_assignment_matches_dense_sampling(oracle_mod):
    w = W.config1(n_envs=1)
    ob = w.objects[0]
    o = O.from_workload_object(ob)
    counts = o.assign_edges()
    assert counts.sum() > 0
    # brute force: sample every edge of every other piece densely
    t = np.linspace(0.0, 1.0, 2001)[:, None]
    for j in range(o.n_pieces):
        pl = o.planes[o.plane_off[j]:o.plane_off[j + 1]]
        n = 0
        for k in range(o.n_pieces):
            if k == j:
                continue
            V = o.verts[o.vert_off[k]:o.vert_off[k + 1]]
            for a, b in o.edges[o.edge_off[k]:o.edge_off[k + 1]]:
                seg = V[a] + t * (V[b] - V[a])
                depth = (seg @ pl[:, :3].T + pl[:, 3]).max(1)  # <= 0 inside piece j
                if (depth < -1e-7).any():
                    n += 1
                elif (depth <= 1e-7).any():
                    n += -10 ** 6  # a grazing edge: undecided by sampling (none expected)
        assert n == counts[j], (j, n, counts[j])


def test_single_pieces_get_nothing(oracle_mod):
    w = W.config0(n_poses=2)
    for ob in w.objects:
        o = O.from_workload_object(ob)
        assert o.assign_edges().tolist() == [0]
