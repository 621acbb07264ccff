"""The oracle's FP32 conditioning probe (oracle.fp32_spread): switched off it
changes nothing, it is deterministic, and its spread is of the size FP32
rounding predicts for a well-conditioned query and far larger for the
ill-conditioned one the GPU tests hold to it."""
import numpy as np

import oracle as O
from paper_2604_17538_amd import workloads as W


def _setup(idx):
    w = W.config0()
    prm = O.default_params(w.L_ref)
    objs = [O.from_workload_object(o) for o in w.objects]
    for o in objs:
        o.build_grid(prm)
    goff, _ = O.layout(objs, w.qa, w.qb)
    cot = W.cotangents(w.n + 11, goff[-1])
    direc = W.directions(w.n + 11, w.n)
    sel = np.array(idx)
    c = np.concatenate([cot[goff[i]:goff[i + 1]] for i in idx])
    return prm, objs, w.qa[sel], w.qb[sel], w.poses[sel], c, direc[sel]


def test_probe_off_is_exact_and_on_is_deterministic():
    prm, objs, qa, qb, poses, c, d = _setup([3, 158, 300])
    g0, h0 = O.grad_hvp(prm, objs, qa, qb, poses, c, d)
    p = O.Params.from_buffer_copy(prm)
    p.jitter, p.jitter_seed = 0.0, 7
    g1, h1 = O.grad_hvp(p, objs, qa, qb, poses, c, d)
    assert np.array_equal(g0, g1) and np.array_equal(h0, h1)
    a = O.fp32_spread(prm, objs, qa, qb, poses, c, d)
    b = O.fp32_spread(prm, objs, qa, qb, poses, c, d)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_spread_size():
    # query 300 (two ellipsoid hulls in contact) is well conditioned: the
    # spread stays within a few hundred unit roundoffs; query 158 (boxes meeting
    # near an edge, contact normals turning within a temperature of the surface)
    # moves by more than 2e-5 of its gradient (1e-4 for some seeds)
    prm, objs, qa, qb, poses, c, d = _setup([300, 158])
    g0 = O.grad_hvp(prm, objs, qa, qb, poses, c)
    dg, _ = O.fp32_spread(prm, objs, qa, qb, poses, c)
    rel = dg / np.linalg.norm(g0, axis=1)
    assert 0 < rel[0] < 1e-5, rel
    assert rel[1] > 2e-5, rel
