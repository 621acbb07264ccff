"""GPU parity on the method's edge cases, element by element against the FP64
oracle through the C ABI:

* minimal pieces: single-piece hulls of 4..12 points (4..20 planes, so the
  plane passes see pieces below, at and above the 16-plane support subset and
  every tail length of the 4-plane blocks);
* a pair far apart (ten times the scene scale: every contact lies beyond d_max,
  the groups take the filtered closed form d_max, W = 0; outside an object's
  grid the broad-phase bound is the 1-Lipschitz extension from the nearest
  voxel, which loosens with distance, so these contacts survive the broad phase
  on both sides and are evaluated, contributing nothing);
* coincident objects (the same object on both sides, identity poses: deep
  penetration, every contact survives) and a rotated copy at zero offset;
* the far-apart query alone in a plan of one query, bitwise equal to its
  results inside the batch.

Tolerances as for the workloads: positions and distances 1e-5 L_s, weights and
normals 1e-4, broad-phase masks bit-exact outside the 1e-6 tie band, gradients
1e-4 and H v 1e-4 relative, each derivative also allowed 4 times the query's
FP32 spread.  An empty batch is rejected by cm_plan_create (tested on the CPU)."""
import sys

import numpy as np
import pytest

import oracle as O
from paper_2604_17538_amd import workloads as W
from tests import parity as PT

pytestmark = pytest.mark.gpu

REL, REL_HVP, K_SPREAD = 1e-4, 1e-4, 4.0
L_REF = 0.1


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


def _workload():
    rng = np.random.Generator(np.random.PCG64(7000))
    objs = []
    for nv in range(4, 13):  # one piece each: 2 nv - 4 planes for points in general position
        axes = rng.uniform(0.02, 0.2, 3)
        objs.append(W.PointObject(np.array([0, nv], np.int64), W.ellipsoid_points(rng, nv, axes)))
    objs.append(W.multi_piece_object(rng, 3, np.array([4, 5, 6]), noise=0.0))
    n_o = len(objs)
    qa, qb = [], []
    for i in range(n_o):
        for j in (i, (i + 3) % n_o):
            qa.append(i)
            qb.append(j)
    qa, qb = np.array(qa, np.int32), np.array(qb, np.int32)
    r = np.array([o.radius() for o in objs])
    poses = W.random_poses(rng, r[qa], r[qb])
    # far apart: every contact filtered
    far = len(qa)
    qa = np.append(qa, np.int32(2)); qb = np.append(qb, np.int32(5))
    p = W.random_poses(rng, r[[2]], r[[5]])
    t = p[0, 11:14]
    p[0, 11:14] = t / np.linalg.norm(t) * 10.0 * (r[2] + r[5])
    poses = np.concatenate([poses, W._f32(p)])
    # coincident: same object, identity poses; and a rotated copy at zero offset
    coinc = len(qa)
    for k, rot in ((n_o - 1, False), (4, True)):
        qa = np.append(qa, np.int32(k)); qb = np.append(qb, np.int32(k))
        p = np.zeros((1, 14)); p[0, 0] = 1.0; p[0, 7] = 1.0
        if rot:
            q = rng.standard_normal(4); p[0, 7:11] = q / np.linalg.norm(q)
        poses = np.concatenate([poses, W._f32(p)])
    return W.Workload("edge", objs, qa, qb, W._f32(poses), L_REF, cot_seed=7001), far, coinc


@pytest.fixture(scope="module")
def edge():
    w, far, coinc = _workload()
    prm = O.default_params(w.L_ref)
    ol = [O.from_workload_object(o) for o in w.objects]
    for o in ol:
        o.build_grid(prm)
    g_o, c_o, goff, coff = O.contacts(prm, ol, w.qa, w.qb, w.poses, want_contacts=True, threads=16)
    cot = W.cotangents(w.cot_seed, goff[-1])
    direc = W.directions(w.cot_seed, w.n)
    gr_o, hv_o = O.grad_hvp(prm, ol, w.qa, w.qb, w.poses, cot, direc, threads=16)
    dg, dh = O.fp32_spread(prm, ol, w.qa, w.qb, w.poses, cot, direc, seeds=(1, 2), threads=16)
    r = np.array([o.radius() for o in ol])
    Lq = r[w.qa] + r[w.qb]
    cq = np.sqrt(np.add.reduceat((cot ** 2).sum(1), goff[:-1]))
    _log("edge: oracle done (%d queries)" % w.n)
    return dict(w=w, far=far, coinc=coinc, prm=prm, objs=ol, g_o=g_o, c_o=c_o, goff=goff, coff=coff, cot=cot,
                dir=direc, gr_o=gr_o, hv_o=hv_o, dg=dg, dh=dh, Lq=Lq, floor=1e-3 * cq * np.maximum(1.0, Lq))


def _ratio(a, b, floor, spread, rel):
    nb = np.linalg.norm(b, axis=1)
    return np.linalg.norm(a - b, axis=1) / np.maximum(rel * np.maximum(nb, floor), K_SPREAD * spread)


def test_edge_cases_element_by_element(edge):
    import torch
    from paper_2604_17538_amd import api
    d = edge
    w = d["w"]
    ctx = api.Context(0, L_ref=w.L_ref)
    hs = ctx.build_objects(w.objects)
    plan = ctx.plan(hs[w.qa], hs[w.qb])
    assert np.array_equal(plan.group_off, d["goff"]) and np.array_equal(plan.contact_off, d["coff"])
    qd = plan.device_queries(w.poses)
    out, dbg = plan.forward(qd, debug=True)
    cot_d = torch.tensor(np.ascontiguousarray(d["cot"].T, np.float32)).cuda()
    dir_d = torch.tensor(d["dir"].astype(np.float32)).cuda()
    out2, grad, hv = plan.step(qd, cot_d, dir_d)
    torch.cuda.synchronize()
    g = out.cpu().numpy().T.astype(np.float64)
    LsG = np.repeat(d["Lq"], np.diff(d["goff"]))
    # records of the forward sweep and of the step (the dual sweep's values)
    for name, gg in (("forward", g), ("step", out2.cpu().numpy().T.astype(np.float64))):
        err = PT.check_groups(gg, d["g_o"], LsG, d["prm"].tau_blend)
        _log("edge records (%s): %s" % (name, err))
        for k in ("pos", "logZ", "W", "n"):
            assert err[k] <= 1.0, (name, k, err)
    # the far-apart query: every contact filtered, groups at the filtered closed form
    far = slice(d["goff"][d["far"]], d["goff"][d["far"] + 1])
    assert np.all(d["g_o"][far, 10] == 0.0)
    assert np.all(g[far, 10] == 0.0) and np.allclose(g[far, 6], d["prm"].d_max)
    # per-contact masks and records
    ex = [ctx.object_export(h) for h in hs]
    perm_obj = [PT.contact_perm(ex[i], d["objs"][i]) for i in range(len(hs))]
    perm = PT.query_contact_perm(perm_obj, w.qa, w.qb, d["coff"])
    c, co = dbg.cpu().numpy().T.astype(np.float64), d["c_o"][perm]
    band = (np.abs(co[:, 12] - d["prm"].d_max) <= PT.BAND) | (co[:, 13] <= PT.BAND)
    assert not np.any((c[:, 0] != co[:, 0]) & ~band)
    cf = slice(d["coff"][d["far"]], d["coff"][d["far"] + 1])
    assert np.all(co[cf, 10] > d["prm"].d_max)  # every contact beyond d_max far apart
    cc = slice(d["coff"][d["coinc"]], d["coff"][d["coinc"] + 1])
    assert c[cc, 0].mean() > 0.5  # deep penetration: most contacts survive
    LsC = np.repeat(d["Lq"], np.diff(d["coff"]))
    dpos = np.abs(c[:, [1, 4, 5, 6]] - co[:, [1, 4, 5, 6]]).max(1) / (PT.POS_TOL * LsC)
    assert dpos.max() <= 1.0, dpos.max()
    # derivatives
    gg, hh = grad.cpu().numpy().astype(np.float64), hv.cpu().numpy().astype(np.float64)
    r = _ratio(gg, d["gr_o"], d["floor"], d["dg"], REL)
    _log("edge gradient: max error / allowed %.3f (query %d)" % (r.max(), int(np.argmax(r))))
    assert r.max() <= 1.0
    r = _ratio(hh, d["hv_o"], d["floor"], d["dh"], REL_HVP)
    _log("edge H v: max error / allowed %.3f (query %d)" % (r.max(), int(np.argmax(r))))
    assert r.max() <= 1.0
    # a plan of one query gives that query's results bitwise
    i = d["far"] - 1
    one = ctx.plan(hs[w.qa[i:i + 1]], hs[w.qb[i:i + 1]])
    q1 = one.device_queries(w.poses[i:i + 1])
    rows = slice(d["goff"][i], d["goff"][i + 1])
    o1, g1, h1 = one.step(q1, cot_d[:, rows].contiguous(), dir_d[i:i + 1].contiguous())
    torch.cuda.synchronize()
    assert np.array_equal(o1.cpu().numpy().T, out2.cpu().numpy().T[rows])
    assert np.array_equal(g1.cpu().numpy(), grad.cpu().numpy()[i:i + 1])
    assert np.array_equal(h1.cpu().numpy(), hv.cpu().numpy()[i:i + 1])
