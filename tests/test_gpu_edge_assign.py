"""GPU parity of the edge assignment of Sec. IV-D.1 (an edge counts in the
group of every convex piece it crosses, not only its own; cm_params
edge_assign = 1) against the FP64 oracle's own assignment: on 8-piece objects
(whose pieces overlap, so many edges cross other pieces) the group records,
the gradient w.r.t. both poses and H v; on single-piece objects (nothing to
cross) the records equal those without the assignment bit for bit."""
import sys

import numpy as np
import pytest

import oracle as O
from paper_2604_17538_amd import workloads as W
from tests import parity as PT

pytestmark = pytest.mark.gpu

REL, K_SPREAD = 1e-4, 4.0


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


def test_crossing_edges_join_their_pieces():
    import torch
    from paper_2604_17538_amd import api
    w = W.config1(n_envs=8)
    prm = O.default_params(w.L_ref)
    objs = [O.from_workload_object(o) for o in w.objects]
    extra = [int(o.assign_edges().sum()) for o in objs]
    for o in objs:
        o.build_grid(prm)
    _log("crossing edges per object: %s (own edges %s)" % (extra[:4], [len(o.edges) for o in objs[:4]]))
    g_o, goff = O.contacts(prm, objs, w.qa, w.qb, w.poses, threads=16)
    cot = W.cotangents(77, goff[-1])
    direc = W.directions(77, w.n)
    gr_o, hv_o = O.grad_hvp(prm, objs, w.qa, w.qb, w.poses, cot, direc, threads=16)
    dg, dh = O.fp32_spread(prm, objs, w.qa, w.qb, w.poses, cot, direc, threads=16)
    ctx = api.Context(0, L_ref=w.L_ref, edge_assign=1)
    hs = ctx.build_objects(w.objects)
    plan = ctx.plan(hs[w.qa], hs[w.qb])
    _, ncon = O.layout(objs, w.qa, w.qb)
    assert np.array_equal(plan.group_off, goff) and np.array_equal(plan.contact_off, ncon)
    qd = plan.device_queries(w.poses)
    cot_d = torch.tensor(np.ascontiguousarray(cot.T, np.float32)).cuda()
    dir_d = torch.tensor(direc.astype(np.float32)).cuda()
    out, grad, hv = plan.step(qd, cot_d, dir_d)
    torch.cuda.synchronize()
    r = np.array([o.radius() for o in objs])
    Lq = r[w.qa] + r[w.qb]
    err = PT.check_groups(out.cpu().numpy().T.astype(np.float64), g_o, np.repeat(Lq, np.diff(goff)), prm.tau_blend)
    _log("edge assignment records: %s" % err)
    for k in ("pos", "logZ", "W", "n"):
        assert err[k] <= 1.0, (k, err)
    cq = np.sqrt(np.add.reduceat((cot ** 2).sum(1), goff[:-1]))
    floor = 1e-3 * cq * np.maximum(1.0, Lq)
    for got, ref, sp in ((grad, gr_o, dg), (hv, hv_o, dh)):
        g = got.cpu().numpy().astype(np.float64)
        allowed = np.maximum(REL * np.maximum(np.linalg.norm(ref, axis=1), floor), K_SPREAD * sp)
        ratio = np.linalg.norm(g - ref, axis=1) / allowed
        _log("derivative max error / allowed %.3f" % ratio.max())
        assert ratio.max() <= 1.0
    # the assignment changes the records of overlapping pieces
    ctx0 = api.Context(0, L_ref=w.L_ref)
    hs0 = ctx0.build_objects(w.objects)
    p0 = ctx0.plan(hs0[w.qa], hs0[w.qb])
    o0 = p0.forward(p0.device_queries(w.poses))
    torch.cuda.synchronize()
    assert not np.array_equal(o0.cpu().numpy(), out.cpu().numpy())


def test_single_pieces_unchanged():
    import torch
    from paper_2604_17538_amd import api
    w = W.config0(n_poses=32)
    outs = []
    for ea in (0, 1):
        ctx = api.Context(0, L_ref=w.L_ref, edge_assign=ea)
        hs = ctx.build_objects(w.objects)
        plan = ctx.plan(hs[w.qa], hs[w.qb])
        outs.append(plan.forward(plan.device_queries(w.poses)).cpu().numpy())
    torch.cuda.synchronize()
    assert np.array_equal(outs[0], outs[1])
