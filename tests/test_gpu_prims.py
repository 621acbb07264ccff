"""GPU parity of the primitive SDF representation (Sec. III-A: superquadrics
intersected with half-spaces (PSQ), swept along quadratic splines with the
soft-branch Cardano projection (XPSQ), folded by smooth union, subtraction and
intersection) against the FP64 oracle, on pairs of primitive objects (cup with
handle, tube, dome, rounded box; mesh side: hulls of points on the primitives'
surfaces):

* a 16-pair batch element by element: group records, per-contact records, the
  gradient w.r.t. both poses and H v, from the separate calls and from the
  one-pass step;
* the isosurface projection onto the primitive SDF;
* a 256-pair batch: sampled queries against the oracle and a rerun bitwise equal.

Tolerances as for the other representations (positions 1e-5 L_s, weights and
normals 1e-4, derivatives 1e-4 relative), each record component and derivative
also allowed 4 times its FP32 spread from the oracle's rounding probe: the XPSQ
projection runs through a cubic's roots, whose conditioning varies."""
import sys

import numpy as np
import pytest

import oracle as O
from paper_2604_17538_amd import workloads as W
from tests import parity as PT

pytestmark = pytest.mark.gpu

REL, K_SPREAD = 1e-4, 4.0
PRIMS = dict(sdf_kind=2)
REC_SEEDS = (1, 2, 3)


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


def _record_spread(prm, objs, qa, qb, poses, g0):
    sp = np.zeros_like(g0)
    for s in REC_SEEDS:
        p = O.Params.from_buffer_copy(prm)
        p.jitter, p.jitter_seed = O.FP32_UNIT_ROUNDOFF, int(s)
        g, _ = O.contacts(p, objs, qa, qb, poses, threads=16)
        sp = np.maximum(sp, np.abs(g - g0))
    return sp


@pytest.fixture(scope="module")
def small():
    import torch
    from paper_2604_17538_amd import api
    w = W.config_prims(n_pairs=16)
    prm = O.default_params(w.L_ref)
    objs = [O.from_workload_object(o) for o in w.objects]  # (no voxel grids: no broad-phase bound)
    g_o, c_o, goff, coff = O.contacts(prm, objs, w.qa, w.qb, w.poses, want_contacts=True, threads=16)
    rsp = _record_spread(prm, objs, w.qa, w.qb, w.poses, g_o)
    cot = W.cotangents(903, goff[-1])
    direc = W.directions(903, w.n)
    gr_o, hv_o = O.grad_hvp(prm, objs, w.qa, w.qb, w.poses, cot, direc, threads=16)
    dg, dh = O.fp32_spread(prm, objs, w.qa, w.qb, w.poses, cot, direc, threads=16)
    _log("prims: oracle done; %d of %d groups active" % (int((g_o[:, 10] > PT.W_FLOOR).sum()), len(g_o)))
    ctx = api.Context(0, L_ref=w.L_ref, **PRIMS)
    hs = ctx.build_objects(w.objects)
    plan = ctx.plan(hs[w.qa], hs[w.qb])
    qd = plan.device_queries(w.poses)
    out, dbg = plan.forward(qd, debug=True)
    cot_d = torch.tensor(np.ascontiguousarray(cot.T, np.float32)).cuda()
    dir_d = torch.tensor(direc.astype(np.float32)).cuda()
    grad = plan.backward(qd, cot_d)
    g2 = torch.empty_like(grad)
    hv = plan.hvp(qd, cot_d, dir_d, grad=g2)
    o3, g3, h3 = plan.step(qd, cot_d, dir_d)
    pin = out[0:3].contiguous()
    proj = plan.project(qd, pin)
    torch.cuda.synchronize()
    r = np.array([o.radius() for o in objs])
    Lq = r[w.qa] + r[w.qb]
    return dict(w=w, prm=prm, objs=objs, g_o=g_o, c_o=c_o, goff=goff, coff=coff, Lq=Lq, ctx=ctx, hs=hs,
                plan=plan, rsp=rsp, cot=cot, gr_o=gr_o, hv_o=hv_o, dg=dg, dh=dh,
                out=out.cpu().numpy().T.astype(np.float64), dbg=dbg.cpu().numpy().T.astype(np.float64),
                grad=grad.cpu().numpy().astype(np.float64), g2=g2.cpu().numpy().astype(np.float64),
                hv=hv.cpu().numpy().astype(np.float64), o3=o3.cpu().numpy().T.astype(np.float64),
                g3=g3.cpu().numpy().astype(np.float64), h3=h3.cpu().numpy().astype(np.float64),
                pin=pin.cpu().numpy().T.astype(np.float64), proj=proj.cpu().numpy().T.astype(np.float64))


def _check_records(d, g, what):
    err = PT.check_groups(g, d["g_o"], np.repeat(d["Lq"], np.diff(d["goff"])), d["prm"].tau_blend,
                          spread=d["rsp"])
    n_sp = int(np.count_nonzero(PT.K_SPREAD * d["rsp"][:, 10] > PT.REL_TOL * np.maximum(d["g_o"][:, 10], 1e-30)))
    _log("prims %s: %s (%d groups' W held to the FP32 spread)" % (what, err, n_sp))
    for k in ("pos", "logZ", "W", "n"):
        assert err[k] <= 1.0, (what, k, err)


def test_records_and_contacts(small):
    d = small
    w = d["w"]
    assert np.array_equal(d["plan"].group_off, d["goff"])
    _check_records(d, d["out"], "records")
    ex = [d["ctx"].object_export(h) for h in d["hs"]]
    perm_obj = [PT.contact_perm(ex[i], d["objs"][i]) for i in range(len(d["hs"]))]
    perm = PT.query_contact_perm(perm_obj, w.qa, w.qb, d["coff"])
    c, co = d["dbg"], d["c_o"][perm]
    bad = np.flatnonzero(~np.isfinite(c[:, 1:10]).all(1))
    if len(bad):
        _log("prims: %d contacts with non-finite records, first: %s" % (len(bad), c[bad[:3]].tolist()))
    assert len(bad) == 0
    assert (c[:, 0] == 1).all() and (co[:, 0] == 1).all()  # no broad-phase bound: every contact evaluated
    LsC = np.repeat(d["Lq"], np.diff(d["coff"]))
    dpos = np.abs(c[:, [1, 4, 5, 6]] - co[:, [1, 4, 5, 6]]).max(1) / (PT.POS_TOL * LsC)
    k = int(np.argmax(dpos))
    _log("prims contacts: %d, max position error / allowed %.3f (contact %d, kind %d)"
         % (len(c), dpos.max(), k, int(co[k, 11])))
    assert dpos.max() <= 1.0, dpos.max()
    wgt, wo = c[:, 3], co[:, 3]
    rel = np.where(wo >= PT.W_FLOOR, np.abs(wgt - wo) / (PT.REL_TOL * wo), np.abs(wgt - wo) / 1e-10)
    assert rel.max() <= 1.0, rel.max()


def _ratio(d, a, b, spread):
    cq = np.sqrt(np.add.reduceat((d["cot"] ** 2).sum(1), d["goff"][:-1]))
    floor = 1e-3 * cq * np.maximum(1.0, d["Lq"])
    allowed = np.maximum(REL * np.maximum(np.linalg.norm(b, axis=1), floor), K_SPREAD * spread)
    r = np.linalg.norm(a - b, axis=1) / allowed
    n_sp = int(np.count_nonzero(K_SPREAD * spread > REL * np.maximum(np.linalg.norm(b, axis=1), floor)))
    _log("max error / allowed %.3f; %d of %d queries held to the FP32 spread" % (r.max(), n_sp, len(r)))
    return r


def test_gradient_and_hvp(small):
    d = small
    for g in (d["grad"], d["g2"], d["g3"]):
        assert _ratio(d, g, d["gr_o"], d["dg"]).max() <= 1.0
    for h in (d["hv"], d["h3"]):
        assert _ratio(d, h, d["hv_o"], d["dh"]).max() <= 1.0
    _check_records(d, d["o3"], "step records")


def test_projection(small):
    d = small
    w = d["w"]
    ref = O.project(d["prm"], d["objs"], w.qa, w.qb, w.poses, d["pin"], threads=16)
    err = np.abs(d["proj"] - ref).max(1) / (PT.POS_TOL * np.repeat(d["Lq"], np.diff(d["goff"])))
    _log("prims projection: max error / allowed %.3f" % err.max())
    assert err.max() <= 1.0


def test_batch_sampled_and_rerun():
    import torch
    from paper_2604_17538_amd import api
    w = W.config_prims(n_pairs=256)
    ctx = api.Context(0, L_ref=w.L_ref, **PRIMS)
    hs = ctx.build_objects(w.objects)
    plan = ctx.plan(hs[w.qa], hs[w.qb])
    qd = plan.device_queries(w.poses)
    out = plan.forward(qd)
    out2 = plan.forward(qd)
    torch.cuda.synchronize()
    g = out.cpu().numpy().T.astype(np.float64)
    assert np.array_equal(out2.cpu().numpy().T, g.astype(np.float32))
    sel = np.linspace(0, w.n - 1, 12).astype(np.int64)
    prm = O.default_params(w.L_ref)
    objs = [None] * len(w.objects)
    for j in sorted(set(int(i) for i in np.r_[w.qa[sel], w.qb[sel]])):
        objs[j] = O.from_workload_object(w.objects[j])
    g_o, goff = O.contacts(prm, objs, w.qa[sel], w.qb[sel], w.poses[sel], threads=16)
    rsp = _record_spread(prm, objs, w.qa[sel], w.qb[sel], w.poses[sel], g_o)
    r = np.array([o.radius() if o is not None else 0.0 for o in objs])
    rows = np.concatenate([np.arange(plan.group_off[i], plan.group_off[i + 1]) for i in sel])
    err = PT.check_groups(g[rows], g_o, np.repeat(r[w.qa[sel]] + r[w.qb[sel]], np.diff(goff)), prm.tau_blend,
                          spread=rsp)
    _log("prims 256-pair batch, 12 sampled queries: %s" % err)
    for k in ("pos", "logZ", "W", "n"):
        assert err[k] <= 1.0, (k, err)
