"""GPU parity of the spline SDF representation (Sec. III-B) against the FP64
oracle, on pairs of the 8-piece workload (unions of 8 convex hulls of
U{32..128} noisy ellipsoid points) with every object's SDF a cubic spline over
a 32^3-cell box around it (vertex AABB grown by 0.1 L_ref):

* the device fit: coefficients of phi and of the normal spline (FP64 fit,
  stored in FP32) and the per-cell lower bounds, against the oracle's fit;
* a 12-pair batch element by element: group records, per-contact records,
  broad-phase masks (bit-exact outside the 1e-6 tie band), the gradient w.r.t.
  both poses and H v (1e-4 relative, or 4 times the query's FP32 spread);
* sampled queries of a 1024-pair batch in one plan, and a rerun bitwise equal.

Tolerances as for the plane representation."""
import sys

import numpy as np
import pytest

import oracle as O
from paper_2604_17538_amd import workloads as W
from tests import parity as PT

pytestmark = pytest.mark.gpu

REL, K_SPREAD = 1e-4, 4.0
SPLINE = dict(sdf_kind=1, grid_margin_rel=0.0)


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


def _params(L_ref):
    # the box margin as the library receives it (an FP32 parameter): the corners
    # of the fit, and so the normal spline near the surface, move with it
    prm = O.default_params(L_ref, grid_margin_rel=0.0)
    prm.grid_margin = float(np.float32(prm.grid_margin))
    return prm


def _oracle_objs(w, idx, prm):
    objs = [None] * len(w.objects)
    for j in sorted(set(int(i) for i in idx)):
        o = O.from_workload_object(w.objects[j])
        o.build_spline(prm)
        o.build_grid(prm)
        objs[j] = o
    return objs


@pytest.fixture(scope="module")
def small():
    import torch
    from paper_2604_17538_amd import api
    w = W.config1(n_envs=12)
    prm = _params(w.L_ref)
    _log("spline: oracle fits")
    objs = _oracle_objs(w, np.r_[w.qa, w.qb], prm)
    g_o, c_o, goff, coff = O.contacts(prm, objs, w.qa, w.qb, w.poses, want_contacts=True, threads=16)
    cot = W.cotangents(901, goff[-1])
    direc = W.directions(901, w.n)
    gr_o, hv_o = O.grad_hvp(prm, objs, w.qa, w.qb, w.poses, cot, direc, threads=16)
    dg, dh = O.fp32_spread(prm, objs, w.qa, w.qb, w.poses, cot, direc, threads=16)
    _log("spline: device")
    ctx = api.Context(0, L_ref=w.L_ref, **SPLINE)
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
    torch.cuda.synchronize()
    r = np.array([o.radius() for o in objs])
    Lq = r[w.qa] + r[w.qb]
    return dict(w=w, prm=prm, objs=objs, g_o=g_o, c_o=c_o, goff=goff, coff=coff, Lq=Lq, ctx=ctx, hs=hs,
                plan=plan, qd=qd, out=out.cpu().numpy().T.astype(np.float64),
                dbg=dbg.cpu().numpy().T.astype(np.float64), gr_o=gr_o, hv_o=hv_o, dg=dg, dh=dh, cot=cot,
                grad=grad.cpu().numpy().astype(np.float64), g2=g2.cpu().numpy().astype(np.float64),
                hv=hv.cpu().numpy().astype(np.float64), o3=o3.cpu().numpy().T.astype(np.float64),
                g3=g3.cpu().numpy().astype(np.float64), h3=h3.cpu().numpy().astype(np.float64))


def test_device_fit_matches_oracle(small):
    d = small
    for j in range(4):
        n, a, h, C = d["ctx"].object_spline(d["hs"][j])
        no, ao, ho, Co = d["objs"][j].spline()
        assert n == no == d["prm"].grid_res
        assert np.allclose(a, ao, atol=1e-6) and np.allclose(h, ho, rtol=1e-6)
        # FP64 fits on both sides (different algorithms: hull triangles and
        # Gauss-Jordan here, candidate features and Thomas there), stored in FP32:
        # phi within the rounding of each coefficient plus two ulps of the field's
        # scale.  The normal data is the direction to the closest surface point;
        # where two features' distances tie to FP64 rounding (delta ~ 1e-17 m),
        # their closest points can lie 2 sqrt(d delta) apart (the distance is
        # strongly convex along the segment joining them), so two exact FP64
        # implementations may differ by 2 sqrt(delta / d) in the normal at a corner
        # a distance d outside: about 1e-6 at d = 1e-4 m.  A coefficient carries
        # about 0.02 of a corner's value: the normal fields are held to 2^-16 of
        # their scale.
        scale = np.abs(Co).reshape(4, -1).max(1)[:, None, None, None]
        slack = np.array([2.0 ** -22, 2.0 ** -16, 2.0 ** -16, 2.0 ** -16])[:, None, None, None]
        err = np.abs(C - Co) / (2.0 ** -23 * np.abs(Co) + slack * scale)
        k = np.unravel_index(np.argmax(err), err.shape)
        _log("spline fit: per field max error %s of the allowed; worst at %s: %.9e vs %.9e (field scale %.3e)"
             % (np.round(err.reshape(4, -1).max(1), 3).tolist(), k, C[k], Co[k], scale[k[0], 0, 0, 0]))
        assert err.max() <= 1.0, err.max()
        G, _, _, _ = d["ctx"].object_grid(d["hs"][j])
        Go = d["objs"][j].grid()[0]
        assert np.abs(G - Go).max() <= 2.0 ** -22 * np.abs(Go).max() + 1e-12


def test_records_and_contacts(small):
    d = small
    w = d["w"]
    assert np.array_equal(d["plan"].group_off, d["goff"])
    err = PT.check_groups(d["out"], d["g_o"], np.repeat(d["Lq"], np.diff(d["goff"])), d["prm"].tau_blend)
    _log("spline records: %s" % err)
    for k in ("pos", "logZ", "W", "n"):
        assert err[k] <= 1.0, (k, err)
    ex = [d["ctx"].object_export(h) for h in d["hs"]]
    perm_obj = [PT.contact_perm(ex[i], d["objs"][i]) for i in range(len(d["hs"]))]
    perm = PT.query_contact_perm(perm_obj, w.qa, w.qb, d["coff"])
    c, co = d["dbg"], d["c_o"][perm]
    band = (np.abs(co[:, 12] - d["prm"].d_max) <= PT.BAND) | (co[:, 13] <= PT.BAND)
    assert not np.any((c[:, 0] != co[:, 0]) & ~band)
    _log("spline survivors: %.4f of %d contacts" % (c[:, 0].mean(), len(c)))
    assert 0.0 < c[:, 0].mean() < 0.5
    LsC = np.repeat(d["Lq"], np.diff(d["coff"]))
    dpos = np.abs(c[:, [1, 4, 5, 6]] - co[:, [1, 4, 5, 6]]).max(1) / (PT.POS_TOL * LsC)
    assert dpos.max() <= 1.0, dpos.max()
    wgt, wo = c[:, 3], co[:, 3]
    rel = np.where(wo >= PT.W_FLOOR, np.abs(wgt - wo) / (PT.REL_TOL * wo), np.abs(wgt - wo) / 1e-10)
    assert rel.max() <= 1.0, rel.max()
    # per-contact normals (mollified, world frame)
    dn = np.abs(c[:, 7:10] - co[:, 7:10]).max(1)
    assert dn.max() <= PT.REL_TOL, dn.max()


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
    err = PT.check_groups(d["o3"], d["g_o"], np.repeat(d["Lq"], np.diff(d["goff"])), d["prm"].tau_blend)
    for k in ("pos", "logZ", "W", "n"):
        assert err[k] <= 1.0, (k, err)


def test_batch_sampled_and_rerun():
    import torch
    from paper_2604_17538_amd import api
    w = W.config1(n_envs=1024)
    ctx = api.Context(0, L_ref=w.L_ref, **SPLINE)
    hs = ctx.build_objects(w.objects)
    plan = ctx.plan(hs[w.qa], hs[w.qb])
    qd = plan.device_queries(w.poses)
    out = plan.forward(qd)
    out2 = plan.forward(qd)
    torch.cuda.synchronize()
    g = out.cpu().numpy().T.astype(np.float64)
    assert np.array_equal(out2.cpu().numpy().T, g.astype(np.float32))
    sel = np.linspace(0, w.n - 1, 8).astype(np.int64)
    prm = _params(w.L_ref)
    objs = _oracle_objs(w, np.r_[w.qa[sel], w.qb[sel]], prm)
    g_o, goff = O.contacts(prm, objs, w.qa[sel], w.qb[sel], w.poses[sel], threads=16)
    r = np.array([o.radius() if o is not None else 0.0 for o in objs])
    rows = np.concatenate([np.arange(plan.group_off[i], plan.group_off[i + 1]) for i in sel])
    err = PT.check_groups(g[rows], g_o, np.repeat(r[w.qa[sel]] + r[w.qb[sel]], np.diff(goff)), prm.tau_blend)
    _log("spline 1024-pair batch, 8 sampled queries: %s" % err)
    for k in ("pos", "logZ", "W", "n"):
        assert err[k] <= 1.0, (k, err)
