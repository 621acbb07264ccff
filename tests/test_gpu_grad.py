"""GPU parity of the adjoint (gradient w.r.t. both poses) and of the
Hessian-vector product against the FP64 oracle's hyper-dual derivatives, on the
full config-0 batch: per query, |grad_gpu - grad_oracle| <= 1e-4 |grad_oracle|
and |Hv_gpu - Hv_oracle| <= 1e-4 |Hv_oracle| (norm-wise over the 12-vector),
the stated bound for gradients and HVP.

Where the reference cancels to zero (separated unit boxes: every output is a
blend of vertices symmetric about the body origin, so rotations leave it fixed)
FP32 leaves rounding noise of order eps |c_q| L_s, the size of the cancelling
terms.  The relative bound is therefore taken against
max(|ref|, 1e-3 |c_q| max(1, L_s)), with c_q the query's cotangents and L_s the
sum of the two bounding radii; the floor binds only where |ref| is below it.

Some queries are ill-conditioned at FP32 precision: perturbing each rounded
intermediate of the exact FP64 evaluation by one FP32 rounding (the oracle's
conditioning probe, oracle.fp32_spread) already moves their result by more
than 1e-4.  No FP32 evaluation can be held below that spread, so each query is
held to max(1e-4 |ref|, K * spread) with K = 4 (the kernels round each such
intermediate a few times: FMA chains, rescaled running sums, the base-2 change
of the exponent).  The test reports how many queries need the spread."""
import sys
import time

import numpy as np
import pytest

import oracle as O
from paper_2604_17538_amd import workloads as W

from tests import parity as PT

pytestmark = pytest.mark.gpu

REL = 1e-4
REL_HVP = 1e-4
K_SPREAD = 4.0


def _ratio(a, b, floor, spread, rel=REL):
    """|a - b| per query over the allowed error max(rel max(|b|, floor), K spread)."""
    nb = np.linalg.norm(b, axis=1)
    allowed = np.maximum(rel * np.maximum(nb, floor), K_SPREAD * spread)
    r = np.linalg.norm(a - b, axis=1) / allowed
    n_cond = int(np.count_nonzero(K_SPREAD * spread > rel * np.maximum(nb, floor)))
    print("max error / allowed %.3f (query %d); %d of %d queries held to the FP32 spread"
          % (r.max(), int(np.argmax(r)), n_cond, len(r)), file=sys.stderr)
    return r


def _step(msg):
    print("[%.1f] %s" % (time.time(), msg), file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def c0g():
    import torch
    from paper_2604_17538_amd import api
    _step("oracle start")
    w = W.config0()
    prm = O.default_params(w.L_ref)
    objs = [O.from_workload_object(o) for o in w.objects]
    for o in objs:
        o.build_grid(prm)
    goff, _ = O.layout(objs, w.qa, w.qb)
    cot = W.cotangents(w.n + 11, goff[-1])
    direc = W.directions(w.n + 11, w.n)
    g_o, hv_o = O.grad_hvp(prm, objs, w.qa, w.qb, w.poses, cot, direc, threads=8)
    r = np.array([o.radius() for o in objs])
    Ls = r[w.qa] + r[w.qb]
    cq = np.sqrt(np.add.reduceat((cot ** 2).sum(1), goff[:-1]))
    floor = 1e-3 * cq * np.maximum(1.0, Ls)
    dg, dh = O.fp32_spread(prm, objs, w.qa, w.qb, w.poses, cot, direc, threads=8)
    g_rec, _ = O.contacts(prm, objs, w.qa, w.qb, w.poses, threads=8)
    LsG = np.repeat(Ls, np.diff(goff))
    _step("oracle done; context")
    ctx = api.Context(0, L_ref=w.L_ref)
    hs = ctx.build_objects(w.objects)
    _step("objects built")
    plan = ctx.plan(hs[w.qa], hs[w.qb])
    qd = plan.device_queries(w.poses)
    cot_d = torch.tensor(cot.T.astype(np.float32)).contiguous().cuda()
    dir_d = torch.tensor(direc.astype(np.float32)).cuda()
    torch.cuda.synchronize()
    _step("plan ready; backward")
    grad = plan.backward(qd, cot_d)
    torch.cuda.synchronize()
    _step("backward done; hvp")
    grad2 = torch.empty_like(grad)
    hv = plan.hvp(qd, cot_d, dir_d, grad=grad2)
    torch.cuda.synchronize()
    _step("hvp done")
    return dict(g_o=g_o, hv_o=hv_o, grad=grad.cpu().numpy().astype(np.float64),
                grad2=grad2.cpu().numpy().astype(np.float64), hv=hv.cpu().numpy().astype(np.float64),
                plan=plan, qd=qd, cot_d=cot_d, dir_d=dir_d, floor=floor, dg=dg, dh=dh,
                g_rec=g_rec, LsG=LsG, tau_b=prm.tau_blend)


def test_gradient_matches_oracle(c0g):
    r = _ratio(c0g["grad"], c0g["g_o"], c0g["floor"], c0g["dg"])
    assert r.max() <= 1.0, (r.max(), int(np.argmax(r)))


def test_hvp_gradient_equals_backward(c0g):
    r = _ratio(c0g["grad2"], c0g["g_o"], c0g["floor"], c0g["dg"])
    assert r.max() <= 1.0, (r.max(), int(np.argmax(r)))


def test_hvp_matches_oracle(c0g):
    r = _ratio(c0g["hv"], c0g["hv_o"], c0g["floor"], c0g["dh"], REL_HVP)
    assert r.max() <= 1.0, (r.max(), int(np.argmax(r)))


def test_adjoint_is_deterministic(c0g):
    import torch
    g = c0g["plan"].backward(c0g["qd"], c0g["cot_d"])
    torch.cuda.synchronize()
    assert np.array_equal(g.cpu().numpy(), c0g["grad"].astype(np.float32))


def _check_step(c0g, out, grad, hv):
    err = PT.check_groups(out.cpu().numpy().T.astype(np.float64), c0g["g_rec"], c0g["LsG"], c0g["tau_b"])
    for k in ("pos", "logZ", "W", "n"):
        assert err[k] <= 1.0, (k, err)
    r = _ratio(grad.cpu().numpy().astype(np.float64), c0g["g_o"], c0g["floor"], c0g["dg"])
    assert r.max() <= 1.0, ("grad", r.max(), int(np.argmax(r)))
    if hv is not None:
        r = _ratio(hv.cpu().numpy().astype(np.float64), c0g["hv_o"], c0g["floor"], c0g["dh"], REL_HVP)
        assert r.max() <= 1.0, ("hvp", r.max(), int(np.argmax(r)))


def test_step_records_gradient_hvp(c0g):
    """cm_contacts_step with a direction: records, gradient and H v from one dual sweep."""
    import torch
    out, grad, hv = c0g["plan"].step(c0g["qd"], c0g["cot_d"], c0g["dir_d"])
    torch.cuda.synchronize()
    _check_step(c0g, out, grad, hv)


def test_step_records_gradient(c0g):
    """cm_contacts_step without a direction: records and gradient from one float sweep."""
    import torch
    out, grad, hv = c0g["plan"].step(c0g["qd"], c0g["cot_d"])
    torch.cuda.synchronize()
    assert hv is None
    _check_step(c0g, out, grad, None)


def test_adjoint_past_the_tape(c0g):
    """A context whose memory budget holds a tape for only a few hundred tiles:
    the adjoint recomputes the forward sweep for the tiles past it.  Gradient
    and H v (separate calls and the one-pass step) stay within the tolerances
    of the oracle; the log reports whether they are bitwise those of the
    fully taped plan."""
    import torch
    from paper_2604_17538_amd import api
    w = W.config0()
    ctx = api.Context(0, L_ref=w.L_ref, budget_bytes=16 << 20)
    hs = ctx.build_objects(w.objects)
    plan = ctx.plan(hs[w.qa], hs[w.qb])
    qd = plan.device_queries(w.poses)
    grad = plan.backward(qd, c0g["cot_d"])
    grad2 = torch.empty_like(grad)
    hv = plan.hvp(qd, c0g["cot_d"], c0g["dir_d"], grad=grad2)
    out, g3, h3 = plan.step(qd, c0g["cot_d"], c0g["dir_d"])
    torch.cuda.synchronize()
    tiles = plan.stats()["tiles"]
    _step("tape overflow: %d tiles; bitwise equal to the taped plan: grad %s, H v %s" % (
        tiles, np.array_equal(grad.cpu().numpy(), c0g["grad"].astype(np.float32)),
        np.array_equal(hv.cpu().numpy(), c0g["hv"].astype(np.float32))))
    assert tiles > 4 * 240  # most tiles lie past a tape of about 240 tiles
    for gg in (grad, grad2, g3):
        r = _ratio(gg.cpu().numpy().astype(np.float64), c0g["g_o"], c0g["floor"], c0g["dg"])
        assert r.max() <= 1.0, ("grad", r.max())
    for hh in (hv, h3):
        r = _ratio(hh.cpu().numpy().astype(np.float64), c0g["hv_o"], c0g["floor"], c0g["dh"], REL_HVP)
        assert r.max() <= 1.0, ("hvp", r.max())
    _check_step(c0g, out, g3, h3)
