"""GPU parity of the Jacobian-vector product (cm_contacts_jvp) on the full
config-0 batch against the FP64 oracle.

Element by element: every group's tangent record (J v)_g against the oracle's
own Jacobian-vector product (one dual slot seeded with v), norm-wise over the
12 components with logZ's scaled by tau_b (a length, like the others), held to
max(1e-4 max(|ref|, 1e-3 max(1, L_s)), 4 x the oracle's FP32 spread of it).

Beside it, the tangent records J v along a unit direction v per query are checked through
the identity sum_g <c_g, (J v)_g> = grad_xi <c, y> . v for random cotangents c:
the right side is the oracle's hyper-dual gradient, so every component of J v
is weighed against the oracle (two independent cotangents per query).  The
tolerance is the gradient's: 1e-4 relative (floor 1e-3 |c| max(1, L_s)), or 4
times the query's FP32 spread (|v| = 1 bounds the projection of the gradient's
spread).  The records written beside the tangents match the oracle's forward
records to the forward tolerances."""
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


def test_jvp_matches_oracle_gradient_projections():
    import torch
    from paper_2604_17538_amd import api
    w = W.config0()
    prm = O.default_params(w.L_ref)
    objs = [O.from_workload_object(o) for o in w.objects]
    for o in objs:
        o.build_grid(prm)
    g_o, goff = O.contacts(prm, objs, w.qa, w.qb, w.poses, threads=16)
    v = W.directions(41, w.n)
    r = np.array([o.radius() for o in objs])
    Lq = r[w.qa] + r[w.qb]

    ctx = api.Context(0, L_ref=w.L_ref)
    hs = ctx.build_objects(w.objects)
    plan = ctx.plan(hs[w.qa], hs[w.qb])
    qd = plan.device_queries(w.poses)
    out, out_t = plan.jvp(qd, torch.tensor(v.astype(np.float32)).cuda())
    torch.cuda.synchronize()
    y = out.cpu().numpy().T.astype(np.float64)
    jv = out_t.cpu().numpy().T.astype(np.float64)
    err = PT.check_groups(y, g_o, np.repeat(Lq, np.diff(goff)), prm.tau_blend)
    _log("jvp records: %s" % err)
    for k in ("pos", "logZ", "W", "n"):
        assert err[k] <= 1.0, (k, err)
    assert np.all(np.isfinite(jv))
    _, jv_o, _ = O.jvp(prm, objs, w.qa, w.qb, w.poses, v, threads=16)
    sp = O.jvp_spread(prm, objs, w.qa, w.qb, w.poses, v, threads=16)
    sc = np.ones(12)
    sc[11] = prm.tau_blend
    LsG = np.repeat(Lq, np.diff(goff))
    nref = np.linalg.norm(jv_o * sc, axis=1)
    allowed = np.maximum(REL * np.maximum(nref, 1e-3 * np.maximum(1.0, LsG)), K_SPREAD * sp)
    ratio = np.linalg.norm((jv - jv_o) * sc, axis=1) / allowed
    _log("jvp tangents element by element: max error / allowed %.3f (group %d); %d of %d groups held to the "
         "FP32 spread" % (ratio.max(), int(np.argmax(ratio)),
                          int(np.count_nonzero(K_SPREAD * sp > REL * np.maximum(nref, 1e-3 * np.maximum(1.0, LsG)))),
                          len(ratio)))
    assert ratio.max() <= 1.0
    for seed in (42, 43):
        cot = W.cotangents(seed, goff[-1])
        gr = O.grad_hvp(prm, objs, w.qa, w.qb, w.poses, cot, threads=16)
        dg, _ = O.fp32_spread(prm, objs, w.qa, w.qb, w.poses, cot, seeds=(1, 2), threads=16)
        s_gpu = np.add.reduceat((cot * jv).sum(1), goff[:-1])
        s_o = (gr * v).sum(1)
        cq = np.sqrt(np.add.reduceat((cot ** 2).sum(1), goff[:-1]))
        floor = 1e-3 * cq * np.maximum(1.0, Lq)
        allowed = np.maximum(REL * np.maximum(np.linalg.norm(gr, axis=1), floor), K_SPREAD * dg)
        ratio = np.abs(s_gpu - s_o) / allowed
        _log("jvp cotangent seed %d: max error / allowed %.3f (query %d)" % (seed, ratio.max(), int(np.argmax(ratio))))
        assert ratio.max() <= 1.0
