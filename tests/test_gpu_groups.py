"""GPU parity of plane-group culling on pieces with many planes: pairs of
single-piece objects, hulls of 1000 ellipsoid points (about 2000 facets, so
more than 64 groups of 16 planes and a second 64-group mask chunk), and of a
box (6 planes: one group, mostly padding), element by element against the FP64
oracle with pruning on and off, and the two runs against each other.

Tolerances as for the 8-piece workload: positions and distances 1e-5 L_s,
weights 1e-4; broad-phase masks bit-exact outside the 1e-6 tie band."""
import sys

import numpy as np
import pytest

import oracle as O
from paper_2604_17538_amd import workloads as W
from tests import parity as PT

pytestmark = pytest.mark.gpu


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


def _workload():
    rng = np.random.Generator(np.random.PCG64(W.SEED_BASE + 61))
    objs = [W.multi_piece_object(rng, 1, [1000], axes_lo=0.05, axes_hi=0.12, centre=0.0) for _ in range(3)]
    objs.append(W.unit_box(0.1))
    qa = np.array([0, 1, 2, 3, 0], np.int32)
    qb = np.array([1, 2, 0, 1, 3], np.int32)
    radii = np.array([o.radius() if hasattr(o, "radius") else 0.0866 for o in objs])
    poses = W.random_poses(rng, radii[qa], radii[qb])
    return W.Workload("groups", objs, qa, qb, poses, 0.1)


@pytest.fixture(scope="module")
def case():
    w = _workload()
    prm = O.default_params(w.L_ref)
    ol = []
    for o in w.objects:
        oo = O.from_workload_object(o)
        oo.build_grid(prm)
        ol.append(oo)
    g_o, c_o, goff, coff = O.contacts(prm, ol, w.qa, w.qb, w.poses, want_contacts=True, threads=16)
    r = np.array([o.radius() for o in ol])
    return w, dict(prm=prm, objs=ol, g_o=g_o, c_o=c_o, goff=goff, coff=coff, Lq=r[w.qa] + r[w.qb])


def _run(w, prune):
    import torch
    from paper_2604_17538_amd import api
    ctx = api.Context(0, L_ref=w.L_ref, prune_pieces=prune)
    hs = ctx.build_objects(w.objects)
    plan = ctx.plan(hs[w.qa], hs[w.qb])
    qd = plan.device_queries(w.poses)
    out, dbg = plan.forward(qd, debug=True)
    torch.cuda.synchronize()
    return ctx, hs, plan, out.cpu().numpy().T.astype(np.float64), dbg.cpu().numpy().T.astype(np.float64)


def test_many_planes_element_by_element(case):
    w, ref = case
    counts = [int(np.diff(o.plane_off)[0]) for o in ref["objs"][:3]]
    _log("groups: facets per piece %s" % counts)
    assert min(counts) > 64 * 16  # more than one 64-group mask chunk
    res = {}
    for prune in (1, 0):
        ctx, hs, plan, g, c = _run(w, prune)
        assert np.array_equal(plan.group_off, ref["goff"]) and np.array_equal(plan.contact_off, ref["coff"])
        err = PT.check_groups(g, ref["g_o"], np.repeat(ref["Lq"], np.diff(ref["goff"])), ref["prm"].tau_blend)
        _log("groups prune=%d: records %s" % (prune, err))
        for k in ("pos", "logZ", "W", "n"):
            assert err[k] <= 1.0, (prune, k, err)
        ex = [ctx.object_export(h) for h in hs]
        perm_obj = [PT.contact_perm(ex[i], ref["objs"][i]) for i in range(len(hs))]
        perm = PT.query_contact_perm(perm_obj, w.qa, w.qb, ref["coff"])
        co = ref["c_o"][perm]
        band = (np.abs(co[:, 12] - ref["prm"].d_max) <= PT.BAND) | (co[:, 13] <= PT.BAND)
        assert not np.any((c[:, 0] != co[:, 0]) & ~band)
        assert 0.0 < c[:, 0].mean() < 1.0
        LsC = np.repeat(ref["Lq"], np.diff(ref["coff"]))
        dpos = np.abs(c[:, [1, 4, 5, 6]] - co[:, [1, 4, 5, 6]]).max(1) / (PT.POS_TOL * LsC)
        wgt, wo = c[:, 3], co[:, 3]
        rel = np.where(wo >= PT.W_FLOOR, np.abs(wgt - wo) / (PT.REL_TOL * wo), np.abs(wgt - wo) / 1e-10)
        _log("groups prune=%d: contacts %d, survivors %.3f, pos %.3f, weights %.3f of the tolerance"
             % (prune, len(c), c[:, 0].mean(), dpos.max(), rel.max()))
        assert dpos.max() <= 1.0 and rel.max() <= 1.0
        res[prune] = (g, c)
    # culling removes only terms below FP32 resolution: the two runs agree far inside the tolerance
    d = PT.check_groups(res[1][0], res[0][0], np.repeat(ref["Lq"], np.diff(ref["goff"])), ref["prm"].tau_blend)
    _log("groups: prune on vs off %s" % d)
    assert d["pos"] <= 0.1 and d["logZ"] <= 0.1
