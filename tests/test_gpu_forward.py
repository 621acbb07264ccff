"""GPU parity of the forward pass against the FP64 oracle (config 0 in full:
two unit boxes and two 64-point ellipsoid hulls at 256 seeded poses each),
element by element: group records, per-contact records, broad-phase masks and
the voxel grids."""
import numpy as np
import pytest

import oracle as O
from paper_2604_17538_amd import workloads as W
from tests import parity as PT

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def c0():
    import torch
    from paper_2604_17538_amd import api
    w = W.config0()
    prm = O.default_params(w.L_ref)
    objs = [O.from_workload_object(o) for o in w.objects]
    for o in objs:
        o.build_grid(prm)
    g_o, c_o, goff, coff = O.contacts(prm, objs, w.qa, w.qb, w.poses, want_contacts=True, threads=8)
    ctx = api.Context(0, L_ref=w.L_ref)
    hs = ctx.build_objects(w.objects)
    plan = ctx.plan(hs[w.qa], hs[w.qb])
    qd = plan.device_queries(w.poses)
    out, dbg = plan.forward(qd, debug=True)
    torch.cuda.synchronize()
    ex = [ctx.object_export(h) for h in hs]
    perm_obj = [PT.contact_perm(ex[i], objs[i]) for i in range(len(objs))]
    perm = PT.query_contact_perm(perm_obj, w.qa, w.qb, coff)
    return dict(w=w, prm=prm, objs=objs, g_o=g_o, c_o=c_o, goff=goff, coff=coff, ctx=ctx, hs=hs, plan=plan,
                g=out.cpu().numpy().T.astype(np.float64), c=dbg.cpu().numpy().T.astype(np.float64), perm=perm,
                qd=qd)


def _Ls(d):
    w, objs = d["w"], d["objs"]
    r = np.array([o.radius() for o in objs])
    Lq = r[w.qa] + r[w.qb]
    return np.repeat(Lq, np.diff(d["goff"])), np.repeat(Lq, np.diff(d["coff"]))


def test_layout_matches_oracle(c0):
    assert np.array_equal(c0["plan"].group_off, c0["goff"])
    assert np.array_equal(c0["plan"].contact_off, c0["coff"])


def test_grids_match(c0):
    for h, o in zip(c0["hs"], c0["objs"]):
        Gp, org_p, h_p, r_p = c0["ctx"].object_grid(h)
        Go, org_o, h_o, r_o = o.grid()
        assert np.allclose(org_p, org_o, atol=1e-6) and np.allclose(h_p, h_o, rtol=1e-6)
        assert abs(r_p - r_o) < 1e-6
        assert np.abs(Gp - Go).max() <= PT.POS_TOL * 2 * o.radius()


def test_broad_phase_masks_bit_exact(c0):
    c, co, perm = c0["c"], c0["c_o"], c0["perm"]
    mo = co[perm, 0]
    mg = c[:, 0]
    diff = mo != mg
    band = (np.abs(co[perm, 12] - c0["prm"].d_max) <= PT.BAND) | (co[perm, 13] <= PT.BAND)
    assert not np.any(diff & ~band), "mask mismatch outside the tie band: %d" % np.sum(diff & ~band)
    assert 0.05 < mg.mean() < 0.99


def test_group_records_within_tolerance(c0):
    LsG, _ = _Ls(c0)
    err = PT.check_groups(c0["g"], c0["g_o"], LsG, c0["prm"].tau_blend)
    for k in ("pos", "logZ", "W", "n"):
        assert err[k] <= 1.0, (k, err)


def test_contact_records_within_tolerance(c0):
    _, LsC = _Ls(c0)
    c, co = c0["c"], c0["c_o"][c0["perm"]]
    both = (c[:, 0] == 1) & (co[:, 0] == 1)
    assert np.all(c[:, 11] == co[:, 11])  # kind
    dpos = np.abs(c[:, [1, 4, 5, 6]] - co[:, [1, 4, 5, 6]]).max(1) / (PT.POS_TOL * LsC)
    assert dpos.max() <= 1.0, dpos.max()
    # raw phi of contacts that both sides evaluated
    assert (np.abs(c[both, 10] - co[both, 10]) / (PT.POS_TOL * LsC[both])).max() <= 1.0
    dn = np.abs(c[:, 7:10] - co[:, 7:10]).max(1)
    assert dn.max() <= PT.REL_TOL, dn.max()
    w, wo = c[:, 3], co[:, 3]
    rel = np.where(wo >= PT.W_FLOOR, np.abs(w - wo) / (PT.REL_TOL * wo), np.abs(w - wo) / 1e-10)
    assert rel.max() <= 1.0, rel.max()
    df = np.abs(c[:, 2] - co[:, 2])
    assert df.max() <= 1e-4


def test_rerun_is_bitwise_deterministic(c0):
    import torch
    out2, dbg2 = c0["plan"].forward(c0["qd"], debug=True)
    torch.cuda.synchronize()
    assert np.array_equal(out2.cpu().numpy().T, c0["g"].astype(np.float32))
