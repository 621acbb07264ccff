"""GPU parity on the differentiation workload (pairs of unions of 1-32 convex
pieces with 8-512 hull vertices each): element by element on a 32-pair batch
(several tiles per entry and ragged tails), with piece pruning on and off, and
on sampled queries of the full 16384-pair batch in the launch configuration the
benchmark times (records, gradient and H v from cm_contacts_step).

Tolerances are those of the config-0 tests: positions and distances 1e-5 L_s,
weights and normals 1e-4, gradients and H v 1e-4 relative, each
derivative also allowed 4 times the query's FP32 spread (oracle.fp32_spread)."""
import sys

import numpy as np
import pytest

import oracle as O
from paper_2604_17538_amd import workloads as W
from tests import parity as PT

pytestmark = pytest.mark.gpu

REL, REL_HVP, K_SPREAD = 1e-4, 1e-4, 4.0


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


def _allowed_ratio(a, b, floor, spread, rel):
    nb = np.linalg.norm(b, axis=1)
    allowed = np.maximum(rel * np.maximum(nb, floor), K_SPREAD * spread)
    return np.linalg.norm(a - b, axis=1) / allowed


def _oracle(w, sel, threads=16):
    prm = O.default_params(w.L_ref)
    objs = {}
    for i in sel:
        for j in (int(w.qa[i]), int(w.qb[i])):
            if j not in objs:
                objs[j] = O.from_workload_object(w.objects[j])
                objs[j].build_grid(prm)
    ol = [objs.get(j) for j in range(len(w.objects))]
    qa, qb, poses = w.qa[sel], w.qb[sel], w.poses[sel]
    g_o, c_o, goff, coff = O.contacts(prm, ol, qa, qb, poses, want_contacts=True, threads=threads)
    cot = W.cotangents(w.cot_seed, goff[-1])
    direc = W.directions(w.cot_seed, len(sel))
    gr_o, hv_o = O.grad_hvp(prm, ol, qa, qb, poses, cot, direc, threads=threads)
    dg, dh = O.fp32_spread(prm, ol, qa, qb, poses, cot, direc, seeds=(1, 2), threads=threads)
    r = np.array([o.radius() if o is not None else 0.0 for o in ol])
    Lq = r[qa] + r[qb]
    cq = np.sqrt(np.add.reduceat((cot ** 2).sum(1), goff[:-1]))
    return dict(prm=prm, objs=ol, g_o=g_o, c_o=c_o, goff=goff, coff=coff, cot=cot, dir=direc, gr_o=gr_o,
                hv_o=hv_o, dg=dg, dh=dh, Lq=Lq, floor=1e-3 * cq * np.maximum(1.0, Lq))


def _check_records(g, ref, name):
    err = PT.check_groups(g, ref["g_o"], np.repeat(ref["Lq"], np.diff(ref["goff"])), ref["prm"].tau_blend)
    for k in ("pos", "logZ", "W", "n"):
        assert err[k] <= 1.0, (name, k, err)


def _check_derivs(grad, hv, ref, name):
    r = _allowed_ratio(grad, ref["gr_o"], ref["floor"], ref["dg"], REL)
    _log("%s: gradient max error / allowed %.3f" % (name, r.max()))
    assert r.max() <= 1.0, (name, "grad", r.max(), int(np.argmax(r)))
    r = _allowed_ratio(hv, ref["hv_o"], ref["floor"], ref["dh"], REL_HVP)
    _log("%s: H v max error / allowed %.3f" % (name, r.max()))
    assert r.max() <= 1.0, (name, "hvp", r.max(), int(np.argmax(r)))


@pytest.fixture(scope="module")
def small():
    w = W.config2(n_pairs=32)
    _log("c2 small: oracle")
    return w, _oracle(w, np.arange(w.n))


@pytest.mark.parametrize("prune", [1, 0])
def test_small_batch_element_by_element(small, prune):
    import torch
    from paper_2604_17538_amd import api
    w, ref = small
    ctx = api.Context(0, L_ref=w.L_ref, prune_pieces=prune)
    hs = ctx.build_objects(w.objects)
    plan = ctx.plan(hs[w.qa], hs[w.qb])
    assert np.array_equal(plan.group_off, ref["goff"]) and np.array_equal(plan.contact_off, ref["coff"])
    qd = plan.device_queries(w.poses)
    out, dbg = plan.forward(qd, debug=True)
    cot_d = torch.tensor(np.ascontiguousarray(ref["cot"].T, np.float32)).cuda()
    dir_d = torch.tensor(ref["dir"].astype(np.float32)).cuda()
    out2, grad, hv = plan.step(qd, cot_d, dir_d)
    torch.cuda.synchronize()
    _check_records(out.cpu().numpy().T.astype(np.float64), ref, "forward prune=%d" % prune)
    _check_records(out2.cpu().numpy().T.astype(np.float64), ref, "step prune=%d" % prune)
    # per-contact records: survivors bit-exact outside the tie band, distances and points to 1e-5 L_s
    ex = [ctx.object_export(h) for h in hs]
    perm_obj = [PT.contact_perm(ex[i], ref["objs"][i]) for i in range(len(hs))]
    perm = PT.query_contact_perm(perm_obj, w.qa, w.qb, ref["coff"])
    c, co = dbg.cpu().numpy().T.astype(np.float64), ref["c_o"][perm]
    band = (np.abs(co[:, 12] - ref["prm"].d_max) <= PT.BAND) | (co[:, 13] <= PT.BAND)
    assert not np.any((c[:, 0] != co[:, 0]) & ~band)
    LsC = np.repeat(ref["Lq"], np.diff(ref["coff"]))
    dpos = np.abs(c[:, [1, 4, 5, 6]] - co[:, [1, 4, 5, 6]]).max(1) / (PT.POS_TOL * LsC)
    assert dpos.max() <= 1.0, dpos.max()
    _check_derivs(grad.cpu().numpy().astype(np.float64), hv.cpu().numpy().astype(np.float64), ref,
                  "step prune=%d" % prune)


def test_full_batch_sampled():
    """The 16384-pair batch in one plan, as the benchmark runs it; 8 queries
    spread over the batch are checked against the oracle run on them alone."""
    import torch
    from paper_2604_17538_amd import api
    w = W.config2()
    ctx = api.Context(0, L_ref=w.L_ref)
    hs = ctx.build_objects(w.objects)
    plan = ctx.plan(hs[w.qa], hs[w.qb])
    qd = plan.device_queries(w.poses)
    sel = np.linspace(0, w.n - 1, 8).astype(np.int64)
    ref = _oracle(w, sel)
    # cotangents and directions for the whole batch; the sampled queries get the oracle's
    cot = np.zeros((plan.G, 12), np.float32)
    direc = np.zeros((w.n, 12), np.float32)
    rng = np.random.default_rng(5)
    cot[:] = rng.standard_normal(cot.shape)
    direc[:] = rng.standard_normal(direc.shape)
    for k, i in enumerate(sel):
        cot[plan.group_off[i]:plan.group_off[i + 1]] = ref["cot"][ref["goff"][k]:ref["goff"][k + 1]]
        direc[i] = ref["dir"][k]
    cot_d = torch.tensor(np.ascontiguousarray(cot.T)).cuda()
    dir_d = torch.tensor(direc).cuda()
    out, grad, hv = plan.step(qd, cot_d, dir_d)
    torch.cuda.synchronize()
    g = out.cpu().numpy().T.astype(np.float64)
    rows = np.concatenate([np.arange(plan.group_off[i], plan.group_off[i + 1]) for i in sel])
    _check_records(g[rows], ref, "full batch")
    _check_derivs(grad.cpu().numpy()[sel].astype(np.float64), hv.cpu().numpy()[sel].astype(np.float64), ref,
                  "full batch")


@pytest.mark.parametrize("variant", ["tight_edge_bound", "no_broad_phase"])
def test_broad_phase_variants(small, variant):
    """The broad phase changes which contacts are evaluated, never an output:
    with the tighter edge bound (max(max(lb1, lb2) - l, (lb1 + lb2 - l) / 2))
    the masks equal the oracle's under the same bound (bit-exact outside the
    tie band) and filter at least as much as the paper's min form; with the
    broad phase off every contact survives.  Records, gradient and H v stay
    within the tolerances of the default oracle."""
    import torch
    from paper_2604_17538_amd import api
    w, ref = small
    kw = {"edge_bound": 1} if variant == "tight_edge_bound" else {"broad_phase": 0}
    ctx = api.Context(0, L_ref=w.L_ref, **kw)
    hs = ctx.build_objects(w.objects)
    plan = ctx.plan(hs[w.qa], hs[w.qb])
    qd = plan.device_queries(w.poses)
    out, dbg = plan.forward(qd, debug=True)
    cot_d = torch.tensor(np.ascontiguousarray(ref["cot"].T, np.float32)).cuda()
    dir_d = torch.tensor(ref["dir"].astype(np.float32)).cuda()
    out2, grad, hv = plan.step(qd, cot_d, dir_d)
    torch.cuda.synchronize()
    _check_records(out.cpu().numpy().T.astype(np.float64), ref, variant)
    _check_records(out2.cpu().numpy().T.astype(np.float64), ref, variant + " step")
    _check_derivs(grad.cpu().numpy().astype(np.float64), hv.cpu().numpy().astype(np.float64), ref, variant)
    ex = [ctx.object_export(h) for h in hs]
    perm_obj = [PT.contact_perm(ex[i], ref["objs"][i]) for i in range(len(hs))]
    perm = PT.query_contact_perm(perm_obj, w.qa, w.qb, ref["coff"])
    mask = dbg.cpu().numpy().T.astype(np.float64)[:, 0]
    if variant == "no_broad_phase":
        assert np.all(mask == 1)
        return
    prm1 = O.default_params(w.L_ref, edge_bound=1)
    _, c1, _, _ = O.contacts(prm1, ref["objs"], w.qa, w.qb, w.poses, want_contacts=True, threads=16)
    c1 = c1[perm]
    band = (np.abs(c1[:, 12] - prm1.d_max) <= PT.BAND) | (c1[:, 13] <= PT.BAND)
    assert not np.any((mask != c1[:, 0]) & ~band)
    c0 = ref["c_o"][perm]
    assert np.all(c1[:, 0] <= c0[:, 0])  # the tighter bound filters a superset
    _log("%s: survivors %d of %d (paper's form %d)" % (variant, int(mask.sum()), len(mask), int(c0[:, 0].sum())))
