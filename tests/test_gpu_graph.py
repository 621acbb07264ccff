"""GPU tests of the captured step (cm_graph_*) and the launch-shape autotuner:
every replay of a graph, with the program's own eager launches and
synchronisations between replays, gives bitwise the results of the eager
cm_contacts_step; a replay after new poses are written into the captured query
buffer gives the eager results for those poses; the launch shape the autotuner
picks, for the dual sweeps and for the float sweeps, changes no result
(fixed-order reductions)."""
import numpy as np
import pytest

from paper_2604_17538_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def setup():
    import torch
    from paper_2604_17538_amd import api
    w = W.config0()
    ctx = api.Context(0, L_ref=w.L_ref)
    hs = ctx.build_objects(w.objects)
    plan = ctx.plan(hs[w.qa], hs[w.qb])
    qd = plan.device_queries(w.poses)
    cot = torch.tensor(np.ascontiguousarray(W.cotangents(5, plan.G).T, np.float32)).cuda()
    direc = torch.tensor(W.directions(5, w.n).astype(np.float32)).cuda()
    return dict(torch=torch, api=api, w=w, ctx=ctx, hs=hs, plan=plan, qd=qd, cot=cot, dir=direc)


def _eager(s, qd):
    out, grad, hv = s["plan"].step(qd, s["cot"], s["dir"])
    s["torch"].cuda.synchronize()
    return out.cpu().numpy(), grad.cpu().numpy(), hv.cpu().numpy()


def test_graph_replays_match_eager(setup):
    s = setup
    torch, plan = s["torch"], s["plan"]
    ref = _eager(s, s["qd"])
    out = torch.empty((12, plan.G), dtype=torch.float32, device="cuda")
    grad = torch.empty((plan.n, 12), dtype=torch.float32, device="cuda")
    hv = torch.empty_like(grad)
    g = plan.graph(s["qd"], s["cot"], grad, s["dir"], hv, out)
    other = s["ctx"].plan(s["hs"][s["w"].qa[:7]], s["hs"][s["w"].qb[:7]])
    oq = other.device_queries(s["w"].poses[:7])
    for k in range(4):
        out.zero_(); grad.zero_(); hv.zero_()
        g.launch()
        torch.cuda.synchronize()
        for a, b in zip((out, grad, hv), ref):
            assert np.array_equal(a.cpu().numpy(), b), "replay %d" % k
        other.forward(oq)  # eager work of the program between replays
        torch.cuda.synchronize()
    # new poses into the captured buffer: the replay computes them
    poses2 = s["w"].poses.copy()
    poses2[:, 11:14] *= 0.97
    s["qd"].copy_(s["plan"].device_queries(poses2))
    ref2 = _eager(s, s["qd"])
    assert not np.array_equal(ref2[1], ref[1])
    g.launch()
    torch.cuda.synchronize()
    for a, b in zip((out, grad, hv), ref2):
        assert np.array_equal(a.cpu().numpy(), b)
    s["qd"].copy_(s["plan"].device_queries(s["w"].poses))
    del g


def _eager_float(s, qd):
    out, grad, _ = s["plan"].step(qd, s["cot"])
    s["torch"].cuda.synchronize()
    return out.cpu().numpy(), grad.cpu().numpy()


def test_autotune_changes_no_result(setup):
    s = setup
    ref = _eager(s, s["qd"])
    ref_f = _eager_float(s, s["qd"])
    torch, plan = s["torch"], s["plan"]
    grad = torch.empty((plan.n, 12), dtype=torch.float32, device="cuda")
    hv = torch.empty_like(grad)
    best = plan.autotune(s["qd"], s["cot"], grad, s["dir"], hv)
    best_f = plan.autotune(s["qd"], s["cot"], grad)  # the float sweeps' shape
    wf, wd = plan.wg_waves
    # resident waves per CU from {8, 16, 24, 32, 48, 64}, workgroups of 1, 2 or 4 waves
    for c, v in ((best, wd), (best_f, wf)):
        assert v in (1, 2, 4) and c * v in (8, 16, 24, 32, 48, 64), (c, v)
    got = _eager(s, s["qd"])
    for a, b in zip(got, ref):
        assert np.array_equal(a, b)
    for a, b in zip(_eager_float(s, s["qd"]), ref_f):
        assert np.array_equal(a, b)


def test_launch_shape_setter(setup):
    s = setup
    plan = s["plan"]
    ref = _eager(s, s["qd"])
    keep, keep_w = plan.launch_shape, plan.wg_waves
    plan.launch_shape = (3, 5)
    assert plan.launch_shape == (3, 5)
    for a, b in zip(_eager(s, s["qd"]), ref):
        assert np.array_equal(a, b)
    plan.launch_shape, plan.wg_waves = (40, 9), (1, 2)  # one- and two-wave workgroups
    for a, b in zip(_eager(s, s["qd"]), ref):
        assert np.array_equal(a, b)
    with pytest.raises(s["api"].CMError):
        plan.launch_shape = (0, 5)
    with pytest.raises(s["api"].CMError):
        plan.wg_waves = (3, 4)
    assert plan.launch_shape == (40, 9) and plan.wg_waves == (1, 2)
    plan.launch_shape, plan.wg_waves = keep, keep_w


def _batch_inputs(s, sel, plan):
    """Poses, cotangents [12, G] and directions [n, 12] of the queries `sel`."""
    w = s["w"]
    return (w.poses[sel], np.ascontiguousarray(W.cotangents(11 + len(sel), plan.G).T, np.float32),
            W.directions(11 + len(sel), len(sel)).astype(np.float32))


def test_reserved_plan_graph_serves_any_batch(setup):
    """One graph captured on a reserved plan (cm_plan_reserve) replays
    whichever batch cm_plan_refill last put into it: two batches of different
    sizes and objects, alternated, each replay bitwise equal to the eager step
    of a plan made for that batch alone; a batch beyond the capacity is
    refused and the plan keeps the one it held."""
    s = setup
    torch, api, ctx, hs, w = s["torch"], s["api"], s["ctx"], s["hs"], s["w"]
    sels = [np.arange(40), np.arange(100, 123)]
    plains = [ctx.plan(hs[w.qa[sel]], hs[w.qb[sel]]) for sel in sels]
    refs = []
    for sel, p in zip(sels, plains):
        poses, cot, direc = _batch_inputs(s, sel, p)
        qd = p.device_queries(poses)
        out, grad, hv = p.step(qd, torch.tensor(cot).cuda(), torch.tensor(direc).cuda())
        torch.cuda.synchronize()
        refs.append((out.cpu().numpy(), grad.cpu().numpy(), hv.cpu().numpy()))
    cap_n = max(len(sel) for sel in sels)
    cap_G = max(p.G for p in plains) + 5
    cap_C = max(p.C for p in plains) + 100
    rp = api.Plan.reserve(ctx, cap_n, cap_G, cap_C)
    assert (rp.rows_n, rp.rows_G, rp.cap_C) == (cap_n, cap_G, cap_C) and rp.n == 0
    q_buf = torch.zeros((cap_n, 64), dtype=torch.uint8, device="cuda")
    cot_buf = torch.zeros((12, cap_G), dtype=torch.float32, device="cuda")
    dir_buf = torch.zeros((cap_n, 12), dtype=torch.float32, device="cuda")
    out = torch.zeros((12, cap_G), dtype=torch.float32, device="cuda")
    grad = torch.zeros((cap_n, 12), dtype=torch.float32, device="cuda")
    hv = torch.zeros_like(grad)

    def load(k):
        sel, p = sels[k], plains[k]
        rp.refill(hs[w.qa[sel]], hs[w.qb[sel]])
        assert rp.G == p.G and rp.n == len(sel) and np.array_equal(rp.group_off, p.group_off)
        poses, cot, direc = _batch_inputs(s, sel, p)
        rp.write_queries(q_buf, poses)
        cot_buf.zero_()
        cot_buf[:, : p.G].copy_(torch.tensor(cot))
        dir_buf.zero_()
        dir_buf[: len(sel)].copy_(torch.tensor(direc))

    def check(k, what):
        p = plains[k]
        torch.cuda.synchronize()
        got = (out.cpu().numpy()[:, : p.G], grad.cpu().numpy()[: p.n], hv.cpu().numpy()[: p.n])
        for a, b, name in zip(got, refs[k], ("records", "gradient", "H v")):
            assert np.array_equal(a, b), "%s: batch %d %s" % (what, k, name)

    load(0)
    rp.step(q_buf, cot_buf, dir_buf, out=out, grad=grad, hv=hv)
    check(0, "eager on the reserved plan")
    g = rp.graph(q_buf, cot_buf, grad, dir_buf, hv, out)
    for rep, k in enumerate((0, 1, 0, 1)):
        load(k)
        out.zero_(); grad.zero_(); hv.zero_()
        g.launch()
        check(k, "replay %d" % rep)
        plains[1 - k].forward(plains[1 - k].device_queries(w.poses[sels[1 - k]]))  # eager work between replays
        torch.cuda.synchronize()
    # a batch beyond the capacity is refused; the plan keeps batch 1
    big = np.arange(cap_n + 1)
    with pytest.raises(api.CMError):
        rp.refill(hs[w.qa[big]], hs[w.qb[big]])
    assert rp.n == len(sels[1])
    out.zero_(); grad.zero_(); hv.zero_()
    g.launch()
    check(1, "replay after a refused refill")
    del g
