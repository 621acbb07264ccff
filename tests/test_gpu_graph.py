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
    assert best in (2, 4, 6, 8, 12, 16)
    best_f = plan.autotune(s["qd"], s["cot"], grad)  # the float sweeps' shape
    assert best_f in (2, 4, 6, 8, 12, 16)
    got = _eager(s, s["qd"])
    for a, b in zip(got, ref):
        assert np.array_equal(a, b)
    for a, b in zip(_eager_float(s, s["qd"]), ref_f):
        assert np.array_equal(a, b)


def test_launch_shape_setter(setup):
    s = setup
    plan = s["plan"]
    ref = _eager(s, s["qd"])
    keep = plan.launch_shape
    plan.launch_shape = (3, 5)
    assert plan.launch_shape == (3, 5)
    for a, b in zip(_eager(s, s["qd"]), ref):
        assert np.array_equal(a, b)
    with pytest.raises(s["api"].CMError):
        plan.launch_shape = (0, 5)
    assert plan.launch_shape == (3, 5)
    plan.launch_shape = keep
