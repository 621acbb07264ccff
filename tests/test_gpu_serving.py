"""GPU tests of the serving loop: every request's results equal those of the
same queries run alone through a plan (bitwise: reductions are per query and
in a fixed order), for mixed forward / forward+gradient traffic arriving while
earlier batches are on the device; admission respects the memory budget.  A
gradient request's records come from the sweep that also feeds its adjoint
(cm_contacts_step), not from a second forward pass."""
import numpy as np
import pytest

from paper_2604_17538_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import torch
    from paper_2604_17538_amd import api
    objs = W.library_objects(24)
    ctx = api.Context(0, L_ref=0.1)
    hs = ctx.build_objects(objs)
    return api, ctx, hs, objs


def _alone(api, ctx, hs, qa, qb, poses, cot):
    """The same queries in a plan of their own: records by the forward pass for
    a forward request; records and gradient from one sweep (cm_contacts_step,
    as the server runs a gradient request) for a gradient request."""
    import torch
    plan = ctx.plan(qa, qb)
    qd = plan.device_queries(poses)
    grad = None
    if cot is None:
        out = plan.forward(qd)
    else:
        cd = torch.tensor(np.ascontiguousarray(cot.T, np.float32)).contiguous().cuda()
        out, g, _ = plan.step(qd, cd)
        grad = g.cpu().numpy()
    torch.cuda.synchronize()
    return out.cpu().numpy().T, grad


def test_mixed_stream_equals_alone(lib):
    api, ctx, hs, objs = lib
    tr = W.serving_trace(objs, rate_hz=2000.0, duration_s=0.03, seed=5, max_pairs=16)
    srv = api.Server(ctx)
    tickets, reqs = [], []
    rng = np.random.default_rng(0)
    for r in range(len(tr.n_pairs)):
        qa, qb = hs[tr.pair_a[r]], hs[tr.pair_b[r]]
        G = sum(ctx.object_info(int(a))[0] + ctx.object_info(int(b))[0] for a, b in zip(qa, qb))
        cot = rng.standard_normal((G, 12)) if tr.want_grad[r] else None
        tickets.append(srv.submit(qa, qb, tr.poses[r], cot))
        reqs.append((qa, qb, tr.poses[r], cot))
    assert len(tickets) >= 20
    for t, (qa, qb, poses, cot) in zip(tickets, reqs):
        out, grad = t.wait()
        o_ref, g_ref = _alone(api, ctx, hs, qa, qb, poses, cot)
        assert np.array_equal(out, o_ref)
        if cot is not None:
            assert np.array_equal(grad, g_ref)
    st = srv.stats()
    assert st["completed"] == len(tickets) and st["queued"] == 0
    assert st["batches"] < len(tickets)  # requests were batched together


def test_request_over_budget_is_rejected(lib):
    api, _, hs, objs = lib
    ctx2 = api.Context(0, L_ref=0.1, budget_bytes=4096)
    h2 = ctx2.build_objects(objs[:2])
    srv = api.Server(ctx2)
    with pytest.raises(api.CMError) as e:
        srv.submit(h2[:1], h2[1:2], np.array([[1, 0, 0, 0, 0, 0, 0, 1, 0, 0, 0, 0.3, 0, 0]]))
    assert e.value.status == -2
    with pytest.raises(api.CMError):  # degenerate quaternion
        srv.submit(h2[:1], h2[1:2], np.zeros((1, 14)))


def test_device_memory_held_stays_within_budget(lib):
    """A small budget (48 MiB) under a burst of mixed traffic: the slots'
    device buffers together never exceed it (the library's own record of the
    bytes it holds), every admitted request completes, and results stay bitwise
    those of the queries run alone."""
    api, _, _, objs = lib
    budget = 48 << 20
    ctx = api.Context(0, L_ref=0.1, budget_bytes=budget)
    hs = ctx.build_objects(objs)
    tr = W.serving_trace(objs, rate_hz=5000.0, duration_s=0.02, seed=9, max_pairs=48)
    srv = api.Server(ctx)
    rng = np.random.default_rng(1)
    tickets, reqs, refused = [], [], 0
    for r in range(len(tr.n_pairs)):
        qa, qb = hs[tr.pair_a[r]], hs[tr.pair_b[r]]
        G = sum(ctx.object_info(int(a))[0] + ctx.object_info(int(b))[0] for a, b in zip(qa, qb))
        cot = rng.standard_normal((G, 12)) if tr.want_grad[r] else None
        try:
            tickets.append(srv.submit(qa, qb, tr.poses[r], cot))
            reqs.append((qa, qb, tr.poses[r], cot))
        except api.CMError as e:
            assert e.status == -2  # this request alone exceeds the budget
            refused += 1
    assert len(tickets) >= 40
    for t in tickets:
        t.wait()
    st = srv.stats()
    assert st["completed"] == len(tickets)
    assert 0 < st["peak_device_bytes"] <= budget, st
    for t, (qa, qb, poses, cot) in list(zip(tickets, reqs))[::7]:
        o_ref, g_ref = _alone(api, ctx, hs, qa, qb, poses, cot)
        assert np.array_equal(t.out, o_ref)
        if cot is not None:
            assert np.array_equal(t.grad, g_ref)
