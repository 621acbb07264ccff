"""GPU test of cm_contacts_fwd_noalloc, the forward pass whose launch scratch
lives in the library's fixed device array: through the C ABI its group records
equal those of cm_contacts_fwd bit for bit, on two calls in a row (the second
with a smaller batch, so it reads what the first left in the shared array),
and a batch whose launch scratch exceeds the array is refused with nothing
launched."""
import numpy as np
import pytest

from paper_2604_17538_amd import workloads as W

pytestmark = pytest.mark.gpu


def _plan_pair(ctx, w, sel):
    hs = ctx.build_objects(w.objects)
    plan = ctx.plan(hs[w.qa[sel]], hs[w.qb[sel]])
    return plan, plan.device_queries(w.poses[sel])


def test_noalloc_equals_forward_twice():
    import torch
    from paper_2604_17538_amd import api
    # first call: 64 pairs of 8-piece objects; second call: 24 pair-queries of
    # the boxes / 64-point hulls workload (fewer entries, words and tiles)
    w1 = W.config1(n_envs=64)
    ctx1 = api.Context(0, L_ref=w1.L_ref)
    p1, q1 = _plan_pair(ctx1, w1, np.arange(w1.n))
    w0 = W.config0(n_poses=16)
    ctx0 = api.Context(0, L_ref=w0.L_ref)
    sel0 = np.r_[0:12, 16:28]
    p0, q0 = _plan_pair(ctx0, w0, sel0)
    for plan, qd in ((p1, q1), (p0, q0)):
        ref = plan.forward(qd)
        got = torch.full_like(ref, float("nan"))
        plan.forward_noalloc(qd, got)
        torch.cuda.synchronize()
        assert np.array_equal(got.cpu().numpy(), ref.cpu().numpy()), "records differ from cm_contacts_fwd"
        assert np.isfinite(got.cpu().numpy()).all()
    # the first plan again after the smaller one: the array holds the second
    # call's contents, which every launch overwrites or clears before use
    ref = p1.forward(q1)
    got = torch.full_like(ref, float("nan"))
    p1.forward_noalloc(q1, got)
    torch.cuda.synchronize()
    assert np.array_equal(got.cpu().numpy(), ref.cpu().numpy())


def test_noalloc_refuses_oversized_batch():
    import torch
    from paper_2604_17538_amd import api
    w = W.config0(n_poses=16)
    ctx = api.Context(0, L_ref=w.L_ref)
    hs = ctx.build_objects(w.objects)
    n = 65536  # pairs of 64-point hulls: about 1.6 KB of launch scratch each
    qa, qb = np.full(n, hs[2]), np.full(n, hs[3])
    plan = ctx.plan(qa, qb)
    poses = np.repeat(w.poses[16:17], n, axis=0)
    qd = plan.device_queries(poses)
    out = torch.zeros((12, plan.G), dtype=torch.float32, device="cuda")
    with pytest.raises(RuntimeError, match="launch scratch"):
        plan.forward_noalloc(qd, out)
    torch.cuda.synchronize()
    assert float(out.abs().max()) == 0.0  # nothing was launched
