"""Host test of the autograd layer (api.ContactFn and its backward Functions)
with a stand-in plan whose records are a known quadratic function of the pose
perturbation xi: y(xi) = y0 + J xi + 1/2 T[xi, xi].  The stand-in answers the
four calls the layer makes (forward, backward = J^T c, hvp = (sum_k c_k T_k) u,
jvp = J u) in closed form, so torch.autograd.grad and
torch.autograd.functional.hvp through ContactFn can be compared with autograd
of the same quadratic written in torch: this checks how the layer composes
the library's entry points (which calls, with which cotangents), for linear
and nonlinear losses of the records.  The entry points themselves are checked
on the GPU (tests/test_gpu_autograd.py)."""
import numpy as np
import pytest
import torch

from paper_2604_17538_amd import api

N, G = 3, 4  # queries, groups


class QuadPlan:
    def __init__(self, seed=0):
        g = torch.Generator().manual_seed(seed)
        self.n, self.G = N, G
        m, k = 12 * G, 12 * N
        self.y0 = torch.randn(m, generator=g, dtype=torch.float64)
        self.J = torch.randn(m, k, generator=g, dtype=torch.float64)
        T = torch.randn(m, k, k, generator=g, dtype=torch.float64)
        self.T = 0.5 * (T + T.transpose(1, 2))
        self.calls = []

    # records as [12, G]; xi as [n, 12]
    def _rec(self, flat):
        return flat.reshape(12, G)

    def forward(self, q_dev):
        self.calls.append("fwd")
        return self._rec(self.y0.clone())

    def backward(self, q_dev, cot):
        self.calls.append("bwd")
        return (self.J.T @ cot.reshape(-1)).reshape(N, 12)

    def hvp(self, q_dev, cot, u):
        self.calls.append("hvp")
        Hc = torch.einsum("k,kij->ij", cot.reshape(-1), self.T)
        return (Hc @ u.reshape(-1)).reshape(N, 12)

    def jvp(self, q_dev, u):
        self.calls.append("jvp")
        return self._rec(self.y0.clone()), self._rec(self.J @ u.reshape(-1))

    def reference(self, xi):
        x = xi.reshape(-1)
        return self._rec(self.y0 + self.J @ x + 0.5 * torch.einsum("kij,i,j->k", self.T, x, x))


LOSSES = {
    "linear": lambda y, c: (c * y).sum(),
    "squared_depth": lambda y, c: (y[6] ** 2).sum() + (c * y).sum(),
    "quartic": lambda y, c: ((y * c).sum(0) ** 2).sum() ** 2 * 1e-2,
}


@pytest.mark.parametrize("loss", sorted(LOSSES))
def test_contactfn_grad_and_hvp_match_torch_autograd(loss):
    P = QuadPlan()
    c = torch.randn(12, G, dtype=torch.float64, generator=torch.Generator().manual_seed(1))
    v = torch.randn(N, 12, dtype=torch.float64, generator=torch.Generator().manual_seed(2))
    fn = LOSSES[loss]
    ContactFn = api.ContactFn

    def f(xi):
        return fn(ContactFn.apply(xi, P, None), c)

    def f_ref(xi):
        return fn(P.reference(xi), c)

    xi = torch.zeros(N, 12, dtype=torch.float64, requires_grad=True)
    g = torch.autograd.grad(f(xi), xi)[0]
    g_ref = torch.autograd.grad(f_ref(xi), xi)[0]
    assert torch.allclose(g, g_ref, rtol=1e-12, atol=1e-12)
    _, hv = torch.autograd.functional.hvp(f, torch.zeros(N, 12, dtype=torch.float64), v)
    _, hv_ref = torch.autograd.functional.hvp(f_ref, torch.zeros(N, 12, dtype=torch.float64), v)
    assert torch.allclose(hv, hv_ref, rtol=1e-10, atol=1e-10)
    # the plain double backward gives the same
    xi = torch.zeros(N, 12, dtype=torch.float64, requires_grad=True)
    g = torch.autograd.grad(f(xi), xi, create_graph=True)[0]
    hv2 = torch.autograd.grad((g * v).sum(), xi)[0]
    assert torch.allclose(hv2, hv_ref, rtol=1e-10, atol=1e-10)
    assert "hvp" in P.calls and "bwd" in P.calls
    if loss != "linear":
        assert "jvp" in P.calls  # the cotangent depends on the records


def test_contactfn_rejects_a_nonzero_perturbation():
    P = QuadPlan()
    xi = torch.zeros(N, 12, dtype=torch.float64)
    xi[1, 4] = 1e-3
    with pytest.raises(ValueError):
        api.ContactFn.apply(xi, P, None)
