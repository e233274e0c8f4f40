"""Adjoint workload on the GPU: torch autograd around the SoftCharge function
(GPU forward and hand-written backward), sensor signal and MSE loss as plain
torch ops, against the oracle's analytic chain (pinned to central differences
in test_adjoint_oracle.py)."""
import sys

import numpy as np
import pytest
import torch

from adjoint_case import oracle_loss_and_grad, oracle_signal
from paper_2404_04994_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def qa():
    from paper_2404_04994_amd import qarray
    assert torch.cuda.is_available()
    qarray.load()
    return qarray


def torch_loss(qa, case, C, G, V, target):
    nbar = qa.soft_charge_autograd(C[:8, :8], G[:8, :], V, case.kT)
    w = torch.linalg.inv(C)[8, :8]
    S = nbar @ w.to(nbar.device)
    return ((S - target) ** 2).mean()


@pytest.mark.parametrize("npix", [24, 100])
def test_adjoint_workload(qa, oracle, npix):
    case = W.adjoint_case(400, npix=npix)
    L_ref, dC_ref, dG_ref, dV_ref, _ = oracle_loss_and_grad(oracle, case)
    target = torch.as_tensor(oracle_signal(oracle, case.cdd_target, case.cgd_target, case.V,
                                           case.kT), device="cuda")
    C = torch.tensor(case.cdd, dtype=torch.float64, requires_grad=True)   # host, FP64
    G = torch.tensor(case.cgd, dtype=torch.float64, requires_grad=True)
    V = torch.tensor(case.V, dtype=torch.float64, device="cuda", requires_grad=True)
    L = torch_loss(qa, case, C, G, V, target)
    L.backward()
    print("L gpu %.12g oracle %.12g" % (L.item(), L_ref), flush=True)
    assert abs(L.item() - L_ref) <= 1e-9 * max(1.0, abs(L_ref))
    for got, ref, name in ((C.grad.numpy(), dC_ref, "C_dd"), (G.grad.numpy(), dG_ref, "C_gd"),
                           (V.grad.cpu().numpy(), dV_ref, "V")):
        rel = np.linalg.norm(got - ref) / max(np.linalg.norm(ref), 1e-300)
        print("grad %s rel err %.3e" % (name, rel), flush=True)
        assert rel <= 1e-8
    sys.stdout.flush()


def test_backward_after_other_diagram_and_repeated(qa):
    """The backward reuses the forward's prologue when the record still holds
    it and relies on its accumulators having been left at zero: repeated
    passes, and a pass after another diagram's forward on the same stream,
    give the same gradients (to atomic-order rounding)."""
    case = W.adjoint_case(400, npix=20)
    other = W.adjoint_case(401, npix=20)
    Vo = torch.tensor(other.V, dtype=torch.float64, device="cuda")

    def grads(interleave):
        C = torch.tensor(case.cdd[:8, :8], dtype=torch.float64, requires_grad=True)
        G = torch.tensor(case.cgd[:8, :], dtype=torch.float64, requires_grad=True)
        V = torch.tensor(case.V, dtype=torch.float64, device="cuda", requires_grad=True)
        nbar = qa.soft_charge_autograd(C, G, V, case.kT)
        if interleave:
            qa.soft_charge(other.cdd[:8, :8], other.cgd[:8, :], Vo, other.kT)
        w = torch.linspace(0.5, 1.5, 8, dtype=torch.float64, device="cuda")
        (nbar @ w).pow(2).sum().backward()
        torch.cuda.synchronize()
        return C.grad.numpy().copy(), G.grad.numpy().copy(), V.grad.cpu().numpy().copy()

    ref = grads(False)
    for interleave in (False, True, False, True):
        got = grads(interleave)
        for a, b in zip(got, ref):
            rel = np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)
            assert rel <= 1e-12, (interleave, rel)
