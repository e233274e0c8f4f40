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
