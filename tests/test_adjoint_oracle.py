"""The oracle's gradient of the adjoint workload (sensor signal + MSE, 9x9
C_dd and C_gd, voltages) against FP64 central differences, h = 1e-6."""
import numpy as np

from adjoint_case import oracle_loss_and_grad, oracle_loss_fixed, oracle_signal
from paper_2404_04994_amd import workloads as W


def test_adjoint_chain_matches_central_differences(oracle):
    case = W.adjoint_case(400, npix=12)
    L, dC, dG, dV, sets = oracle_loss_and_grad(oracle, case)
    target = oracle_signal(oracle, case.cdd_target, case.cgd_target, case.V, case.kT)
    h = 1e-6
    fdC = np.zeros((9, 9))
    fdG = np.zeros((9, 9))
    for i in range(9):
        for j in range(9):
            e = np.zeros((9, 9)); e[i, j] = h
            fdC[i, j] = (oracle_loss_fixed(oracle, case, case.cdd + e, case.cgd, case.V, sets, target)
                         - oracle_loss_fixed(oracle, case, case.cdd - e, case.cgd, case.V, sets,
                                             target)) / (2 * h)
            fdG[i, j] = (oracle_loss_fixed(oracle, case, case.cdd, case.cgd + e, case.V, sets, target)
                         - oracle_loss_fixed(oracle, case, case.cdd, case.cgd - e, case.V, sets,
                                             target)) / (2 * h)
    # voltages: one +-h evaluation per gate over all pixels (pixels independent)
    P = case.V.shape[0]
    fdV = np.zeros_like(case.V)
    for j in range(9):
        e = np.zeros_like(case.V); e[:, j] = h
        n0, fm, k = sets
        Ci = np.linalg.inv(case.cdd)[8, :8]
        nbp, _, _ = oracle.soft_fixed(case.cdd[:8, :8], case.cgd[:8, :], case.V + e, case.kT, n0, fm, k)
        nbm, _, _ = oracle.soft_fixed(case.cdd[:8, :8], case.cgd[:8, :], case.V - e, case.kT, n0, fm, k)
        fdV[:, j] = (((nbp @ Ci) - target) ** 2 - ((nbm @ Ci) - target) ** 2) / P / (2 * h)
    for a, b in ((dC, fdC), (dG, fdG), (dV, fdV)):
        assert np.linalg.norm(a - b) <= 1e-6 * max(1e-3, np.linalg.norm(b))
    assert np.abs(dG[8]).max() == 0.0  # the sensor row of C_gd does not enter
