"""The adjoint workload: a 2x4 open array with one sensor dot (index 8).

Array charges are the softargmin over the 8 array dots, computed with the
8x8 block of C_dd and the 8x9 block of C_gd -- the sensor dot is left out of
the array's charge computation but the sensor gate's cross-talk is kept
(Sec. 4.1).  The sensor signal is the linear response of the sensor
potential (Eq. for the potential): S_p = sum_i (C_dd^-1)[8, i] <n_i>_p with
the 9x9 inverse.  The loss is L = mean_p (S_p - T_p)^2 against a target
diagram T made with perturbed capacitances.

Everything here is FP64 numpy on top of the oracle (reference side of the
tests).
"""
import numpy as np


def oracle_loss_and_grad(O, case, V=None):
    """L and (dL/dC_dd 9x9, dL/dC_gd 9x9, dL/dV) by the chain rule over the
    oracle's analytic softargmin adjoint (candidate sets fixed)."""
    V = case.V if V is None else V
    C, G, kT = case.cdd, case.cgd, case.kT
    target = oracle_signal(O, case.cdd_target, case.cgd_target, V, kT)
    st = O.method_setup(C[:8, :8], G[:8, :], V)
    nbar, _, _ = O.soft_fixed(C[:8, :8], G[:8, :], V, kT, st["n0"], st["freemask"], st["k"])
    Ci = np.linalg.inv(C)
    w = Ci[8, :8]
    S = nbar @ w
    P = V.shape[0]
    L = float(np.mean((S - target) ** 2))
    dS = 2.0 * (S - target) / P
    Gbar = dS[:, None] * w[None, :]
    dC8, dG8, dV = O.soft_grad(C[:8, :8], G[:8, :], V, kT, st["n0"], st["freemask"], st["k"], Gbar)
    dCi = np.zeros((9, 9))
    dCi[8, :8] = nbar.T @ dS
    dC = -Ci.T @ dCi @ Ci.T
    dC[:8, :8] += dC8
    dG = np.zeros((9, 9))
    dG[:8, :] = dG8
    return L, dC, dG, dV, (st["n0"], st["freemask"], st["k"])


def oracle_signal(O, C, G, V, kT):
    nbar, _, _ = O.method_soft(C[:8, :8], G[:8, :], V, kT=kT)
    return nbar @ np.linalg.inv(C)[8, :8]


def oracle_loss_fixed(O, case, C, G, V, sets, target):
    n0, fm, k = sets
    nbar, _, _ = O.soft_fixed(C[:8, :8], G[:8, :], V, case.kT, n0, fm, k)
    S = nbar @ np.linalg.inv(C)[8, :8]
    return float(np.mean((S - target) ** 2))
