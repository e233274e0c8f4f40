"""The lower bound behind the bound-ordered scorer, checked with numpy on
small random capacitance matrices (CPU, no library call).

For U(n0 + b) - U(n0) = b^T g + 1/2 b^T A b with A = C_dd^{-1} and
g = A y (y = n0 - x_u), split b into a low part (dots 0..7) and a high part
(dots 8..N-1).  Minimising over a real-valued low part gives
    L(b_hi) = K + b_hi^T s + 1/2 b_hi^T S b_hi,
    S = (C_dd,HH)^{-1},  s = S y_hi,  K = 1/2 y_hi^T s - 1/2 y^T g,
and with the low part's sum fixed at m (closed arrays)
    L_m(b_hi) = L(b_hi) + (m - mu - w^T b_hi)^2 / (2 gamma),
    mu = -1^T A_LL^{-1} g_lo,  w = S C_HL 1,  gamma = 1^T A_LL^{-1} 1.
The tests check the block-inverse identities these use and that each bound
lies below every integer state it covers (brute force over the low part).
"""
import itertools

import numpy as np
import pytest

from paper_2404_04994_amd import workloads as W


def _energies(A, g, bhi, nlo):
    """E(b_lo, b_hi) for every b_lo in {0,1}^nlo (rows) -- brute force."""
    out = []
    for blo in itertools.product((0.0, 1.0), repeat=nlo):
        b = np.concatenate([np.array(blo), bhi])
        out.append((b @ g + 0.5 * b @ A @ b, sum(blo)))
    return out


@pytest.mark.parametrize("n,seed", [(13, 1), (14, 2), (16, 3)])
def test_block_inverse_identities(n, seed):
    cdd, _ = W.random_maxwell(n, seed)
    A = np.linalg.inv(cdd)
    L, H = slice(0, 8), slice(8, n)
    S = np.linalg.inv(cdd[H, H])
    # Schur complement of A_LL in A is the inverse of C_dd's high block
    assert np.allclose(A[H, H] - A[H, L] @ np.linalg.solve(A[L, L], A[L, H]), S, atol=1e-12)
    # A_LL^{-1} is the Schur complement of C_HH in C_dd
    assert np.allclose(np.linalg.inv(A[L, L]), cdd[L, L] - cdd[L, H] @ S @ cdd[H, L], atol=1e-12)
    # the low minimiser's sum moves with b_hi by w = S C_HL 1
    w = S @ cdd[H, L] @ np.ones(8)
    assert np.allclose(-np.ones(8) @ np.linalg.solve(A[L, L], A[L, H]), w, atol=1e-12)


@pytest.mark.parametrize("seed", [11, 12])
def test_bound_below_every_state(seed):
    """Both bounds against brute force over the low part, on a 13-dot array
    (5 high dots, every high part)."""
    n = 13
    rng = np.random.default_rng(seed)
    cdd, cgd = W.random_maxwell(n, seed)
    A = np.linalg.inv(cdd)
    L, H = slice(0, 8), slice(8, n)
    S = np.linalg.inv(cdd[H, H])
    Q = np.linalg.inv(A[L, L])
    w = S @ cdd[H, L] @ np.ones(8)
    gamma = np.ones(8) @ Q @ np.ones(8)
    x_u = cgd @ rng.uniform(-1, 3, n)
    n0 = np.floor(x_u)
    y = n0 - x_u
    g = A @ y
    s = S @ y[H]
    K = 0.5 * y[H] @ s - 0.5 * y @ g
    mu = -np.ones(8) @ Q @ g[L]
    gap_min = np.inf
    for bits in itertools.product((0.0, 1.0), repeat=n - 8):
        bhi = np.array(bits)
        Lb = K + bhi @ s + 0.5 * bhi @ S @ bhi
        es = _energies(A, g, bhi, 8)
        emin = min(e for e, _ in es)
        assert Lb <= emin + 1e-12
        gap_min = min(gap_min, emin - Lb)
        for m in range(9):
            Lm = Lb + (m - mu - w @ bhi) ** 2 / (2.0 * gamma)
            em = min(e for e, c in es if c == m)
            assert Lm <= em + 1e-12
            assert Lm >= Lb - 1e-15
    assert gap_min >= -1e-12


def test_bound_is_exact_for_a_real_low_part():
    """The bound is the minimum over a real low part: at b_lo = -A_LL^{-1} g'
    the energy equals L (a wrong sign or block would break this)."""
    n = 14
    cdd, cgd = W.random_maxwell(n, 21)
    A = np.linalg.inv(cdd)
    L, H = slice(0, 8), slice(8, n)
    S = np.linalg.inv(cdd[H, H])
    rng = np.random.default_rng(5)
    y = rng.uniform(-1, 0, n)
    g = A @ y
    s = S @ y[H]
    K = 0.5 * y[H] @ s - 0.5 * y @ g
    bhi = rng.integers(0, 2, n - 8).astype(float)
    gp = g[L] + A[L, H] @ bhi
    blo = -np.linalg.solve(A[L, L], gp)
    b = np.concatenate([blo, bhi])
    assert abs((b @ g + 0.5 * b @ A @ b) - (K + bhi @ s + 0.5 * bhi @ S @ bhi)) < 1e-12


@pytest.mark.parametrize("n,seed", [(13, 21), (16, 22)])
def test_single_flip_delta(n, seed):
    """The setup's guess takes its best single flip: flipping dot i of b
    changes E(b) = b^T g + 1/2 b^T A b by (1 - 2 b_i) (g + A b)_i + A_ii / 2
    (checked against the energies directly, for random states)."""
    rng = np.random.default_rng(seed)
    cdd, cgd = W.random_maxwell(n, seed)
    A = np.linalg.inv(cdd)
    x_u = cgd @ rng.uniform(-1, 3, cgd.shape[1])
    y = np.floor(x_u) - x_u
    g = A @ y

    def E(b):
        return b @ g + 0.5 * b @ A @ b

    for _ in range(20):
        b = rng.integers(0, 2, n).astype(float)
        gd = g + A @ b
        for i in range(n):
            f = b.copy()
            f[i] = 1.0 - f[i]
            de = (1.0 - 2.0 * b[i]) * gd[i] + 0.5 * A[i, i]
            assert abs((E(f) - E(b)) - de) <= 1e-12 * (1.0 + abs(E(b)))
