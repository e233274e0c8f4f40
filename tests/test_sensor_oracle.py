"""Charge-sensor oracle (Sec. 5.1) pinned by what the model fixes: a
single sensor's charge is the 1-D convex minimum, its Coulomb-peak
conditions sit where two sensor charges are degenerate (V = (k + 1/2)/c_g
for an isolated sensor, the analogue of the single-dot transitions), the
potential moves by column i of C_dd^{-1} when array dot i gains a carrier,
and the noise constructions reduce to their definitions on hand-made draws."""
import numpy as np
import pytest


def isolated_sensor(cg=0.8, cs=2.0):
    # one array dot (uncoupled) and one sensor dot, one gate each
    cdd = np.array([[1.0, 0.0], [0.0, cs]])
    cgd = np.array([[1.0, 0.0], [0.0, cg]])
    return cdd, cgd


def test_sensor_charge_is_rounded_continuous_minimum(oracle):
    rng = np.random.default_rng(3)
    cdd = np.array([[1.2, -0.2, -0.05], [-0.2, 1.3, -0.1], [-0.05, -0.1, 1.5]])
    cgd = rng.uniform(0.1, 1.0, (3, 3))
    V = rng.uniform(-1, 5, (400, 3))
    na = rng.integers(0, 4, (400, 2))
    ns = oracle.sensor_charges_brute(cdd, cgd, V, na, 1)[:, 0]
    A = np.linalg.inv(cdd)
    xu = V @ cgd.T
    xs = xu[:, 2] - (A[2, :2] @ (na - xu[:, :2]).T) / A[2, 2]
    # 1-D convex quadratic in the sensor charge: nearest integer, at least 0
    assert (ns == np.maximum(0, np.round(xs)).astype(int)).all()


def test_isolated_sensor_peaks(oracle):
    cg, cs = 0.8, 2.0
    cdd, cgd = isolated_sensor(cg, cs)
    gamma = 0.02
    for k in range(4):
        vk = (k + 0.5) / cg
        V = np.array([[0.0, vk - 1e-6], [0.0, vk + 1e-6]])
        ns = oracle.sensor_charges_brute(cdd, cgd, V, np.zeros((2, 1)), 1)[:, 0]
        assert list(ns) == [k, k + 1]
        r, _ = oracle.sensor_signal(cdd, cgd, V, np.zeros((2, 1)), 1, gamma)
        # at the degeneracy one of the two terms is at its maximum 1 (adding a
        # carrier on the left, removing one on the right); the other sits a
        # charging energy A_ss = 1/c_s away, and an empty sensor has no
        # removal term
        far = 1.0 / (1.0 + (1.0 / cs / gamma) ** 2)
        np.testing.assert_allclose(r[:, 0], [1.0 + (far if k > 0 else 0.0), 1.0 + far], rtol=1e-4)
    # away from the peaks the response is small and periodic in V with 1/c_g
    V = np.stack([np.zeros(50), np.linspace(1.0, 1.0 + 1.0 / cg, 50)], axis=1)
    r1, _ = oracle.sensor_signal(cdd, cgd, V, np.zeros((50, 1)), 1, gamma)
    V2 = V.copy()
    V2[:, 1] += 1.0 / cg
    r2, _ = oracle.sensor_signal(cdd, cgd, V2, np.zeros((50, 1)), 1, gamma)
    np.testing.assert_allclose(r1, r2, rtol=1e-9, atol=1e-12)


def test_potential_moves_by_inverse_column(oracle):
    rng = np.random.default_rng(5)
    cdd = np.array([[1.2, -0.2, -0.02], [-0.2, 1.3, -0.03], [-0.02, -0.03, 3.0]])
    cgd = np.diag([0.7, 0.8, 0.9])
    V = rng.uniform(0, 3, (50, 3))
    na = rng.integers(0, 3, (50, 2))
    ns = oracle.sensor_charges_brute(cdd, cgd, V, na, 1)
    _, v0 = oracle.sensor_signal(cdd, cgd, V, na, 1, 0.05, n_sens=ns)
    na1 = na.copy()
    na1[:, 1] += 1
    _, v1 = oracle.sensor_signal(cdd, cgd, V, na1, 1, 0.05, n_sens=ns)
    np.testing.assert_allclose(v1 - v0, np.tile(np.linalg.inv(cdd)[:, 1], (50, 1)), atol=1e-12)


def test_pink_noise_constructions(oracle):
    P, K = 37, 4
    ones = [np.ones((P + (1 << k) - 1) >> k) for k in range(K)]
    np.testing.assert_allclose(oracle.pink_noise(ones, P), np.full(P, K / np.sqrt(K)))
    # a single nonzero draw of octave 2 covers four consecutive samples
    d = [np.zeros((P + (1 << k) - 1) >> k) for k in range(K)]
    d[2][3] = 1.0
    out = oracle.pink_noise(d, P)
    assert list(np.nonzero(out)[0]) == [12, 13, 14, 15]
    assert np.allclose(out[12:16], 1.0 / np.sqrt(K))


def test_telegraph_noise(oracle):
    u = np.array([0.9, 0.1, 0.5, 0.05, 0.9, 0.01, 0.02])
    assert list(oracle.telegraph_noise(u, 0.2)) == [0, 1, 1, 0, 0, 1, 0]
