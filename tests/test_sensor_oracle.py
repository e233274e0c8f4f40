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


def test_gaussian_profile_height_and_area(oracle):
    """Gaussian sensor peak (Sec. 5.1) pinned by the closed forms of
    exp(-x^2 / (2 gamma^2)): height 1 at the Coulomb-peak condition, e^{-1/2}
    where the addition energy is gamma, and area sqrt(2 pi) gamma in the
    energy coordinate.  An isolated sensor's addition energy moves by
    c_g / c_s per volt, so one peak swept in V has area sqrt(2 pi) gamma c_s / c_g.
    A width convention exp(-x^2 / gamma^2) fails the second and third checks."""
    cg, cs = 0.8, 2.0
    cdd, cgd = isolated_sensor(cg, cs)
    gamma = 0.02
    k = 2
    vk = (k + 0.5) / cg
    # just below the degeneracy the sensor holds k, so only the addition term
    # is near its peak; dV = gamma c_s / c_g puts the addition energy at gamma
    dv = gamma * cs / cg
    V = np.array([[0.0, vk - 1e-12], [0.0, vk - dv], [0.0, vk - 2.0 * dv]])
    ns = oracle.sensor_charges_brute(cdd, cgd, V, np.zeros((3, 1)), 1)[:, 0]
    assert list(ns) == [k, k, k]
    r, v = oracle.sensor_signal(cdd, cgd, V, np.zeros((3, 1)), 1, gamma, shape="gaussian")
    np.testing.assert_allclose(v[:, 1] + 0.5 / cs, [0.0, gamma, 2.0 * gamma], atol=1e-10)
    np.testing.assert_allclose(r[:, 0], [1.0, np.exp(-0.5), np.exp(-2.0)], rtol=1e-9)
    # area of the peak over one period centred on it (the other terms sit a
    # charging energy 1/c_s = 25 gamma away: e^{-312}, nothing)
    x = np.linspace(vk - 0.5 / cg, vk + 0.5 / cg, 40001)
    Vs = np.stack([np.zeros_like(x), x], axis=1)
    rs, _ = oracle.sensor_signal(cdd, cgd, Vs, np.zeros((len(x), 1)), 1, gamma, shape="gaussian")
    area = np.trapezoid(rs[:, 0], x)
    np.testing.assert_allclose(area, np.sqrt(2.0 * np.pi) * gamma * cs / cg, rtol=1e-6)


def test_lorentzian_half_width(oracle):
    """Lorentzian 1 / (1 + (x / gamma)^2): one half where the addition energy is gamma."""
    cg, cs = 0.8, 2.0
    cdd, cgd = isolated_sensor(cg, cs)
    gamma = 0.01
    vk = 1.5 / cg
    V = np.array([[0.0, vk - gamma * cs / cg]])
    r, _ = oracle.sensor_signal(cdd, cgd, V, np.zeros((1, 1)), 1, gamma)
    far = 1.0 / (1.0 + ((1.0 / cs - gamma) / gamma) ** 2)  # removal term of the held carrier
    np.testing.assert_allclose(r[0, 0], 0.5 + far, rtol=1e-9)


def _sensor_enumeration(cdd, cgd, V, n_array, S, nmax):
    """Every sensor charge vector in {0..nmax}^S scored by the full quadratic
    form; lexicographically smallest on exact ties.  Independent of the
    oracle's search (no continuous minimum, no box around it)."""
    A = np.linalg.inv(cdd)
    N = cdd.shape[0]
    Na = N - S
    grid = np.array(np.meshgrid(*[np.arange(nmax + 1)] * S, indexing="ij")).reshape(S, -1).T
    out = np.zeros((V.shape[0], S), np.int64)
    for p in range(V.shape[0]):
        xu = cgd @ V[p]
        z = np.concatenate([np.tile(n_array[p] - xu[:Na], (len(grid), 1)), grid - xu[Na:]], axis=1)
        e = 0.5 * np.einsum("ki,ij,kj->k", z, A, z)
        out[p] = grid[int(np.argmin(e))]      # argmin takes the first (lexicographic) minimum
        # the minimum is interior to the enumerated box, so the box is wide enough
        assert (out[p] < nmax).all()
    return out


@pytest.mark.parametrize("S,nmax", [(2, 24), (3, 12)])
def test_multi_sensor_search_matches_enumeration(oracle, S, nmax):
    """Two and three sensor dots coupled to each other and to the array
    (Sec. 5.1): the oracle's sensor charges equal an exhaustive enumeration of
    a wide box of sensor charges starting at zero."""
    rng = np.random.default_rng(40 + S)
    Na = 3
    N = Na + S
    cdd = np.diag(rng.uniform(1.0, 1.4, N))
    for i in range(N):
        for j in range(i + 1, N):
            # strong sensor-sensor coupling, so the sensors' minimum is not
            # the per-sensor rounding
            lo, hi = (0.3, 0.5) if (i >= Na and j >= Na) else (0.02, 0.15)
            cdd[i, j] = cdd[j, i] = -rng.uniform(lo, hi)
    assert np.all(np.linalg.eigvalsh(cdd) > 0)
    cgd = np.diag(rng.uniform(0.5, 1.0, N)) + rng.uniform(0.0, 0.1, (N, N))
    P = 60 if S == 2 else 25
    V = rng.uniform(-1.0, 8.0, (P, N))
    na = rng.integers(0, 4, (P, Na))
    got = oracle.sensor_charges_brute(cdd, cgd, V, na, S)
    ref = _sensor_enumeration(cdd, cgd, V, na, S, nmax)
    assert (got == ref).all(), np.where((got != ref).any(1))[0]
    # the sweep reaches empty sensors (the n >= 0 bound active) and sensors
    # holding several carriers
    assert (ref == 0).any() and (ref >= 3).any()
    # and pixels where rounding the sensors' joint continuous minimum is not
    # the minimum, so a search that stopped there would fail
    A = np.linalg.inv(cdd)
    xu = V @ cgd.T
    xs = xu[:, Na:] - np.linalg.solve(A[Na:, Na:], A[Na:, :Na] @ (na - xu[:, :Na]).T).T
    assert (np.maximum(0, np.round(xs)) != ref).any(1).sum() >= 3
