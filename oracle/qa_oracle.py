"""ctypes/numpy wrapper around ``liboracle.so`` (``qa_oracle.c``).

TEST INFRASTRUCTURE ONLY (tests, smoke check, CPU baseline of the benchmark).

Every function takes FP64 numpy arrays in the paper's notation:
``cdd`` (N x N Maxwell dot-dot block), ``cgd`` (N x G gate-dot block),
``V`` (P x G gate voltages, one row per pixel), ``closed``/``nhat`` for the
closed-array constraint (Sec. 2, constraint iii), ``t`` the threshold of
Sec. 3.2.2 (1.0 = the default algorithm), ``kT`` the temperature of the
softargmin (Sec. 4.2) in the energy units of U.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "qa_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

INFO_QP = 1
INFO_AMBIGUOUS = 2
INFO_DOUBLED = 4
INFO_FAIL = 8


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (FP64, no contraction, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
             "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        _lib = C.CDLL(_LIB)
        d, i32, i64, u32 = C.POINTER(C.c_double), C.POINTER(C.c_int32), C.POINTER(C.c_int64), C.POINTER(C.c_uint32)
        sig = {
            "orc_inverse": (C.c_int, [C.c_int, d, d]),
            "orc_is_pd": (C.c_int, [C.c_int, d]),
            "orc_xu": (None, [C.c_int64, C.c_int, C.c_int, d, d, d]),
            "orc_energy": (C.c_double, [C.c_int, d, d, i32]),
            "orc_analytic_min": (None, [C.c_int, d, d, C.c_int, C.c_int, d]),
            "orc_qp_enum": (C.c_int, [C.c_int, d, d, C.c_int, C.c_int, d]),
            "orc_qp_open_chandrasekaran": (C.c_int, [C.c_int, d, d, d]),
            "orc_cont_min": (C.c_int, [C.c_int, d, d, C.c_int, C.c_int, d, i32]),
            "orc_candidates": (C.c_double, [C.c_int, d, C.c_int, C.c_int, C.c_double, i32, u32, i32]),
            "orc_method_gs": (C.c_int64, [C.c_int64, C.c_int, C.c_int, d, d, d, C.c_int, C.c_int,
                                          C.c_double, i32, d, d, i64, i32]),
            "orc_method_setup": (C.c_int64, [C.c_int64, C.c_int, C.c_int, d, d, d, C.c_int, C.c_int,
                                             C.c_double, d, i32, u32, i32, i32]),
            "orc_soft_fixed": (None, [C.c_int64, C.c_int, C.c_int, d, d, d, C.c_double, i32, u32, i32,
                                      d, d, d]),
            "orc_method_soft": (C.c_int64, [C.c_int64, C.c_int, C.c_int, d, d, d, C.c_int, C.c_int,
                                            C.c_double, C.c_double, d, d, d]),
            "orc_soft_grad": (None, [C.c_int64, C.c_int, C.c_int, d, d, d, C.c_double, i32, u32, i32,
                                     d, d, d, d]),
            "orc_exact_box": (C.c_int64, [C.c_int64, C.c_int, C.c_int, d, d, d, C.c_int, C.c_int,
                                          i32, d, d, i64]),
            "orc_exact_compositions": (C.c_int64, [C.c_int64, C.c_int, C.c_int, d, d, d, C.c_int,
                                                   i32, d, d]),
            "orc_exact_se": (C.c_int64, [C.c_int64, C.c_int, C.c_int, d, d, d, C.c_int, C.c_int,
                                         i32, d, d, i64]),
            "orc_exact_soft": (C.c_int64, [C.c_int64, C.c_int, C.c_int, d, d, d, C.c_int, C.c_int,
                                           C.c_double, d, i64]),
            "orc_set_threads": (None, [C.c_int]),
            "orc_max_threads": (C.c_int, []),
        }
        for name, (res, args) in sig.items():
            f = getattr(_lib, name)
            f.restype = res
            f.argtypes = args
    return _lib


def _d(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _i(a):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


def _l(a):
    return a.ctypes.data_as(C.POINTER(C.c_int64))


def _u(a):
    return a.ctypes.data_as(C.POINTER(C.c_uint32))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _prep(cdd, cgd, V):
    cdd, cgd, V = _f64(cdd), _f64(cgd), _f64(V)
    n, g = cgd.shape
    assert cdd.shape == (n, n) and 1 <= n <= 16
    V = V.reshape(-1, g)
    return cdd, cgd, np.ascontiguousarray(V), n, g, V.shape[0]


def set_threads(n: int) -> None:
    lib().orc_set_threads(int(n))


def max_threads() -> int:
    return int(lib().orc_max_threads())


def inverse(cdd):
    cdd = _f64(cdd)
    n = cdd.shape[0]
    A = np.empty((n, n))
    if lib().orc_inverse(n, _d(cdd), _d(A)):
        raise ValueError("singular matrix")
    return A


def is_pd(cdd) -> bool:
    cdd = _f64(cdd)
    return lib().orc_is_pd(cdd.shape[0], _d(cdd)) == 0


def xu(cgd, V):
    cgd = _f64(cgd)
    n, g = cgd.shape
    V = _f64(V).reshape(-1, g)
    out = np.empty((V.shape[0], n))
    lib().orc_xu(V.shape[0], n, g, _d(cgd), _d(V), _d(out))
    return out


def energy(A, x_u, q) -> float:
    A, x_u = _f64(A), _f64(x_u)
    q = np.ascontiguousarray(q, dtype=np.int32)
    return float(lib().orc_energy(A.shape[0], _d(A), _d(x_u), _i(q)))


def analytic_min(cdd, x_u, closed=False, nhat=0):
    cdd, x_u = _f64(cdd), _f64(x_u)
    x = np.empty(cdd.shape[0])
    lib().orc_analytic_min(cdd.shape[0], _d(cdd), _d(x_u), int(closed), int(nhat), _d(x))
    return x


def qp_enum(cdd, x_u, closed=False, nhat=0):
    cdd, x_u = _f64(cdd), _f64(x_u)
    x = np.empty(cdd.shape[0])
    r = lib().orc_qp_enum(cdd.shape[0], _d(cdd), _d(x_u), int(closed), int(nhat), _d(x))
    if r < 0:
        raise RuntimeError("no KKT point found")
    return x


def qp_open_chandrasekaran(cdd, x_u):
    cdd, x_u = _f64(cdd), _f64(x_u)
    x = np.empty(cdd.shape[0])
    r = lib().orc_qp_open_chandrasekaran(cdd.shape[0], _d(cdd), _d(x_u), _d(x))
    if r < 0:
        raise RuntimeError("Chandrasekaran iteration failed")
    return x, r


def cont_min(cdd, x_u, closed=False, nhat=0):
    """Constrained continuous minimum of Sec. 3.1: returns (x*, used_qp)."""
    cdd, x_u = _f64(cdd), _f64(x_u)
    x = np.empty(cdd.shape[0])
    path = np.zeros(1, np.int32)
    if lib().orc_cont_min(cdd.shape[0], _d(cdd), _d(x_u), int(closed), int(nhat), _d(x), _i(path)):
        raise RuntimeError("QP failed")
    return x, bool(path[0])


def candidates(x, closed=False, nhat=0, t=1.0):
    """(n0, freemask, k, t_used) describing the candidate set n0 + 1_s."""
    x = _f64(x)
    n = x.shape[0]
    n0 = np.empty(n, np.int32)
    fm = np.zeros(1, np.uint32)
    k = np.zeros(1, np.int32)
    tu = lib().orc_candidates(n, _d(x), int(closed), int(nhat), float(t), _i(n0), _u(fm), _i(k))
    return n0, int(fm[0]), int(k[0]), float(tu)


def candidate_list(n0, freemask, k):
    """Explicit list of candidate charge vectors (for tests)."""
    n = len(n0)
    out = []
    for s in range(1 << n):
        if s & ~freemask:
            continue
        if k >= 0 and bin(s).count("1") != k:
            continue
        out.append([n0[i] + ((s >> i) & 1) for i in range(n)])
    return np.array(out, dtype=np.int64).reshape(-1, n)


def method_gs(cdd, cgd, V, closed=False, nhat=0, t=1.0):
    """O-method at T = 0.  Returns dict(n, e1, e2, ncand, info)."""
    cdd, cgd, V, n, g, P = _prep(cdd, cgd, V)
    ns = np.empty((P, n), np.int32)
    e1, e2 = np.empty(P), np.empty(P)
    nc = np.empty(P, np.int64)
    info = np.empty(P, np.int32)
    lib().orc_method_gs(P, n, g, _d(cdd), _d(cgd), _d(V), int(closed), int(nhat), float(t),
                        _i(ns), _d(e1), _d(e2), _l(nc), _i(info))
    return dict(n=ns, e1=e1, e2=e2, ncand=nc, info=info)


def method_setup(cdd, cgd, V, closed=False, nhat=0, t=1.0):
    cdd, cgd, V, n, g, P = _prep(cdd, cgd, V)
    xs = np.empty((P, n))
    n0 = np.empty((P, n), np.int32)
    fm = np.empty(P, np.uint32)
    k = np.empty(P, np.int32)
    info = np.empty(P, np.int32)
    lib().orc_method_setup(P, n, g, _d(cdd), _d(cgd), _d(V), int(closed), int(nhat), float(t),
                           _d(xs), _i(n0), _u(fm), _i(k), _i(info))
    return dict(xstar=xs, n0=n0, freemask=fm, k=k, info=info)


def soft_fixed(cdd, cgd, V, kT, n0, freemask, k):
    cdd, cgd, V, n, g, P = _prep(cdd, cgd, V)
    n0 = np.ascontiguousarray(n0, np.int32)
    fm = np.ascontiguousarray(freemask, np.uint32)
    k = np.ascontiguousarray(k, np.int32)
    nbar = np.empty((P, n))
    emin, logZ = np.empty(P), np.empty(P)
    lib().orc_soft_fixed(P, n, g, _d(cdd), _d(cgd), _d(V), float(kT), _i(n0), _u(fm), _i(k),
                         _d(nbar), _d(emin), _d(logZ))
    return nbar, emin, logZ


def method_soft(cdd, cgd, V, closed=False, nhat=0, t=1.0, kT=0.01):
    cdd, cgd, V, n, g, P = _prep(cdd, cgd, V)
    nbar = np.empty((P, n))
    emin, logZ = np.empty(P), np.empty(P)
    lib().orc_method_soft(P, n, g, _d(cdd), _d(cgd), _d(V), int(closed), int(nhat), float(t),
                          float(kT), _d(nbar), _d(emin), _d(logZ))
    return nbar, emin, logZ


def soft_grad(cdd, cgd, V, kT, n0, freemask, k, Gbar):
    """Analytic FP64 adjoint of the fixed-set softargmin: (dCdd, dCgd, dV)."""
    cdd, cgd, V, n, g, P = _prep(cdd, cgd, V)
    n0 = np.ascontiguousarray(n0, np.int32)
    fm = np.ascontiguousarray(freemask, np.uint32)
    k = np.ascontiguousarray(k, np.int32)
    Gbar = _f64(Gbar).reshape(P, n)
    dC, dG, dV = np.empty((n, n)), np.empty((n, g)), np.empty((P, g))
    lib().orc_soft_grad(P, n, g, _d(cdd), _d(cgd), _d(V), float(kT), _i(n0), _u(fm), _i(k),
                        _d(Gbar), _d(dC), _d(dG), _d(dV))
    return dC, dG, dV


def exact_box(cdd, cgd, V, closed=False, nhat=0):
    cdd, cgd, V, n, g, P = _prep(cdd, cgd, V)
    ns = np.empty((P, n), np.int32)
    e1, e2 = np.empty(P), np.empty(P)
    size = np.empty(P, np.int64)
    lib().orc_exact_box(P, n, g, _d(cdd), _d(cgd), _d(V), int(closed), int(nhat), _i(ns),
                        _d(e1), _d(e2), _l(size))
    return dict(n=ns, e1=e1, e2=e2, boxsize=size)


def exact_compositions(cdd, cgd, V, nhat):
    cdd, cgd, V, n, g, P = _prep(cdd, cgd, V)
    ns = np.empty((P, n), np.int32)
    e1, e2 = np.empty(P), np.empty(P)
    lib().orc_exact_compositions(P, n, g, _d(cdd), _d(cgd), _d(V), int(nhat), _i(ns), _d(e1), _d(e2))
    return dict(n=ns, e1=e1, e2=e2)


def exact_se(cdd, cgd, V, closed=False, nhat=0):
    cdd, cgd, V, n, g, P = _prep(cdd, cgd, V)
    ns = np.empty((P, n), np.int32)
    e1, e2 = np.empty(P), np.empty(P)
    nodes = np.empty(P, np.int64)
    lib().orc_exact_se(P, n, g, _d(cdd), _d(cgd), _d(V), int(closed), int(nhat), _i(ns),
                       _d(e1), _d(e2), _l(nodes))
    return dict(n=ns, e1=e1, e2=e2, nodes=nodes)


def exact_soft(cdd, cgd, V, closed=False, nhat=0, kT=0.01):
    cdd, cgd, V, n, g, P = _prep(cdd, cgd, V)
    nbar = np.empty((P, n))
    cnt = np.empty(P, np.int64)
    lib().orc_exact_soft(P, n, g, _d(cdd), _d(cgd), _d(V), int(closed), int(nhat), float(kT),
                         _d(nbar), _l(cnt))
    return nbar, cnt


# ---------------------------------------------------------------------------
# Analytic utilities (Sec. 5.3), numpy FP64 with library primitives
# ---------------------------------------------------------------------------

def optimal_gate_voltages(cdd, cgd, q):
    """App. H: minimise F over the gate voltages for fixed charges q.  With
    the Cholesky factor L of C_dd (C_dd = L L^T), R = L^-1 satisfies
    R^T R = C_dd^-1 and F = 1/2 |R (q - C_gd V)|^2, a linear least-squares
    problem solved by the pseudo-inverse: V = (R C_gd)^+ R q."""
    cdd = np.asarray(cdd, np.float64)
    cgd = np.asarray(cgd, np.float64)
    L = np.linalg.cholesky(cdd)
    R = np.linalg.inv(L)
    return np.linalg.pinv(R @ cgd) @ (R @ np.asarray(q, np.float64))


def virtual_gate_matrix(cdd, cgd):
    """App. I: the dot potentials move by C_dd^-1 C_gd dV (Eq. for the
    potential); alpha = (C_dd^-1 C_gd)^+ (G x N), column i the gate change that
    moves dot i's potential by one unit."""
    cdd = np.asarray(cdd, np.float64)
    cgd = np.asarray(cgd, np.float64)
    return np.linalg.pinv(np.linalg.solve(cdd, cgd))


# ---------------------------------------------------------------------------
# Charge sensors (Sec. 5.1), numpy FP64
# ---------------------------------------------------------------------------

def sensor_charges_brute(cdd, cgd, V, n_array, n_sensor, span=6):
    """The sensor dots' charges minimising U over every integer vector in a
    box of +-span around the continuous minimum (clipped at 0), with the
    array dots' charges held fixed (Sec. 5.1).  Brute force: every candidate
    is scored by the full quadratic form.  Returns (P x S int64)."""
    cdd = np.asarray(cdd, np.float64)
    cgd = np.asarray(cgd, np.float64)
    V = np.atleast_2d(np.asarray(V, np.float64))
    na = np.atleast_2d(np.asarray(n_array, np.float64))
    N = cdd.shape[0]
    Na, S = N - n_sensor, n_sensor
    A = np.linalg.inv(cdd)
    P = V.shape[0]
    out = np.zeros((P, S), np.int64)
    grids = np.array(np.meshgrid(*[np.arange(-span, span + 1)] * S, indexing="ij")).reshape(S, -1).T
    for p in range(P):
        xu = cgd @ V[p]
        za = na[p] - xu[:Na]
        # continuous minimum over the sensor charges (unconstrained)
        xs = xu[Na:] - np.linalg.solve(A[Na:, Na:], A[Na:, :Na] @ za)
        base = np.floor(np.maximum(xs, 0.0)).astype(np.int64)
        best, bn = np.inf, None
        for d in grids:
            ns = base + d
            if (ns < 0).any():
                continue
            z = np.concatenate([za, ns - xu[Na:]])
            e = 0.5 * z @ A @ z
            # ties to the lexicographically smallest sensor charge vector
            if e < best or (e == best and tuple(ns) < tuple(bn)):
                best, bn = e, ns
        out[p] = bn
    return out


def sensor_signal(cdd, cgd, V, n_array, n_sensor, gamma, shape="lorentzian", n_sens=None):
    """Sensor response (Sec. 5.1): with the array charges fixed and the
    sensor charges at their minimum, the sensor potentials follow Eq. for the
    potential, v = C_dd^-1 (n - C_gd V); adding a carrier to sensor s costs
    v_s + A_ss / 2 and removing one -v_s + A_ss / 2 (zero at the two nearest
    Coulomb-peak conditions), and the response is the peak profile of each
    (Lorentzian 1 / (1 + (x / gamma)^2) or Gaussian exp(-x^2 / (2 gamma^2)))
    summed, the removal term only when the sensor holds a carrier.
    Returns (P x S)."""
    cdd = np.asarray(cdd, np.float64)
    cgd = np.asarray(cgd, np.float64)
    V = np.atleast_2d(np.asarray(V, np.float64))
    na = np.atleast_2d(np.asarray(n_array, np.float64))
    N = cdd.shape[0]
    Na = N - n_sensor
    A = np.linalg.inv(cdd)
    if n_sens is None:
        n_sens = sensor_charges_brute(cdd, cgd, V, na, n_sensor)
    xu = V @ cgd.T
    n = np.concatenate([na, n_sens.astype(np.float64)], axis=1)
    v = (n - xu) @ A.T
    diag = np.diag(A)[Na:]
    vs = v[:, Na:]
    prof = (lambda x: 1.0 / (1.0 + (x / gamma) ** 2)) if shape == "lorentzian" else \
        (lambda x: np.exp(-x * x / (2.0 * gamma * gamma)))
    up = prof(vs + 0.5 * diag)
    down = np.where(n_sens > 0, prof(-vs + 0.5 * diag), 0.0)
    return up + down, v


def pink_noise(draws_by_octave, P):
    """Voss-McCartney pink (1/f) noise: K octave sources, source k holding a
    standard-normal draw for every 2^k consecutive samples; sample t is the
    sum of the sources' current draws over sqrt(K) (unit variance).
    draws_by_octave[k] has ceil(P / 2^k) entries."""
    K = len(draws_by_octave)
    t = np.arange(P)
    return sum(np.asarray(draws_by_octave[k])[t >> k] for k in range(K)) / np.sqrt(K)


def telegraph_noise(u, rate):
    """Random telegraph (sensor jump) noise: the state starts at 0 and flips
    at sample t when the uniform draw u_t < rate; the state at t counts the
    flips up to and including t, mod 2."""
    flips = (np.asarray(u) < rate).astype(np.int64)
    return np.cumsum(flips) % 2
