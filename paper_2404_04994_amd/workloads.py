"""Seeded synthetic inputs for the constant-capacitance ground-state path.

This module only draws capacitance matrices and gate-voltage sweeps; it holds
none of the method's arithmetic (no inverse capacitance, no energies, no
continuous minimum).  Both the HIP path and the FP64 oracle are fed from it.

Conventions (paper Sec. 2):
* ``cdd`` is the Maxwell dot-dot block: diagonal = total capacitance of the
  dot, off-diagonal = minus the dot-dot coupling.  Draws that are not positive
  definite are rejected (App. B gives the physical condition).
* ``cgd`` is the N x G gate-dot block with positive couplings, as in the
  worked example of Sec. 5 (so that the open continuous minimum C_gd V has
  the sign of the applied voltage).
* ``V`` is P x G (FP64), one row per pixel.  For a 2-D sweep of gates
  (i0, i1) over arrays (a, b), pixel ``p = j * len(a) + i`` holds
  ``V[p, i0] = a[i]`` and ``V[p, i1] = b[j]`` (row index = second gate), the
  layout of a ``meshgrid`` raster.

The paper benchmarks on random capacitance matrices and random gate voltages
(Sec. 7); it uses no public dataset.  The structured arrays below (double dot,
linear chain, 4x4 grid, ragged batch, 2x4 array with a sensor dot) stand in
for those workloads with the shapes and value ranges stated next to each.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Diagram:
    """One stability diagram: capacitances, voltages and the solve mode."""

    cdd: np.ndarray
    cgd: np.ndarray
    V: np.ndarray
    closed: bool = False
    nhat: int = 0
    kT: float = 0.0
    t: float = 1.0
    shape: tuple = ()
    meta: dict = field(default_factory=dict)
    # the affine sweep that V rasters, when it is one: v0, e1, e2 (G each),
    # a0, a1, nx, b0, b1, ny with V = sweep_voltages(sweep) (see there)
    sweep: dict | None = None

    @property
    def n_dot(self) -> int:
        return self.cdd.shape[0]

    @property
    def n_gate(self) -> int:
        return self.cgd.shape[1]

    @property
    def P(self) -> int:
        return self.V.shape[0]


def _is_pd(m: np.ndarray) -> bool:
    try:
        np.linalg.cholesky(m)
        return True
    except np.linalg.LinAlgError:
        return False


def sweep2d(n_gate: int, gates, a, b, base=None) -> np.ndarray:
    """Raster of two gates over ``a`` x ``b``; other gates at ``base``."""
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    V = np.zeros((len(b) * len(a), n_gate))
    if base is not None:
        V[:] = np.asarray(base, np.float64)[None, :]
    ii, jj = np.meshgrid(np.arange(len(a)), np.arange(len(b)))
    V[:, gates[0]] = a[ii.ravel()]
    V[:, gates[1]] = b[jj.ravel()]
    return V


def sweep_voltages(sw: dict) -> np.ndarray:
    """The P x G voltages of an affine two-coordinate sweep: pixel
    p = j * nx + i holds (v0 + a_i e1) + b_j e2 with a = linspace(a0, a1, nx)
    and b = linspace(b0, b1, ny), in numpy's FP64 arithmetic (each operation
    rounded on its own)."""
    a = np.linspace(sw["a0"], sw["a1"], sw["nx"])
    b = np.linspace(sw["b0"], sw["b1"], sw["ny"])
    aa, bb = np.meshgrid(a, b)
    v0, e1, e2 = (np.asarray(sw[k], np.float64) for k in ("v0", "e1", "e2"))
    return v0[None, :] + aa.ravel()[:, None] * e1[None, :] + bb.ravel()[:, None] * e2[None, :]


def gate_sweep(n_gate: int, gates, lo: float, hi: float, npix: int, base=None) -> dict:
    """The sweep of gates (i0, i1) over linspace(lo, hi, npix) each, other
    gates at ``base``: the same voltages as ``sweep2d`` (a swept gate's base
    entry is replaced, so v0 is zero there)."""
    v0 = np.zeros(n_gate) if base is None else np.array(base, np.float64)
    v0[list(gates)] = 0.0
    e1 = np.zeros(n_gate)
    e2 = np.zeros(n_gate)
    e1[gates[0]] = 1.0
    e2[gates[1]] = 1.0
    return dict(v0=v0, e1=e1, e2=e2, a0=lo, a1=hi, nx=npix, b0=lo, b1=hi, ny=npix)


def _maxwell(diag, pairs, rng, lo_hi):
    """Maxwell block with the given diagonal and -U[lo, hi] on the pairs."""
    n = len(diag)
    c = np.diag(np.asarray(diag, np.float64))
    for (i, j), (lo, hi) in zip(pairs, lo_hi):
        v = rng.uniform(lo, hi)
        c[i, j] = c[j, i] = -v
    return c


def grid_pairs(rows: int, cols: int):
    """Nearest-neighbour and diagonal-neighbour index pairs of a rows x cols array."""
    idx = lambda r, c: r * cols + c
    nn, dg = [], []
    for r in range(rows):
        for c in range(cols):
            if c + 1 < cols:
                nn.append((idx(r, c), idx(r, c + 1)))
            if r + 1 < rows:
                nn.append((idx(r, c), idx(r + 1, c)))
            if r + 1 < rows and c + 1 < cols:
                dg.append((idx(r, c), idx(r + 1, c + 1)))
            if r + 1 < rows and c - 1 >= 0:
                dg.append((idx(r, c), idx(r + 1, c - 1)))
    return nn, dg


def _plunger_cgd(n_dot, n_gate, nn_pairs, rng, diag=(0.5, 1.0), cross=(0.05, 0.15)):
    cgd = np.zeros((n_dot, n_gate))
    for i in range(min(n_dot, n_gate)):
        cgd[i, i] = rng.uniform(*diag)
    for i, j in nn_pairs:
        if j < n_gate:
            cgd[i, j] = rng.uniform(*cross)
        if i < n_gate:
            cgd[j, i] = rng.uniform(*cross)
    return cgd


# ---------------------------------------------------------------------------
# the five workloads
# ---------------------------------------------------------------------------

def double_dot(seed: int = 0, npix: int = 100, lo: float = -2.0, hi: float = 8.0) -> Diagram:
    """Open double dot, 2 plunger gates, both swept over [lo, hi] (npix x npix).
    C_dd diagonal U[1.0, 1.4], coupling U[0.1, 0.3]; C_gd diagonal U[0.5, 1.0],
    cross terms U[0.05, 0.15]."""
    rng = np.random.default_rng(seed)
    cdd = _maxwell(rng.uniform(1.0, 1.4, 2), [(0, 1)], rng, [(0.1, 0.3)])
    cgd = np.array([[rng.uniform(0.5, 1.0), rng.uniform(0.05, 0.15)],
                    [rng.uniform(0.05, 0.15), rng.uniform(0.5, 1.0)]])
    ax = np.linspace(lo, hi, npix)
    return Diagram(cdd, cgd, sweep2d(2, (0, 1), ax, ax), shape=(npix, npix),
                   meta=dict(workload="open double dot", seed=seed),
                   sweep=gate_sweep(2, (0, 1), lo, hi, npix))


def chain4(seed: int = 100, npix: int = 100, kT: float = 0.0) -> Diagram:
    """Open 4-dot linear chain with 5 gates (4 plungers + 1 gate coupled to every
    dot by U[0, 0.05]); nearest-neighbour couplings U[0.1, 0.3], next-nearest
    U[0.02, 0.06]; gates 2 and 3 (indices 1, 2) swept over [-2, 8]."""
    rng = np.random.default_rng(seed)
    nn = [(0, 1), (1, 2), (2, 3)]
    nnn = [(0, 2), (1, 3)]
    while True:
        cdd = _maxwell(rng.uniform(1.0, 1.4, 4), nn + nnn, rng,
                       [(0.1, 0.3)] * 3 + [(0.02, 0.06)] * 2)
        if _is_pd(cdd):
            break
    cgd = _plunger_cgd(4, 5, nn, rng)
    cgd[:, 4] = rng.uniform(0.0, 0.05, 4)
    ax = np.linspace(-2.0, 8.0, npix)
    return Diagram(cdd, cgd, sweep2d(5, (1, 2), ax, ax), kT=kT, shape=(npix, npix),
                   meta=dict(workload="open 4-dot chain", seed=seed),
                   sweep=gate_sweep(5, (1, 2), -2.0, 8.0, npix))


def grid4x4(seed: int = 200, npix: int = 100, t: float = 1.0) -> Diagram:
    """Open 16-dot 4x4 array with 16 plunger gates.  Nearest-neighbour couplings
    U[0.1, 0.3], diagonal-neighbour U[0.02, 0.08], diagonal U[1.0, 1.4].  The
    sweep moves two virtual gates (App. I): V = V0 + a d_5 + b d_6 with
    d_i = C_gd^{-1} C_dd e_i, V0 = C_gd^{-1} y0, y0 ~ U[1, 3]^16 and
    a, b in linspace(-2, 8, npix)."""
    rng = np.random.default_rng(seed)
    nn, dg = grid_pairs(4, 4)
    rejected = 0
    while True:
        cdd = _maxwell(rng.uniform(1.0, 1.4, 16), nn + dg, rng,
                       [(0.1, 0.3)] * len(nn) + [(0.02, 0.08)] * len(dg))
        if _is_pd(cdd):
            break
        rejected += 1
    cgd = _plunger_cgd(16, 16, nn, rng)
    y0 = rng.uniform(1.0, 3.0, 16)
    V0 = np.linalg.solve(cgd, y0)
    d5 = np.linalg.solve(cgd, cdd[:, 5])
    d6 = np.linalg.solve(cgd, cdd[:, 6])
    ax = np.linspace(-2.0, 8.0, npix)
    aa, bb = np.meshgrid(ax, ax)
    V = V0[None, :] + aa.ravel()[:, None] * d5[None, :] + bb.ravel()[:, None] * d6[None, :]
    return Diagram(cdd, cgd, V, t=t, shape=(npix, npix),
                   meta=dict(workload="open 16-dot 4x4 array", seed=seed, rejected=rejected),
                   sweep=dict(v0=V0, e1=d5, e2=d6, a0=-2.0, a1=8.0, nx=npix, b0=-2.0, b1=8.0,
                              ny=npix))


def ragged_diagram(d: int, npix: int = 64) -> Diagram:
    """Diagram ``d`` of the ragged dataset batch: N ~ U{2..8} dots, a 2 x N/2
    layout with probability 1/2 when N is even (linear otherwise), couplings and
    plungers as the double dot, closed with probability 1/2 with N_hat ~ U{1..N},
    kT ~ U[0, 0.02], gates 0 and 1 swept over [-2, 8] on npix x npix."""
    rng = np.random.default_rng(3_000_000 + d)
    n = int(rng.integers(2, 9))
    if n % 2 == 0 and rng.random() < 0.5:
        nn, _ = grid_pairs(2, n // 2)
        layout = "2x%d" % (n // 2)
    else:
        nn = [(i, i + 1) for i in range(n - 1)]
        layout = "linear"
    while True:
        cdd = _maxwell(rng.uniform(1.0, 1.4, n), nn, rng, [(0.1, 0.3)] * len(nn))
        if _is_pd(cdd):
            break
    cgd = _plunger_cgd(n, n, nn, rng)
    closed = bool(rng.random() < 0.5)
    nhat = int(rng.integers(1, n + 1)) if closed else 0
    kT = float(rng.uniform(0.0, 0.02))
    ax = np.linspace(-2.0, 8.0, npix)
    return Diagram(cdd, cgd, sweep2d(n, (0, 1), ax, ax), closed=closed, nhat=nhat, kT=kT,
                   shape=(npix, npix), meta=dict(workload="ragged batch item", d=d, layout=layout),
                   sweep=gate_sweep(n, (0, 1), -2.0, 8.0, npix))


def ragged_batch(n_diag: int = 4096, npix: int = 64, start: int = 0):
    return [ragged_diagram(start + d, npix) for d in range(n_diag)]


@dataclass
class AdjointCase:
    """2x4 open array plus one sensor dot (index 8) and its gate (index 8)."""

    cdd: np.ndarray      # 9 x 9 Maxwell block (array + sensor)
    cgd: np.ndarray      # 9 x 9
    V: np.ndarray        # P x 9
    kT: float
    cdd_target: np.ndarray
    cgd_target: np.ndarray
    shape: tuple
    sweep: dict | None = None


def adjoint_case(seed: int = 400, npix: int = 100, kT: float = 0.02) -> AdjointCase:
    """Couplings of the array as the 4x4 grid; the sensor dot couples to all 8
    dots by U[0.02, 0.08]; plungers as the 4x4 grid; the sensor gate couples
    to the sensor dot by U[0.5, 1.0] and to each array dot by U[0, 0.05].
    Gates 0 and 1 sweep [-2, 8]; the other plungers sit at C_gd^{-1} y0 with
    y0 ~ U[1, 3]; the sensor gate at 0 V.  The target capacitances multiply
    every entry by (1 + 0.05 eps), eps ~ N(0, 1), symmetrically for C_dd."""
    rng = np.random.default_rng(seed)
    nn, dg = grid_pairs(2, 4)
    while True:
        cdd = np.zeros((9, 9))
        cdd[:8, :8] = _maxwell(rng.uniform(1.0, 1.4, 8), nn + dg, rng,
                               [(0.1, 0.3)] * len(nn) + [(0.02, 0.08)] * len(dg))
        cdd[8, 8] = rng.uniform(1.0, 1.4)
        cs = rng.uniform(0.02, 0.08, 8)
        cdd[8, :8] = -cs
        cdd[:8, 8] = -cs
        if _is_pd(cdd):
            break
    cgd = np.zeros((9, 9))
    cgd[:8, :8] = _plunger_cgd(8, 8, nn, rng)
    cgd[8, 8] = rng.uniform(0.5, 1.0)
    cgd[:8, 8] = rng.uniform(0.0, 0.05, 8)
    y0 = rng.uniform(1.0, 3.0, 8)
    base = np.zeros(9)
    base[:8] = np.linalg.solve(cgd[:8, :8], y0)
    ax = np.linspace(-2.0, 8.0, npix)
    V = sweep2d(9, (0, 1), ax, ax, base=base)
    eps = rng.standard_normal((9, 9))
    eps = np.triu(eps) + np.triu(eps, 1).T
    cdd_t = cdd * (1.0 + 0.05 * eps)
    cgd_t = cgd * (1.0 + 0.05 * rng.standard_normal((9, 9)))
    return AdjointCase(cdd, cgd, V, kT, cdd_t, cgd_t, (npix, npix),
                       gate_sweep(9, (0, 1), -2.0, 8.0, npix, base=base))


def paper_example():
    """The double dot of the worked example (Sec. 5): C_dd, C_gd as printed,
    both gates over linspace(-3, 3, 100), closed arrays with 2 charges."""
    cdd = np.array([[1.3, -0.1], [-0.1, 1.3]])
    cgd = np.array([[1.0, 0.2], [0.2, 1.0]])
    ax = np.linspace(-3.0, 3.0, 100)
    return Diagram(cdd, cgd, sweep2d(2, (0, 1), ax, ax), shape=(100, 100),
                   meta=dict(workload="worked example of Sec. 5"))


def random_maxwell(n_dot: int, seed: int, n_gate: int | None = None, dot_scale: float = 1.0):
    """Random capacitances as in the paper's benchmark (Sec. 7): every element
    of the (N + G) x (N + G) capacitance matrix between the nodes (dots, then
    gates) drawn from U[0, 1), symmetric (the upper triangle, diagonal
    included, is drawn and mirrored; a diagonal element is the node's
    capacitance to ground), then converted to the Maxwell form of App. B:
    diagonal = the sum of the node's row, off-diagonal = minus the element.
    Returns (cdd, cgd) with cgd taken positive (coupling).

    ``dot_scale`` multiplies the dot-dot elements before the conversion;
    1 is the paper's draw.  Values below 1 give a weakly coupled variant that
    is not the paper's benchmark."""
    rng = np.random.default_rng(seed)
    n_gate = n_dot if n_gate is None else n_gate
    m = n_dot + n_gate
    c = np.triu(rng.uniform(0.0, 1.0, (m, m)))
    c = c + np.triu(c, 1).T
    off = c - np.diag(np.diag(c))
    off[:n_dot, :n_dot] *= dot_scale
    maxwell = np.diag(off.sum(axis=1) + np.diag(c)) - off
    cdd = maxwell[:n_dot, :n_dot].copy()
    cgd = -maxwell[:n_dot, n_dot:].copy()
    return cdd, cgd


def paper_replica(n_dot: int, seed: int = 500, npix: int = 100, closed: bool = False,
                  vmin: float = -1.0, vmax: float = 2.0, dot_scale: float = 1.0) -> Diagram:
    """The paper's benchmark (Sec. 7): random capacitances (``random_maxwell``,
    one gate per dot) and npix x npix gate-voltage configurations drawn
    uniformly in [vmin, vmax]^G (the paper gives no range; negative voltages
    make some analytic minima infeasible, so the QP runs too); closed arrays
    hold as many carriers as dots.  ``dot_scale`` < 1 is the weakly coupled
    variant (not the paper's draw)."""
    cdd, cgd = random_maxwell(n_dot, seed, dot_scale=dot_scale)
    rng = np.random.default_rng(seed + 7)
    V = rng.uniform(vmin, vmax, (npix * npix, cgd.shape[1]))
    return Diagram(cdd, cgd, V, closed=closed, nhat=n_dot if closed else 0,
                   meta=dict(workload="paper benchmark replica" if dot_scale == 1.0 else
                             "paper benchmark replica, dot-dot couplings x %g" % dot_scale,
                             seed=seed))
