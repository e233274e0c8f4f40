"""Matrix-core scorer (dense box, T = 0, N >= 9) against the FP64 oracle.

The integer ground state must equal the oracle's replay of the method at
every pixel except near ties (FP64 gap < 1e-9) and candidate-set boundary
pixels; the approximate forms (FP32, split BF16) get there through the
certified error band plus the FP64 re-score of flagged pixels.
"""
import sys

import numpy as np
import pytest
import torch

from paper_2404_04994_amd import workloads as W

pytestmark = pytest.mark.gpu

PRECS = ["fp32", "bf16x3", "bf16x2"]


@pytest.fixture(scope="module")
def qa():
    from paper_2404_04994_amd import qarray
    assert torch.cuda.is_available()
    qarray.load()
    return qarray


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def compare(qa, oracle, d, prec, idx=None, t=1.0, closed=False, nhat=0):
    V = torch.as_tensor(d.V).cuda()
    n, st = qa.ground_state(d.cdd, d.cgd, V, precision=prec, stats=True, t=t, closed=closed,
                            nhat=nhat)
    n = n.cpu().numpy()
    if idx is None:
        idx = np.arange(d.P)
    ref = oracle.method_gs(d.cdd, d.cgd, d.V[idx], t=t, closed=closed, nhat=nhat)
    excl = (ref["e2"] - ref["e1"] < 1e-9) | ((ref["info"] & oracle.INFO_AMBIGUOUS) > 0)
    bad = (n[idx] != ref["n"]).any(1) & ~excl
    say("N=%d P=%d t=%.3f checked=%d prec=%s mismatches=%d excluded=%d near_tie=%d qp=%d "
        "candidates=%d" % (d.n_dot, d.P, t, len(idx), prec, bad.sum(), excl.sum(),
                           st["near_tie_pixels"], st["qp_pixels"], st["candidates"]))
    assert bad.sum() == 0, np.where(bad)[0][:10]
    if closed:
        assert (n[idx].sum(1) == nhat).all()
    if t >= 1.0 and not closed:
        assert st["candidates"] == d.P << d.n_dot
    elif len(idx) == d.P:
        assert st["candidates"] == ref["ncand"].sum()
    return n, st


@pytest.mark.parametrize("prec", PRECS)
def test_grid16_small_full_parity(qa, oracle, prec):
    """4x4 array on a 40 x 40 sweep: every pixel against the oracle.  The
    share of pixels the band sends to the FP64 re-score is bounded: the
    BF16x2 band (2^-15 S) is four times wider than the FP32 / BF16x3 one."""
    d = W.grid4x4(201, npix=40)
    _, st = compare(qa, oracle, d, prec)
    assert st["near_tie_pixels"] <= (0.12 if prec == "bf16x2" else 0.05) * d.P


@pytest.fixture(scope="module")
def headline(oracle):
    """The full 100 x 100 16-dot diagram and the oracle's replay of the method
    at every one of its 10^4 pixels (computed once for the three forms)."""
    d = W.grid4x4(200)
    ref = oracle.method_gs(d.cdd, d.cgd, d.V)
    return d, ref


@pytest.mark.parametrize("prec", PRECS)
def test_grid16_full_size(qa, oracle, headline, prec):
    """The full 100 x 100 16-dot diagram (the headline workload): every pixel
    against the oracle, for each approximate scoring form, and every pixel
    against the FP64 GPU form."""
    d, ref = headline
    V = torch.as_tensor(d.V).cuda()
    n, st = qa.ground_state(d.cdd, d.cgd, V, precision=prec, stats=True)
    n = n.cpu().numpy()
    excl = (ref["e2"] - ref["e1"] < 1e-9) | ((ref["info"] & oracle.INFO_AMBIGUOUS) > 0)
    bad = (n != ref["n"]).any(1) & ~excl
    say("full 16-dot diagram, %s: %d pixels checked, mismatches %d, excluded %d, near ties "
        "re-scored %d, qp %d" % (prec, d.P, bad.sum(), excl.sum(), st["near_tie_pixels"],
                                 st["qp_pixels"]))
    assert bad.sum() == 0, np.where(bad)[0][:10]
    assert excl.sum() <= 5
    assert st["candidates"] == d.P << d.n_dot
    assert st["qp_pixels"] == int(((ref["info"] & oracle.INFO_QP) > 0).sum())
    n64, st64 = qa.ground_state(d.cdd, d.cgd, V, precision="fp64", stats=True)
    diff = (n != n64.cpu().numpy()).any(1).sum()
    say("vs fp64 GPU: differing pixels", diff, "fp64 gaps<1e-9", st64["fp64_gap_below_1e9"])
    assert diff <= st64["fp64_gap_below_1e9"]


@pytest.mark.parametrize("n_dot", [9, 10, 11, 12, 13, 14, 15])
def test_partial_high_index(qa, oracle, n_dot):
    """9..15 dots: the high index has 1..7 bits, so row tiles are partly
    masked (N < 12) or fewer than sixteen (N < 16)."""
    rng = np.random.default_rng(n_dot)
    cdd = np.diag(rng.uniform(1.0, 1.4, n_dot))
    for i in range(n_dot - 1):
        cdd[i, i + 1] = cdd[i + 1, i] = -rng.uniform(0.1, 0.3)
    for i in range(n_dot - 2):
        cdd[i, i + 2] = cdd[i + 2, i] = -rng.uniform(0.02, 0.06)
    cgd = np.diag(rng.uniform(0.5, 1.0, n_dot))
    y0 = rng.uniform(1, 3, n_dot)
    ax = np.linspace(-2, 8, 24)
    aa, bb = np.meshgrid(ax, ax)
    d3 = np.linalg.solve(cgd, cdd[:, 3])
    d10 = np.linalg.solve(cgd, cdd[:, n_dot - 1])
    V = np.linalg.solve(cgd, y0)[None, :] + aa.ravel()[:, None] * d3 + bb.ravel()[:, None] * d10
    d = W.Diagram(cdd, cgd, V)
    for prec in PRECS:
        compare(qa, oracle, d, prec)


@pytest.mark.parametrize("t", [2 / 3, 0.5, 1 / 3, 0.1, 0.0])
@pytest.mark.parametrize("prec", PRECS)
def test_grid16_thresholded(qa, oracle, prec, t):
    """Thresholded candidate sets (Sec. 3.2.2) on the matrix cores: each
    pixel scores only the sub-box of its free dots; every pixel of a 40 x 40
    sweep against the oracle's replay at the same t, and the number of
    candidates equals the sum of the sub-box sizes."""
    d = W.grid4x4(203, npix=40)
    compare(qa, oracle, d, prec, t=t)


@pytest.mark.parametrize("n_dot", [9, 11, 13, 16])
def test_thresholded_partial_high_index(qa, oracle, n_dot):
    """Sub-boxes on 9..16 dots: the fixed-dot penalty and the tile skips
    combine with the absent high dots of N < 16."""
    rng = np.random.default_rng(50 + n_dot)
    cdd = np.diag(rng.uniform(1.0, 1.4, n_dot))
    for i in range(n_dot - 1):
        cdd[i, i + 1] = cdd[i + 1, i] = -rng.uniform(0.1, 0.3)
    cgd = np.diag(rng.uniform(0.5, 1.0, n_dot))
    V = rng.uniform(-1, 6, (700, n_dot))
    d = W.Diagram(cdd, cgd, V)
    for t in (0.8, 0.5, 0.25):
        compare(qa, oracle, d, "bf16x3", t=t)
    compare(qa, oracle, d, "fp32", t=0.5)


@pytest.mark.parametrize("nhat", [8, 20, 30])
@pytest.mark.parametrize("prec", PRECS)
def test_grid16_closed(qa, oracle, prec, nhat):
    """Closed 16-dot array (Sec. 2, constraint iii) on the matrix cores: the
    subsets of the free dots with exactly k raised, every pixel against the
    oracle, candidate counts C(free, k) summed."""
    d = W.grid4x4(207, npix=12)
    compare(qa, oracle, d, prec, closed=True, nhat=nhat)


@pytest.mark.parametrize("n_dot", [9, 11, 12, 13, 14, 15, 16])
def test_closed_replica_and_thresholded(qa, oracle, n_dot):
    """The paper's closed benchmark inputs (as many carriers as dots), dense
    and thresholded (t < 1 closed pixels may double their threshold)."""
    d = W.paper_replica(n_dot, seed=700 + n_dot, npix=15, closed=True)
    for t in (1.0, 0.5, 0.2):
        compare(qa, oracle, d, "bf16x3", t=t, closed=True, nhat=n_dot)
    compare(qa, oracle, d, "fp32", closed=True, nhat=n_dot)


def test_ragged_pixel_count(qa, oracle):
    d = W.grid4x4(202, npix=40)
    for P in (1, 5, 63, 1001):
        sub = W.Diagram(d.cdd, d.cgd, d.V[:P])
        compare(qa, oracle, sub, "bf16x3")


def test_graph_replays_match_eager(qa, oracle):
    """Replays of the captured graph, with other eager work and waits between
    them, give the eager result every time (single-diagram and soft paths)."""
    d = W.grid4x4(206, npix=24)
    c = W.chain4(131, npix=30)
    V = torch.as_tensor(d.V).cuda()
    Vc = torch.as_tensor(c.V).cuda()
    qa.graphs_enable(False)
    ref = qa.ground_state(d.cdd, d.cgd, V, precision="bf16x3").cpu()
    ref_soft, _ = qa.soft_charge(c.cdd, c.cgd, Vc, 0.02)
    ref_soft = ref_soft.cpu()
    try:
        qa.graphs_enable(True)
        out = torch.empty_like(ref).cuda()
        for i in range(5):
            qa.ground_state(d.cdd, d.cgd, V, precision="bf16x3", out=out)
            torch.cuda.synchronize()
            assert torch.equal(out.cpu(), ref), i
            qa.graphs_enable(False)
            qa.ground_state(c.cdd, c.cgd, Vc)           # eager work between replays
            torch.cuda.synchronize()
            qa.graphs_enable(True)
            nb, _ = qa.soft_charge(c.cdd, c.cgd, Vc, 0.02)
            torch.cuda.synchronize()
            assert torch.equal(nb.cpu(), ref_soft), i
    finally:
        qa.graphs_enable(False)


@pytest.mark.parametrize("prec", PRECS)
def test_bound_order_equals_exhaustive(qa, prec):
    """The bound-ordered search of the dense box (N >= 13) returns, at every
    pixel of the full 100 x 100 16-dot diagram, the state the exhaustive
    scorer returns, while computing a fraction of the energies."""
    d = W.grid4x4(200)
    V = torch.as_tensor(d.V).cuda()
    nb, sb = qa.ground_state(d.cdd, d.cgd, V, precision=prec, stats=True)
    ne, se = qa.ground_state(d.cdd, d.cgd, V, precision=prec, stats=True, exhaustive=True)
    diff = (nb.cpu().numpy() != ne.cpu().numpy()).any(1).sum()
    say("%s: bound scored %d of %d states (%.2f%%), near ties %d / exhaustive %d, diff %d"
        % (prec, sb["scored"], sb["candidates"], 100.0 * sb["scored"] / sb["candidates"],
           sb["near_tie_pixels"], se["near_tie_pixels"], diff))
    assert diff == 0
    assert sb["candidates"] == se["candidates"] == d.P << 16
    assert se["scored"] == se["candidates"]
    # every pixel scores at least the row (256 states) that holds its argmin;
    # the bound order leaves most of the box unscored
    assert 256 * d.P <= sb["scored"] < sb["candidates"] // 8


@pytest.mark.parametrize("n_dot,seed", [(13, 601), (14, 602), (15, 603), (16, 604)])
def test_bound_order_paper_replica(qa, oracle, n_dot, seed):
    """Random capacitances of the paper's benchmark (Sec. 7), 13..16 dots:
    the bound-ordered search against the oracle at every pixel, and against
    the exhaustive scorer."""
    d = W.paper_replica(n_dot, seed=seed, npix=24)
    n, st = compare(qa, oracle, d, "bf16x3")
    V = torch.as_tensor(d.V).cuda()
    ne = qa.ground_state(d.cdd, d.cgd, V, precision="bf16x3", exhaustive=True).cpu().numpy()
    assert (n == ne).all()
    assert st["scored"] < st["candidates"]
    compare(qa, oracle, d, "fp32")
    compare(qa, oracle, d, "bf16x2")


@pytest.mark.parametrize("case", ["closed20", "closed_replica", "t0.5", "t0.333", "closed_t0.5"])
def test_bound_order_closed_and_thresholded_equal_exhaustive(qa, case):
    """Bound-ordered search of the thresholded sub-boxes and of the closed
    subsets (the closed bound adds the fixed low-part sum): at every pixel the
    exhaustive scorer's state, with fewer energies computed."""
    if case == "closed_replica":
        d = W.paper_replica(16, seed=730, npix=60, closed=True)
        kw = dict(closed=True, nhat=16)
    else:
        d = W.grid4x4(208, npix=60)
        kw = {}
        if case.startswith("closed"):
            kw = dict(closed=True, nhat=20)
        if "t0." in case:
            kw["t"] = float(case.split("t")[-1])
    V = torch.as_tensor(d.V).cuda()
    for prec in PRECS:
        nb, sb = qa.ground_state(d.cdd, d.cgd, V, precision=prec, stats=True, **kw)
        ne, se = qa.ground_state(d.cdd, d.cgd, V, precision=prec, stats=True, exhaustive=True,
                                 **kw)
        diff = (nb.cpu().numpy() != ne.cpu().numpy()).any(1).sum()
        say("%s %s: scored %d (exhaustive %d) of %d candidates, near ties %d / %d, diff %d"
            % (case, prec, sb["scored"], se["scored"], sb["candidates"], sb["near_tie_pixels"],
               se["near_tie_pixels"], diff))
        assert diff == 0
        assert sb["candidates"] == se["candidates"]
        if kw.get("closed"):
            assert (nb.cpu().numpy().sum(1) == kw["nhat"]).all()
