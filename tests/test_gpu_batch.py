"""Ragged batch (mixed dot counts, open and closed arrays, mixed kT) in one
persistent launch, against the FP64 oracle diagram by diagram."""
import sys

import numpy as np
import pytest
import torch

from paper_2404_04994_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def qa():
    from paper_2404_04994_amd import qarray
    assert torch.cuda.is_available()
    qarray.load()
    return qarray


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def check_diagram(oracle, d, n, nbar):
    """One diagram's outputs against the oracle at every pixel: n bit-exact
    except FP64 ties and candidate-set boundary pixels, <n> within
    1e-5 max(1, |n_ref|) (kT > 0) or equal to n (kT = 0).  Returns the
    largest scaled soft-charge error."""
    ref = oracle.method_gs(d.cdd, d.cgd, d.V, closed=d.closed, nhat=d.nhat, t=d.t)
    excl = (ref["e2"] - ref["e1"] < 1e-9) | ((ref["info"] & oracle.INFO_AMBIGUOUS) > 0)
    bad = (n != ref["n"]).any(1) & ~excl
    assert bad.sum() == 0, np.where(bad)[0][:5]
    worst = 0.0
    if nbar is not None:
        if d.kT > 0:
            rs, _, _ = oracle.method_soft(d.cdd, d.cgd, d.V, closed=d.closed, nhat=d.nhat,
                                          t=d.t, kT=d.kT)
            err = (np.abs(nbar - rs) / np.maximum(1, np.abs(rs)))[~excl]
            worst = float(err.max(initial=0))
        else:
            assert (nbar[~excl] == ref["n"][~excl]).all()
    return worst


def check_batch(qa, oracle, diagrams, with_nbar=True):
    b = qa.Batch(diagrams)
    st = b.run(with_nbar=with_nbar, stats=True)
    say("batch of %d diagrams, %d pixels: %s" % (len(diagrams), b.pixels, st))
    assert st["pixels"] == b.pixels and st["qp_failures"] == 0
    worst = 0.0
    for i, d in enumerate(diagrams):
        n, nbar = b.result(i)
        try:
            worst = max(worst, check_diagram(oracle, d, n, nbar if with_nbar else None))
        except AssertionError as e:
            raise AssertionError("diagram %d: %s" % (i, e))
    say("max scaled soft-charge error %.3e" % worst)
    assert worst <= 1e-5
    return b, st


def test_ragged_dataset_full_shape(qa, oracle):
    """The dataset workload at its full shape: 4096 diagrams of 64 x 64
    pixels (16.8 M pixels, 262 144 work items against a few thousand
    resident blocks, so the queue's shards run dry and blocks take work from
    other shards).  A seeded subset of 64 diagrams is compared with the
    oracle at every pixel (n and <n>); every closed diagram holds N_hat
    carriers at every pixel."""
    ds = W.ragged_batch(4096, npix=64)
    b = qa.Batch(ds)
    say("full ragged batch packed: %d pixels" % b.pixels)
    b.run()                       # first call tunes the launch shape
    st = b.run(stats=True)
    say("full ragged batch: %s" % st)
    assert b.pixels == 4096 * 64 * 64
    assert st["pixels"] == b.pixels and st["qp_failures"] == 0
    n_all = b.n.cpu().numpy()
    nbar_all = b.nbar.cpu().numpy()
    for i, d in enumerate(ds):
        if d.closed:
            o = int(b.out_offsets[i])
            rows = n_all[o:o + d.P * d.n_dot].reshape(d.P, d.n_dot)
            assert (rows.sum(1) == d.nhat).all(), i
    sub = np.random.default_rng(31).choice(len(ds), 64, replace=False)
    worst = 0.0
    for i in sub:
        d = ds[i]
        o = int(b.out_offsets[i])
        n = n_all[o:o + d.P * d.n_dot].reshape(d.P, d.n_dot)
        nbar = nbar_all[o:o + d.P * d.n_dot].reshape(d.P, d.n_dot)
        try:
            worst = max(worst, check_diagram(oracle, d, n, nbar))
        except AssertionError as e:
            raise AssertionError("diagram %d (N=%d, closed=%s, kT=%g): %s"
                                 % (i, d.n_dot, d.closed, d.kT, e))
    say("64 diagrams (%d pixels) match the oracle; max scaled soft-charge error %.3e"
        % (sum(ds[i].P for i in sub), worst))
    assert worst <= 1e-5


def test_ragged_dataset_subset(qa, oracle):
    """48 diagrams of the ragged dataset (2..8 dots, 50 % closed, kT in
    [0, 0.02]) at 24 x 24 pixels."""
    check_batch(qa, oracle, W.ragged_batch(48, npix=24))


def test_ragged_with_large_and_thresholded(qa, oracle):
    ds = W.ragged_batch(6, npix=16, start=100)
    g = W.grid4x4(205, npix=12)
    g.kT = 0.01
    ds.append(g)
    c = W.chain4(120, npix=20)
    c.t, c.closed, c.nhat = 0.4, True, 3
    ds.append(c)
    c2 = W.chain4(121, npix=21)  # ragged pixel count (441)
    c2.kT = 0.03
    ds.append(c2)
    check_batch(qa, oracle, ds)


def test_batch_replays_and_no_nbar(qa, oracle):
    """Repeated runs of one batch, launched directly and as graph replays, give
    the first result; the same layout with other matrices (identical headers,
    so only the matrix part of the uploaded plan differs) is uploaded again;
    a batch with other sizes re-plans; nbar may be omitted."""
    ds = W.ragged_batch(10, npix=16, start=200)
    b = qa.Batch(ds)
    b.run()
    first = b.n.clone()
    try:
        for graphs in (False, True):
            qa.graphs_enable(graphs)
            for _ in range(3):
                b.run()
                torch.cuda.synchronize()
                assert torch.equal(first, b.n), graphs
    finally:
        qa.graphs_enable(False)
    for d in ds:
        d.cgd = d.cgd * 1.07
    check_batch(qa, oracle, ds)
    check_batch(qa, oracle, W.ragged_batch(7, npix=20, start=300), with_nbar=False)


def test_empty_diagram_in_batch(qa, oracle):
    ds = W.ragged_batch(3, npix=10, start=400)
    ds[1].V = ds[1].V[:0]
    check_batch(qa, oracle, ds)
