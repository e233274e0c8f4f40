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


def check_batch(qa, oracle, diagrams, with_nbar=True):
    b = qa.Batch(diagrams)
    st = b.run(with_nbar=with_nbar, stats=True)
    say("batch of %d diagrams, %d pixels: %s" % (len(diagrams), b.pixels, st))
    assert st["pixels"] == b.pixels and st["qp_failures"] == 0
    worst = 0.0
    for i, d in enumerate(diagrams):
        n, nbar = b.result(i)
        ref = oracle.method_gs(d.cdd, d.cgd, d.V, closed=d.closed, nhat=d.nhat, t=d.t)
        excl = (ref["e2"] - ref["e1"] < 1e-9) | ((ref["info"] & oracle.INFO_AMBIGUOUS) > 0)
        bad = (n != ref["n"]).any(1) & ~excl
        assert bad.sum() == 0, (i, np.where(bad)[0][:5])
        if with_nbar:
            if d.kT > 0:
                rs, _, _ = oracle.method_soft(d.cdd, d.cgd, d.V, closed=d.closed, nhat=d.nhat,
                                              t=d.t, kT=d.kT)
                err = (np.abs(nbar - rs) / np.maximum(1, np.abs(rs)))[~excl]
                worst = max(worst, err.max(initial=0))
            else:
                assert (nbar[~excl] == ref["n"][~excl]).all()
    say("max scaled soft-charge error %.3e" % worst)
    assert worst <= 1e-5
    return b, st


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
