"""The constrained continuous minimum x* (Sec. 3.1: analytic minimum, else
the exact QP of Sec. 3.1.2) of the HIP path against the oracle, pixel by
pixel, to 1e-9 (scaled by max(1, |x|)).  The integer ground states can hide
a wrong x* (any box that contains the argmin gives the same answer), so x* is
checked on its own."""
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


def check_x(qa, oracle, cdd, cgd, V, closed=False, nhat=0, label=""):
    ref = oracle.method_setup(cdd, cgd, V, closed=closed, nhat=nhat)
    x, fl, st = qa.continuous_min(cdd, cgd, torch.as_tensor(V).cuda(), closed, nhat, stats=True)
    x, fl = x.cpu().numpy(), fl.cpu().numpy()
    err = (np.abs(x - ref["xstar"]) / np.maximum(1.0, np.abs(ref["xstar"]))).max(initial=0)
    qp_ref = (ref["info"] & oracle.INFO_QP) > 0
    print("%s N=%d P=%d closed=%s nhat=%d: max scaled |dx|=%.2e qp=%d (oracle %d) unsettled=%d"
          % (label, cdd.shape[0], V.shape[0], closed, nhat, err, (fl & 1).sum(), qp_ref.sum(),
             (fl & 2).sum()), flush=True)
    sys.stdout.flush()
    assert err <= 1e-9
    assert ((fl & 1) > 0).tolist() == qp_ref.tolist()
    assert (fl & 2).sum() == 0 and st["qp_failures"] == 0
    assert (x >= 0).all()
    if closed:
        assert np.abs(x.sum(1) - nhat).max() <= 1e-9 * max(1, nhat)


def test_open_grid16(qa, oracle):
    d = W.grid4x4(200)
    check_x(qa, oracle, d.cdd, d.cgd, d.V, label="16-dot")


@pytest.mark.parametrize("nhat", [0, 1, 2, 4, 7])
def test_closed_chain4(qa, oracle, nhat):
    d = W.chain4(102, npix=60)
    check_x(qa, oracle, d.cdd, d.cgd, d.V, True, nhat, "chain4")


def test_open_chain4_and_double_dot(qa, oracle):
    for d in (W.chain4(100), W.double_dot(0)):
        check_x(qa, oracle, d.cdd, d.cgd, d.V)


@pytest.mark.parametrize("n,nhat", [(8, 3), (8, 6), (12, 9), (12, 4), (16, 10)])
def test_closed_larger(qa, oracle, n, nhat):
    rng = np.random.default_rng(1000 + n * 10 + nhat)
    cdd = np.diag(rng.uniform(1.0, 1.4, n))
    for i in range(n - 1):
        cdd[i, i + 1] = cdd[i + 1, i] = -rng.uniform(0.1, 0.3)
    cgd = np.diag(rng.uniform(0.5, 1.0, n))
    V = rng.uniform(-1, 3, (300, n))
    check_x(qa, oracle, cdd, cgd, V, True, nhat, "closed")
