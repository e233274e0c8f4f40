"""qa_ground_state_noalloc (the ground state with the library's static
device scratch, for callers that cannot allocate) against qa_ground_state:
the integer ground states must be identical at every pixel.  Consecutive
calls share one scratch array, so each case runs right after a larger or
differently shaped one: what an earlier call left there must not leak."""
import ctypes as C
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


def both(qa, d, precision="fp64", t=1.0, closed=False, nhat=0):
    """The diagram through both entry points, on the current stream."""
    V = torch.as_tensor(d.V, device="cuda")
    ref = qa.ground_state(d.cdd, d.cgd, V, closed=closed, nhat=nhat, t=t, precision=precision)
    out = torch.full((d.P, d.n_dot), -7, dtype=torch.int32, device="cuda")
    qa.ground_state_noalloc(d.cdd, d.cgd, V, out, closed=closed, nhat=nhat, t=t,
                            precision=precision)
    torch.cuda.synchronize()
    return ref.cpu().numpy(), out.cpu().numpy()


def test_two_calls_second_smaller(qa, oracle):
    """The 16-dot 100 x 100 diagram (split-BF16 matrix-core scorer), then a
    4-dot 30 x 30 sweep (table scorer, fewer dots and gates) in the same
    scratch; the second also against the oracle."""
    big = W.grid4x4(200)
    say("noalloc: 16-dot 100x100 bf16x3, P=%d" % big.P)
    ref, out = both(qa, big, precision="bf16x3")
    assert (out == ref).all(), np.argwhere((out != ref).any(1))[:5]
    small = W.chain4(101, npix=30)
    say("noalloc: 4-dot 30x30 fp64, P=%d" % small.P)
    ref, out = both(qa, small)
    assert (out == ref).all(), np.argwhere((out != ref).any(1))[:5]
    o = oracle.method_gs(small.cdd, small.cgd, small.V)
    tie = (o["e2"] - o["e1"] < 1e-9) | ((o["info"] & oracle.INFO_AMBIGUOUS) > 0)
    assert ((out != o["n"]).any(1) & ~tie).sum() == 0


def test_maximum_size_then_ragged_closed(qa):
    """The largest sweep the scratch holds (256 x 256 = 65536 pixels), then a
    closed thresholded 8-dot array on a ragged pixel count, then a double dot
    with two gates (the zero padding of C_gd must be rewritten)."""
    big = W.grid4x4(203, npix=256)
    assert big.P == qa.NOALLOC_MAX_PIXELS
    say("noalloc: 16-dot 256x256 fp32, P=%d" % big.P)
    ref, out = both(qa, big, precision="fp32")
    assert (out == ref).all()
    rep = W.paper_replica(8, seed=508, npix=37, closed=True)
    say("noalloc: closed 8-dot t=0.5, P=%d" % rep.P)
    ref, out = both(qa, rep, t=0.5, closed=True, nhat=8)
    assert (out == ref).all()
    assert (out.sum(1) == 8).all()
    dd = W.double_dot(3, npix=41)
    say("noalloc: double dot, P=%d" % dd.P)
    ref, out = both(qa, dd)
    assert (out == ref).all()


def test_sixteen_dot_after_small_and_thresholded(qa):
    """Back to 16 dots after smaller problems: a thresholded sub-box search
    (BF16x2) on a ragged 77 x 77 sweep."""
    g = W.grid4x4(207, npix=77)
    say("noalloc: 16-dot 77x77 bf16x2 t=0.5, P=%d" % g.P)
    ref, out = both(qa, g, precision="bf16x2", t=0.5)
    assert (out == ref).all()


def test_rejects_beyond_maximum(qa):
    d = W.chain4(102, npix=10)
    lib = qa.load()
    pb, keep = qa.make_problem(d.cdd, d.cgd)
    V = torch.zeros((qa.NOALLOC_MAX_PIXELS + 1, d.cgd.shape[1]), dtype=torch.float64,
                    device="cuda")
    out = torch.zeros((qa.NOALLOC_MAX_PIXELS + 1, 4), dtype=torch.int32, device="cuda")
    st = lib.qa_ground_state_noalloc(C.byref(pb), C.c_void_p(V.data_ptr()), V.shape[0],
                                     C.c_void_p(out.data_ptr()), None)
    assert st == 2 and b"static scratch" in lib.qa_last_error()
    torch.cuda.synchronize()
    assert int(out.abs().sum()) == 0  # nothing was enqueued
    del keep
