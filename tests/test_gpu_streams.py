"""Calls on two HIP streams at once use separate workspaces: results equal
those of the same calls made one after another on one stream."""
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


def test_two_streams_match_serial(qa):
    big = W.grid4x4(200)
    small = W.chain4(105, npix=60)
    Vb = torch.as_tensor(big.V, device="cuda")
    Vs = torch.as_tensor(small.V, device="cuda")
    # serial references on the default stream
    ref_b = qa.ground_state(big.cdd, big.cgd, Vb, precision="bf16x3").cpu()
    ref_s = qa.ground_state(small.cdd, small.cgd, Vs).cpu()
    ref_nb, _ = qa.soft_charge(small.cdd, small.cgd, Vs, 0.01)
    ref_nb = ref_nb.cpu()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    torch.cuda.synchronize()
    outs = []
    for _ in range(3):
        with torch.cuda.stream(s1):
            nb1 = qa.ground_state(big.cdd, big.cgd, Vb, precision="bf16x3", stream=s1)
        with torch.cuda.stream(s2):
            ns2 = qa.ground_state(small.cdd, small.cgd, Vs, stream=s2)
            soft2, _ = qa.soft_charge(small.cdd, small.cgd, Vs, 0.01, stream=s2)
        outs.append((nb1, ns2, soft2))
    torch.cuda.synchronize()
    for nb1, ns2, soft2 in outs:
        assert torch.equal(nb1.cpu(), ref_b)
        assert torch.equal(ns2.cpu(), ref_s)
        assert torch.equal(soft2.cpu(), ref_nb)
    for s in (s1, s2):
        qa.release(s)
