"""Sweep entry points (qa_grid: the voltages formed inside the kernels from
v0, e1, e2 and two linspace ranges) against the explicit-voltage entry
points on the same sweeps: ground states, soft charges and the batch are
bitwise identical, the adjoint's gradients identical up to the order of
its atomic sums.  The explicit-voltage path is itself compared with the
oracle in the other GPU tests."""
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


def bits(x):
    return np.ascontiguousarray(x).view(np.int64 if x.dtype == np.float64 else np.int32)


CASES = [
    ("double dot 100x100", lambda: W.double_dot(0), dict()),
    ("4-dot chain 37x37", lambda: W.chain4(101, npix=37), dict()),
    ("closed 4-dot chain, t = 0.4", lambda: W.chain4(102, npix=30), dict(closed=True, nhat=3, t=0.4)),
    ("16-dot 100x100 bf16x3", lambda: W.grid4x4(200), dict(precision="bf16x3")),
    ("16-dot 77x77 fp32, t = 0.5", lambda: W.grid4x4(207, npix=77), dict(precision="fp32", t=0.5)),
    ("16-dot 40x40 fp64", lambda: W.grid4x4(201, npix=40), dict()),
]


@pytest.mark.parametrize("name,make,kw", CASES, ids=[c[0] for c in CASES])
def test_ground_state_grid_equals_explicit(qa, name, make, kw):
    d = make()
    say("ground state over a sweep: %s, P=%d" % (name, d.P))
    V = torch.as_tensor(d.V, device="cuda")
    ref, st_ref = qa.ground_state(d.cdd, d.cgd, V, stats=True, **kw)
    got, st = qa.ground_state_grid(d.cdd, d.cgd, d.sweep, stats=True, **kw)
    assert np.array_equal(ref.cpu().numpy(), got.cpu().numpy())
    assert st == st_ref


def test_ragged_sweep_shapes(qa):
    """nx != ny, a single row and a single column, a descending range."""
    d = W.chain4(103, npix=10)
    for nx, ny, a0, a1 in ((23, 7, -2.0, 8.0), (1, 9, 3.0, 3.0), (31, 1, 8.0, -2.0)):
        sw = dict(d.sweep, nx=nx, ny=ny, a0=a0, a1=a1)
        V = torch.as_tensor(W.sweep_voltages(sw), device="cuda")
        ref = qa.ground_state(d.cdd, d.cgd, V).cpu().numpy()
        got = qa.ground_state_grid(d.cdd, d.cgd, sw).cpu().numpy()
        assert got.shape == (nx * ny, 4)
        assert np.array_equal(ref, got), (nx, ny)


@pytest.mark.parametrize("closed", [False, True])
def test_soft_charge_grid_equals_explicit(qa, closed):
    d = W.chain4(104, npix=45)
    kw = dict(closed=True, nhat=2) if closed else {}
    V = torch.as_tensor(d.V, device="cuda")
    nb_ref, saved_ref = qa.soft_charge(d.cdd, d.cgd, V, 0.01, **kw)
    nb, saved = qa.soft_charge_grid(d.cdd, d.cgd, d.sweep, 0.01, **kw)
    assert np.array_equal(bits(nb_ref.cpu().numpy()), bits(nb.cpu().numpy()))


def test_backward_grid_equals_explicit(qa):
    """The adjoint over the sensor workload's sweep (8 dots, 9 gates, the
    other plungers held at their base voltages)."""
    a = W.adjoint_case(400, npix=60)
    cdd, cgd = a.cdd[:8, :8], a.cgd[:8, :]
    V = torch.as_tensor(a.V, device="cuda")
    gbar = torch.randn((a.V.shape[0], 8), dtype=torch.float64, device="cuda",
                       generator=torch.Generator(device="cuda").manual_seed(3))
    nb_ref, saved_ref = qa.soft_charge(cdd, cgd, V, a.kT)
    ref = qa.soft_charge_backward(cdd, cgd, V, a.kT, gbar, saved_ref)
    nb, saved = qa.soft_charge_grid(cdd, cgd, a.sweep, a.kT)
    got = qa.soft_charge_backward_grid(cdd, cgd, a.sweep, a.kT, gbar, saved)
    assert np.array_equal(bits(nb_ref.cpu().numpy()), bits(nb.cpu().numpy()))
    for r, g, name in zip(ref, got, ("C_dd", "C_gd", "V")):
        r, g = r.cpu().numpy(), g.cpu().numpy()
        rel = np.abs(r - g).max() / max(np.abs(r).max(), 1e-300)
        say("grad %s: max relative difference %.2e" % (name, rel))
        assert rel <= 1e-12


def test_batch_of_sweeps_equals_explicit(qa):
    """48 ragged diagrams (2..8 dots, open and closed, kT in [0, 0.02])."""
    ds = W.ragged_batch(48, npix=24, start=700)
    ref = qa.Batch(ds)
    ref.run()
    got = qa.Batch(ds, sweeps=True)
    st = got.run(stats=True)
    assert got.V is None and st["pixels"] == got.pixels
    assert torch.equal(ref.n, got.n)
    assert np.array_equal(bits(ref.nbar.cpu().numpy()), bits(got.nbar.cpu().numpy()))


def test_full_dataset_batch_of_sweeps(qa):
    """The dataset workload at its full shape (4096 diagrams x 64 x 64) as
    sweeps equals the explicit-voltage batch at every pixel."""
    ds = W.ragged_batch(4096, npix=64)
    ref = qa.Batch(ds)
    ref.run()
    ref.run()
    got = qa.Batch(ds, sweeps=True)
    got.run()
    got.run()
    torch.cuda.synchronize()
    say("full batch of sweeps: %d pixels" % got.pixels)
    assert torch.equal(ref.n, got.n)
    assert torch.equal(ref.nbar, got.nbar)
