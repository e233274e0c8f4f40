"""The sweep descriptions of the synthetic workloads (qa_grid's v0, e1, e2
and the two linspace ranges) reproduce the explicit voltages bitwise, so the
GPU's sweep entry points can be compared with its explicit-voltage ones on
identical inputs.  Also the linspace construction the kernels replay: point
i is i * step + start, the last point the end itself."""
import numpy as np
import pytest

from paper_2404_04994_amd import workloads as W


@pytest.mark.parametrize("make", [
    lambda: W.double_dot(0), lambda: W.double_dot(3, npix=41), lambda: W.chain4(100),
    lambda: W.chain4(101, npix=37), lambda: W.grid4x4(200), lambda: W.grid4x4(207, npix=77),
    lambda: W.ragged_diagram(5), lambda: W.ragged_diagram(11, npix=24),
    lambda: W.adjoint_case(400, npix=20),
])
def test_sweep_reproduces_voltages(make):
    d = make()
    V = W.sweep_voltages(d.sweep)
    assert V.shape == np.asarray(d.V).shape
    assert np.array_equal(V.view(np.int64), np.ascontiguousarray(d.V).view(np.int64))


@pytest.mark.parametrize("lo,hi,num", [(-2.0, 8.0, 100), (-3.0, 3.0, 64), (0.1, 0.7, 7),
                                       (5.0, -1.5, 13), (2.0, 2.0, 5), (-1.0, 4.0, 1),
                                       (-1.0, 4.0, 2)])
def test_linspace_points(lo, hi, num):
    """numpy's linspace as the kernels form it: FP64 i * ((hi - lo) / (num - 1))
    + lo, each operation rounded on its own, the last point hi (one point: lo)."""
    ref = np.linspace(lo, hi, num)
    step = (hi - lo) / (num - 1) if num > 1 else 0.0
    pts = [np.float64(i) * np.float64(step) + np.float64(lo) for i in range(num)]
    if num > 1:
        pts[-1] = hi
    assert np.array_equal(np.array(pts).view(np.int64), ref.view(np.int64))
