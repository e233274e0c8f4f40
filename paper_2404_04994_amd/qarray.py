"""Thin Python binding of libqarray.so (C ABI in include/qarray.h).

Argument marshalling only: every step of the ground-state path runs in the
HIP kernels of the library.  torch supplies device memory and streams.  The
binding fails loudly (``QArrayError``) when the library or a GPU is missing;
there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqarray.so")

QA_OPEN, QA_CLOSED = 0, 1
PRECISION = {"fp64": 0, "fp32": 1, "bf16x3": 2, "bf16x2": 3}
STATUS = {0: "QA_OK", 1: "QA_E_NULL", 2: "QA_E_SHAPE", 3: "QA_E_NOT_SYMMETRIC", 4: "QA_E_NOT_PD",
          5: "QA_E_RANGE", 6: "QA_E_UNSUPPORTED", 7: "QA_E_WORKSPACE", 8: "QA_E_DEVICE"}
EXPORTS = ("qa_ground_state", "qa_ground_state_noalloc", "qa_ground_state_grid",
           "qa_soft_charge_grid", "qa_soft_charge_backward_grid", "qa_ground_state_batched_grid",
           "qa_continuous_min", "qa_soft_charge", "qa_soft_charge_backward", "qa_saved_bytes",
           "qa_ground_state_batched", "qa_last_error", "qa_release", "qa_version",
           "qa_timing_enable", "qa_timing_reset", "qa_timing_sum", "qa_graphs_enable",
           "qa_time_kernels")


class QArrayError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s: %s" % (STATUS.get(status, status), msg))
        self.status = status


class Problem(C.Structure):
    _fields_ = [("n_dot", C.c_int32), ("n_gate", C.c_int32),
                ("cdd", C.POINTER(C.c_double)), ("cgd", C.POINTER(C.c_double)),
                ("mode", C.c_int32), ("n_charge", C.c_int32),
                ("kT", C.c_double), ("threshold", C.c_double),
                ("precision", C.c_int32), ("flags", C.c_int32)]


FLAG_EXHAUSTIVE = 1


class Grid(C.Structure):
    """qa_grid: V(i, j) = (v0 + a_i e1) + b_j e2, a = linspace(a0, a1, nx),
    b = linspace(b0, b1, ny), pixel p = j * nx + i."""
    _fields_ = [("v0", C.POINTER(C.c_double)), ("e1", C.POINTER(C.c_double)),
                ("e2", C.POINTER(C.c_double)), ("a0", C.c_double), ("a1", C.c_double),
                ("b0", C.c_double), ("b1", C.c_double), ("nx", C.c_int32), ("ny", C.c_int32)]


def make_grid(sweep):
    """Grid struct from a sweep description (dict with v0, e1, e2, a0, a1, nx,
    b0, b1, ny) plus the host arrays it points into (keep both alive)."""
    arrs = tuple(np.ascontiguousarray(_host(sweep[k]), np.float64).ravel()
                 for k in ("v0", "e1", "e2"))
    dp = C.POINTER(C.c_double)
    g = Grid(arrs[0].ctypes.data_as(dp), arrs[1].ctypes.data_as(dp), arrs[2].ctypes.data_as(dp),
             float(sweep["a0"]), float(sweep["a1"]), float(sweep["b0"]), float(sweep["b1"]),
             int(sweep["nx"]), int(sweep["ny"]))
    return g, arrs


class Stats(C.Structure):
    _fields_ = [(name, C.c_int64) for name in
                ("pixels", "qp_pixels", "qp_failures", "doubled_pixels", "near_tie_pixels",
                 "fp64_gap_below_1e9", "candidates", "scored")]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


_lib = None


def load():
    """Load libqarray.so (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise QArrayError(6, "libqarray.so not built (run paper_2404_04994_amd.build)")
        lib = C.CDLL(LIB_PATH)
        vp, pb, st = C.c_void_p, C.POINTER(Problem), C.POINTER(Stats)
        i64p = C.POINTER(C.c_int64)
        lib.qa_ground_state.argtypes = [pb, vp, C.c_int64, vp, st, vp]
        lib.qa_ground_state_noalloc.argtypes = [pb, vp, C.c_int64, vp, vp]
        gp = C.POINTER(Grid)
        lib.qa_ground_state_grid.argtypes = [pb, gp, vp, st, vp]
        lib.qa_soft_charge_grid.argtypes = [pb, gp, vp, vp, st, vp]
        lib.qa_soft_charge_backward_grid.argtypes = [pb, gp, vp, vp, vp, vp, vp, vp]
        lib.qa_ground_state_batched_grid.argtypes = [pb, C.c_int32, gp, i64p, vp, vp, st, vp]
        lib.qa_soft_charge.argtypes = [pb, vp, C.c_int64, vp, vp, st, vp]
        lib.qa_continuous_min.argtypes = [pb, vp, C.c_int64, vp, vp, st, vp]
        lib.qa_soft_charge_backward.argtypes = [pb, vp, C.c_int64, vp, vp, vp, vp, vp, vp]
        lib.qa_ground_state_batched.argtypes = [pb, C.c_int32, vp, i64p, i64p, i64p, vp, vp, st, vp]
        lib.qa_saved_bytes.argtypes = [C.c_int64, C.c_int32]
        lib.qa_saved_bytes.restype = C.c_size_t
        lib.qa_last_error.restype = C.c_char_p
        lib.qa_version.restype = C.c_char_p
        lib.qa_release.argtypes = [vp]
        lib.qa_timing_enable.argtypes = [C.c_int]
        lib.qa_graphs_enable.argtypes = [C.c_int]
        lib.qa_timing_reset.argtypes = [vp]
        lib.qa_timing_sum.argtypes = [vp, C.POINTER(C.c_double), i64p]
        lib.qa_timing_sum.restype = C.c_int
        lib.qa_time_kernels.argtypes = [pb, vp, C.c_int64, vp, C.c_int32, C.POINTER(C.c_double), vp]
        lib.qa_time_kernels.restype = C.c_int
        lib.qa_sensor_response.argtypes = [pb, C.POINTER(Sensor), vp, C.c_int64, vp, vp, vp, vp, vp]
        lib.qa_sensor_response.restype = C.c_int
        lib.qa_sensor_noise_len.argtypes = [C.c_int64, C.c_int32, C.c_int32]
        lib.qa_sensor_noise_len.restype = C.c_size_t
        lib.qa_optimal_gate_voltages.argtypes = [pb, vp, vp]
        lib.qa_optimal_gate_voltages.restype = C.c_int
        lib.qa_virtual_gate_matrix.argtypes = [pb, vp]
        lib.qa_virtual_gate_matrix.restype = C.c_int
        for f in ("qa_ground_state_grid", "qa_soft_charge_grid", "qa_soft_charge_backward_grid",
                  "qa_ground_state_batched_grid"):
            getattr(lib, f).restype = C.c_int
        for f in ("qa_ground_state", "qa_ground_state_noalloc", "qa_continuous_min", "qa_soft_charge", "qa_soft_charge_backward",
                  "qa_ground_state_batched"):
            getattr(lib, f).restype = C.c_int
        _lib = lib
    return _lib


def _check(status: int):
    if status != 0:
        raise QArrayError(status, load().qa_last_error().decode())


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _host(m):
    if isinstance(m, torch.Tensor):
        m = m.detach().cpu().numpy()
    return np.ascontiguousarray(m, dtype=np.float64)


def make_problem(cdd, cgd, closed=False, nhat=0, kT=0.0, t=1.0, precision="fp64", flags=0):
    """Problem struct plus the host arrays it points into (keep both alive)."""
    cdd, cgd = _host(cdd), _host(cgd)
    if cdd.ndim != 2 or cgd.ndim != 2 or cdd.shape[0] != cdd.shape[1] or cgd.shape[0] != cdd.shape[0]:
        raise QArrayError(2, "cdd must be N x N and cgd N x G")
    prec = PRECISION[precision] if isinstance(precision, str) else int(precision)
    pb = Problem(cdd.shape[0], cgd.shape[1], cdd.ctypes.data_as(C.POINTER(C.c_double)),
                 cgd.ctypes.data_as(C.POINTER(C.c_double)), QA_CLOSED if closed else QA_OPEN,
                 int(nhat), float(kT), float(t), prec, int(flags))
    return pb, (cdd, cgd)


def _device_V(V, n_gate):
    if not isinstance(V, torch.Tensor):
        V = torch.as_tensor(np.asarray(V, np.float64))
    if not V.is_cuda:
        V = V.cuda()
    V = V.to(torch.float64).contiguous().view(-1, n_gate)
    return V


def ground_state(cdd, cgd, V, closed=False, nhat=0, t=1.0, precision="fp64", stream=None,
                 stats=False, out=None, exhaustive=False):
    """T = 0 ground state of every pixel (Eq. argmin); int32 tensor (P, N) on the GPU.
    With stats=True returns (n, stats_dict) and waits for the stream.
    exhaustive=True makes the matrix-core scorer compute every energy of the
    dense box instead of searching it in bound order (same result)."""
    lib = load()
    pb, keep = make_problem(cdd, cgd, closed, nhat, 0.0, t, precision,
                            FLAG_EXHAUSTIVE if exhaustive else 0)
    V = _device_V(V, pb.n_gate)
    P = V.shape[0]
    if out is None:
        out = torch.empty((P, pb.n_dot), dtype=torch.int32, device=V.device)
    st = Stats() if stats else None
    _check(lib.qa_ground_state(C.byref(pb), C.c_void_p(V.data_ptr()), P,
                               C.c_void_p(out.data_ptr()), C.byref(st) if st else None,
                               _stream(stream)))
    del keep
    return (out, st.as_dict()) if stats else out


def ground_state_grid(cdd, cgd, sweep, closed=False, nhat=0, t=1.0, precision="fp64",
                      stream=None, stats=False, exhaustive=False, device="cuda"):
    """qa_ground_state_grid: the ground state of every pixel of a sweep
    (int32 (nx * ny, N) on the GPU; the voltages are formed in the kernel)."""
    lib = load()
    pb, keep = make_problem(cdd, cgd, closed, nhat, 0.0, t, precision,
                            FLAG_EXHAUSTIVE if exhaustive else 0)
    g, gkeep = make_grid(sweep)
    out = torch.empty((g.nx * g.ny, pb.n_dot), dtype=torch.int32, device=device)
    st = Stats() if stats else None
    _check(lib.qa_ground_state_grid(C.byref(pb), C.byref(g), C.c_void_p(out.data_ptr()),
                                    C.byref(st) if st else None, _stream(stream)))
    del keep, gkeep
    return (out, st.as_dict()) if stats else out


def soft_charge_grid(cdd, cgd, sweep, kT, closed=False, nhat=0, t=1.0, stream=None,
                     device="cuda"):
    """qa_soft_charge_grid: (nbar float64 (P, N), saved buffer)."""
    lib = load()
    pb, keep = make_problem(cdd, cgd, closed, nhat, kT, t, "fp64")
    g, gkeep = make_grid(sweep)
    P = g.nx * g.ny
    nbar = torch.empty((P, pb.n_dot), dtype=torch.float64, device=device)
    saved = torch.empty(max(saved_bytes(P, pb.n_dot), 1), dtype=torch.uint8, device=device)
    _check(lib.qa_soft_charge_grid(C.byref(pb), C.byref(g), C.c_void_p(nbar.data_ptr()),
                                   C.c_void_p(saved.data_ptr()), None, _stream(stream)))
    del keep, gkeep
    return nbar, saved


def soft_charge_backward_grid(cdd, cgd, sweep, kT, grad_nbar, saved, closed=False, nhat=0,
                              t=1.0, want_V=True, stream=None):
    """qa_soft_charge_backward_grid: (dL/dC_dd, dL/dC_gd, dL/dV or None)."""
    lib = load()
    pb, keep = make_problem(cdd, cgd, closed, nhat, kT, t, "fp64")
    g, gkeep = make_grid(sweep)
    P = g.nx * g.ny
    gb = grad_nbar.to(torch.float64).contiguous()
    dev = gb.device
    dC = torch.empty((pb.n_dot, pb.n_dot), dtype=torch.float64, device=dev)
    dG = torch.empty((pb.n_dot, pb.n_gate), dtype=torch.float64, device=dev)
    dV = torch.empty((P, pb.n_gate), dtype=torch.float64, device=dev) if want_V else None
    _check(lib.qa_soft_charge_backward_grid(
        C.byref(pb), C.byref(g), C.c_void_p(gb.data_ptr()), C.c_void_p(saved.data_ptr()),
        C.c_void_p(dC.data_ptr()), C.c_void_p(dG.data_ptr()),
        C.c_void_p(dV.data_ptr()) if dV is not None else None, _stream(stream)))
    del keep, gkeep
    return dC, dG, dV


NOALLOC_MAX_PIXELS = 65536


def ground_state_noalloc(cdd, cgd, V, out, closed=False, nhat=0, t=1.0, precision="fp64",
                         stream=None, exhaustive=False):
    """qa_ground_state_noalloc: the ground state into the caller's int32 (P, N)
    tensor `out`, with the library's static device scratch (P <= 65536; calls
    on one GPU must not overlap)."""
    lib = load()
    pb, keep = make_problem(cdd, cgd, closed, nhat, 0.0, t, precision,
                            FLAG_EXHAUSTIVE if exhaustive else 0)
    V = _device_V(V, pb.n_gate)
    P = V.shape[0]
    if (out.dtype != torch.int32 or not out.is_contiguous() or out.device != V.device
            or tuple(out.shape) != (P, pb.n_dot)):
        raise QArrayError(2, "out must be a contiguous int32 (P, N) tensor on V's device")
    _check(lib.qa_ground_state_noalloc(C.byref(pb), C.c_void_p(V.data_ptr()), P,
                                       C.c_void_p(out.data_ptr()), _stream(stream)))
    del keep
    return out


def continuous_min(cdd, cgd, V, closed=False, nhat=0, stream=None, stats=False):
    """x* of every pixel (Sec. 3.1): (x FP64 (P, N), flags int32 (P,)[, stats])."""
    lib = load()
    pb, keep = make_problem(cdd, cgd, closed, nhat, 0.0, 1.0, "fp64")
    V = _device_V(V, pb.n_gate)
    P = V.shape[0]
    x = torch.empty((P, pb.n_dot), dtype=torch.float64, device=V.device)
    fl = torch.empty(max(P, 1), dtype=torch.int32, device=V.device)
    st = Stats() if stats else None
    _check(lib.qa_continuous_min(C.byref(pb), C.c_void_p(V.data_ptr()), P, C.c_void_p(x.data_ptr()),
                                 C.c_void_p(fl.data_ptr()), C.byref(st) if st else None,
                                 _stream(stream)))
    del keep
    return (x, fl[:P], st.as_dict()) if stats else (x, fl[:P])


def saved_bytes(P: int, n_dot: int) -> int:
    return int(load().qa_saved_bytes(P, n_dot))


def soft_charge(cdd, cgd, V, kT, closed=False, nhat=0, t=1.0, stream=None, stats=False):
    """Softargmin (Sec. 4.2) per pixel: (nbar float64 (P, N), saved uint8 buffer[, stats])."""
    lib = load()
    pb, keep = make_problem(cdd, cgd, closed, nhat, kT, t, "fp64")
    V = _device_V(V, pb.n_gate)
    P = V.shape[0]
    nbar = torch.empty((P, pb.n_dot), dtype=torch.float64, device=V.device)
    saved = torch.empty(max(saved_bytes(P, pb.n_dot), 1), dtype=torch.uint8, device=V.device)
    st = Stats() if stats else None
    _check(lib.qa_soft_charge(C.byref(pb), C.c_void_p(V.data_ptr()), P,
                              C.c_void_p(nbar.data_ptr()), C.c_void_p(saved.data_ptr()),
                              C.byref(st) if st else None, _stream(stream)))
    del keep
    return (nbar, saved, st.as_dict()) if stats else (nbar, saved)


def soft_charge_backward(cdd, cgd, V, kT, grad_nbar, saved, closed=False, nhat=0, t=1.0,
                         want_V=True, stream=None):
    """Adjoint of soft_charge: (dL/dC_dd, dL/dC_gd, dL/dV or None), FP64 device tensors."""
    lib = load()
    pb, keep = make_problem(cdd, cgd, closed, nhat, kT, t, "fp64")
    V = _device_V(V, pb.n_gate)
    P = V.shape[0]
    g = grad_nbar.to(torch.float64).contiguous()
    dC = torch.empty((pb.n_dot, pb.n_dot), dtype=torch.float64, device=V.device)
    dG = torch.empty((pb.n_dot, pb.n_gate), dtype=torch.float64, device=V.device)
    dV = torch.empty_like(V) if want_V else None
    _check(lib.qa_soft_charge_backward(C.byref(pb), C.c_void_p(V.data_ptr()), P,
                                       C.c_void_p(g.data_ptr()), C.c_void_p(saved.data_ptr()),
                                       C.c_void_p(dC.data_ptr()), C.c_void_p(dG.data_ptr()),
                                       C.c_void_p(dV.data_ptr()) if dV is not None else None,
                                       _stream(stream)))
    del keep
    return dC, dG, dV


class SoftCharge(torch.autograd.Function):
    """<n> = softargmin over the candidate set, differentiable in C_dd, C_gd and V.
    The backward recomputes candidate energies on the GPU (nothing but the
    per-pixel candidate set and normaliser is saved)."""

    @staticmethod
    def forward(ctx, cdd, cgd, V, kT, closed=False, nhat=0, t=1.0):
        # the library reads the matrices on the host: one copy of both (a
        # single device-to-host transfer when they live on the GPU), kept for
        # the backward
        n, g = cdd.shape[0], cgd.shape[1]
        if cdd.is_cuda or cgd.is_cuda:
            both = torch.cat([cdd.detach().reshape(-1), cgd.detach().reshape(-1).to(cdd.device)])
            both = both.to(torch.float64).cpu().numpy()
            cdd_h, cgd_h = both[:n * n].reshape(n, n), both[n * n:].reshape(n, g)
        else:
            cdd_h, cgd_h = _host(cdd), _host(cgd)
        nbar, saved = soft_charge(cdd_h, cgd_h, V, kT, closed, nhat, t)
        ctx.save_for_backward(V)
        ctx.host = (cdd_h, cgd_h)
        ctx.devs = (cdd.device, cdd.dtype, cgd.device, cgd.dtype)
        ctx.saved_buf = saved
        ctx.args = (float(kT), bool(closed), int(nhat), float(t))
        return nbar

    @staticmethod
    def backward(ctx, grad_nbar):
        (V,) = ctx.saved_tensors
        cdd_h, cgd_h = ctx.host
        cdev, cdt, gdev, gdt = ctx.devs
        kT, closed, nhat, t = ctx.args
        dC, dG, dV = soft_charge_backward(cdd_h, cgd_h, V, kT, grad_nbar, ctx.saved_buf, closed,
                                          nhat, t, want_V=ctx.needs_input_grad[2])
        dC = dC.to(cdev, cdt) if ctx.needs_input_grad[0] else None
        dG = dG.to(gdev, gdt) if ctx.needs_input_grad[1] else None
        dV = dV.to(V.device, V.dtype).view_as(V) if ctx.needs_input_grad[2] else None
        return dC, dG, dV, None, None, None, None


def soft_charge_autograd(cdd, cgd, V, kT, closed=False, nhat=0, t=1.0):
    return SoftCharge.apply(cdd, cgd, V, kT, closed, nhat, t)


class Batch:
    """A ragged batch of diagrams packed for qa_ground_state_batched: the
    problem array (host), the concatenated voltages (device) and the offsets.
    Outputs: n (int32) and nbar (FP64) flat device tensors; rows of diagram d
    start at out_offsets[d] elements."""

    def __init__(self, diagrams, device="cuda", sweeps=False):
        """sweeps=True: every diagram is passed as its sweep description
        (qa_ground_state_batched_grid; no voltages in device memory)."""
        self.diagrams = list(diagrams)
        nd = len(self.diagrams)
        self.problems = (Problem * nd)()
        self._keep = []
        self.grids = (Grid * nd)() if sweeps else None
        v_off, p_cnt, o_off = [], [], []
        vo = oo = 0
        for i, d in enumerate(self.diagrams):
            pb, keep = make_problem(d.cdd, d.cgd, d.closed, d.nhat, d.kT, d.t, "fp64")
            self.problems[i] = pb
            self._keep.append(keep)
            if sweeps:
                self.grids[i], gkeep = make_grid(d.sweep)
                self._keep.append(gkeep)
            v_off.append(vo)
            p_cnt.append(d.P)
            o_off.append(oo)
            vo += d.P * d.n_gate
            oo += d.P * d.n_dot
        self.v_offsets = np.array(v_off, np.int64)
        self.pix_counts = np.array(p_cnt, np.int64)
        self.out_offsets = np.array(o_off, np.int64)
        self.V = None if sweeps else torch.as_tensor(
            np.concatenate([np.ascontiguousarray(d.V, np.float64).ravel() for d in self.diagrams]),
            device=device)
        self.n = torch.empty(max(oo, 1), dtype=torch.int32, device=device)
        self.nbar = torch.empty(max(oo, 1), dtype=torch.float64, device=device)
        self.pixels = int(self.pix_counts.sum())

    def run(self, with_nbar=True, stream=None, stats=False):
        lib = load()
        i64 = lambda a: a.ctypes.data_as(C.POINTER(C.c_int64))
        st = Stats() if stats else None
        nbar = C.c_void_p(self.nbar.data_ptr()) if with_nbar else None
        if self.grids is not None:
            _check(lib.qa_ground_state_batched_grid(
                self.problems, len(self.diagrams), self.grids, i64(self.out_offsets),
                C.c_void_p(self.n.data_ptr()), nbar, C.byref(st) if st else None,
                _stream(stream)))
        else:
            _check(lib.qa_ground_state_batched(
                self.problems, len(self.diagrams), C.c_void_p(self.V.data_ptr()),
                i64(self.v_offsets), i64(self.pix_counts), i64(self.out_offsets),
                C.c_void_p(self.n.data_ptr()), nbar, C.byref(st) if st else None,
                _stream(stream)))
        return st.as_dict() if stats else None

    def result(self, d):
        """(n, nbar) of diagram d as host arrays (P_d x N_d)."""
        dg = self.diagrams[d]
        o, k = int(self.out_offsets[d]), dg.P * dg.n_dot
        return (self.n[o:o + k].view(dg.P, dg.n_dot).cpu().numpy(),
                self.nbar[o:o + k].view(dg.P, dg.n_dot).cpu().numpy())


class Sensor(C.Structure):
    _fields_ = [("n_sensor", C.c_int32), ("shape", C.c_int32), ("gamma", C.c_double),
                ("white", C.c_double), ("pink", C.c_double), ("pink_octaves", C.c_int32),
                ("reserved", C.c_int32), ("jump", C.c_double), ("jump_rate", C.c_double)]


SENSOR_SHAPE = {"lorentzian": 0, "gaussian": 1}


def sensor_noise_len(P: int, n_sensor: int, pink_octaves: int = 0) -> int:
    return int(load().qa_sensor_noise_len(P, n_sensor, pink_octaves))


def sensor_noise(P, n_sensor, pink_octaves=0, generator=None, device="cuda"):
    """Draws in the layout qa_sensor_response reads: standard-normal white
    and octave draws, then uniform jump draws (torch's generator)."""
    n = sensor_noise_len(P, n_sensor, pink_octaves)
    buf = torch.randn(n, dtype=torch.float64, device=device, generator=generator)
    buf[n - P * n_sensor:] = torch.rand(P * n_sensor, dtype=torch.float64, device=device,
                                        generator=generator)
    return buf


def sensor_response(cdd, cgd, V, n_sensor, n_array=None, gamma=0.05, shape="lorentzian",
                    white=0.0, pink=0.0, pink_octaves=0, jump=0.0, jump_rate=0.0, noise=None,
                    stream=None):
    """Charge-sensor signal (P x n_sensor, FP64 on the GPU) of the whole
    system (the last n_sensor dots are sensors) given the array charges
    n_array (int32 ground states or FP64 soft charges, P x N_array)."""
    lib = load()
    pb, keep = make_problem(cdd, cgd)
    V = _device_V(V, pb.n_gate)
    P = V.shape[0]
    sp = Sensor(int(n_sensor), SENSOR_SHAPE[shape] if isinstance(shape, str) else int(shape),
                float(gamma), float(white), float(pink), int(pink_octaves), 0, float(jump),
                float(jump_rate))
    n_int = n_dbl = None
    if n_array is not None:
        n_array = torch.as_tensor(n_array).to(V.device).contiguous()
        if n_array.dtype == torch.int32:
            n_int = n_array
        else:
            n_dbl = n_array.to(torch.float64).contiguous()
    out = torch.empty((P, int(n_sensor)), dtype=torch.float64, device=V.device)
    if noise is not None:
        noise = torch.as_tensor(noise, dtype=torch.float64).to(V.device).contiguous()
    _check(lib.qa_sensor_response(
        C.byref(pb), C.byref(sp), C.c_void_p(V.data_ptr()), P,
        C.c_void_p(n_int.data_ptr()) if n_int is not None else None,
        C.c_void_p(n_dbl.data_ptr()) if n_dbl is not None else None,
        C.c_void_p(noise.data_ptr()) if noise is not None else None,
        C.c_void_p(out.data_ptr()), _stream(stream)))
    del keep
    return out


def optimal_gate_voltages(cdd, cgd, q):
    """Gate voltages minimising the free energy of charges q (host FP64)."""
    pb, keep = make_problem(cdd, cgd)
    qh = np.ascontiguousarray(np.asarray(q, np.float64).ravel())
    v = np.empty(pb.n_gate, np.float64)
    _check(load().qa_optimal_gate_voltages(C.byref(pb), C.c_void_p(qh.ctypes.data),
                                           C.c_void_p(v.ctypes.data)))
    del keep
    return v


def virtual_gate_matrix(cdd, cgd):
    """alpha = (C_dd^-1 C_gd)^+ (G x N, host FP64)."""
    pb, keep = make_problem(cdd, cgd)
    a = np.empty((pb.n_gate, pb.n_dot), np.float64)
    _check(load().qa_virtual_gate_matrix(C.byref(pb), C.c_void_p(a.ctypes.data)))
    del keep
    return a


def graphs_enable(on: bool = True):
    load().qa_graphs_enable(1 if on else 0)


def timing_enable(on: bool = True):
    load().qa_timing_enable(1 if on else 0)


def timing_reset(stream=None):
    load().qa_timing_reset(_stream(stream))


def timing_sum(stream=None):
    """(ms per stage [setup, scoring, re-score] summed since the reset, calls)."""
    ms = (C.c_double * 3)()
    calls = C.c_int64(0)
    _check(load().qa_timing_sum(_stream(stream), ms, C.byref(calls)))
    return [ms[0], ms[1], ms[2]], int(calls.value)


def time_kernels(cdd, cgd, V, out, reps, t=1.0, precision="fp64", exhaustive=False, stream=None):
    """qa_time_kernels: mean ms per launch of (the setup kernel, the scorer),
    each over `reps` back-to-back launches between HIP events on the stream;
    `out` (int32 (P, N)) receives the ground state."""
    pb, keep = make_problem(cdd, cgd, False, 0, 0.0, t, precision,
                            FLAG_EXHAUSTIVE if exhaustive else 0)
    V = _device_V(V, pb.n_gate)
    ms = (C.c_double * 2)()
    _check(load().qa_time_kernels(C.byref(pb), C.c_void_p(V.data_ptr()), V.shape[0],
                                  C.c_void_p(out.data_ptr()), int(reps), ms, _stream(stream)))
    del keep
    return ms[0], ms[1]


def release(stream=None):
    load().qa_release(_stream(stream))


def version() -> str:
    return load().qa_version().decode()
