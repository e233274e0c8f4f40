"""MI355X-native constant-capacitance-model ground-state path (arXiv 2404.04994).

The compute lives in ``libqarray.so`` (hand-written HIP for gfx950 behind a
C ABI, declared in ``include/qarray.h``).  ``paper_2404_04994_amd.qarray`` is the
thin Python binding; ``paper_2404_04994_amd.workloads`` draws seeded inputs.
The binding is imported lazily so that the input generators can be used
without loading the GPU library.
"""

__all__ = ["qarray", "workloads"]


def __getattr__(name):
    if name in ("qarray", "workloads"):
        import importlib
        return importlib.import_module(__name__ + "." + name)
    raise AttributeError(name)
