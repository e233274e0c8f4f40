"""FP64 CPU oracle for the constant-capacitance ground-state path.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke``
and by the ``cpu_baseline`` leg of ``bench.py``.  The HIP product library never
imports, links or calls anything in this directory.
"""
from .qa_oracle import *  # noqa: F401,F403
