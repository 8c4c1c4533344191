"""FP64 CPU oracle of the quasi-static PIC slice loop (HiPACE++,
arXiv:2109.10277).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by
``__graft_entry__.smoke()`` and by the ``cpu_baseline`` leg of ``bench.py``.
The product path (``paper_2109_10277_amd``) never imports it and shares no
code with it.

Parity pins: every function here is pinned by the ``-m "not gpu"`` tests in
``tests/test_oracle_*.py`` against closed forms, invariants, library
routines or brute force; none is "parity unpinned".
"""
from .qsp_oracle import *  # noqa: F401,F403
from . import qsp_oracle  # noqa: F401
