"""CPU FP64 oracle for the PSTT2 hot path -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
import this package.  The product path (the HIP library and its Python
binding) never calls it and shares no code with it.

Contents
  tt_sketch.py plain, slow PSTT2 / PSTT2-onepass / PSTT (paper Section 3.2), the
             Khatri-Rao sketches, CPQR bases, core formation, TT evaluation.
  tt_svd.py  sequential TT-SVD and Parallel-TTSVD (Sections 2.2 and 3.1), used as
             a second, deterministic reference.

Parity status of each function is listed in the header of its module.
"""
from .tt_sketch import *  # noqa: F401,F403
from .tt_svd import ttsvd, parallel_ttsvd  # noqa: F401
