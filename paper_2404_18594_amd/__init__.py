"""MI355X-native hot path of the cluster discrete truncated Wigner
approximation (C-dTWA, Nagao & Yunoki, arXiv:2404.18594).

The computation runs in the HIP library ``libcdtwa.so`` (C ABI in
``include/cdtwa.h``); this package holds its ctypes binding and a quench
driver.  Build the library with ``python paper_2404_18594_amd/build.py``.
"""
from .binding import (EXPORTS, F32, F64, LIB_PATH, NOBS, OBS_NAMES, CdtwaError, Plan, Problem,  # noqa: F401
                      library)
from .driver import estimates, run_quench  # noqa: F401
