"""MI355X-native hot path of the cluster discrete truncated Wigner
approximation (C-dTWA, Nagao & Yunoki, arXiv:2404.18594).

The computation runs in the HIP library ``libcdtwa.so`` (C ABI in
``include/cdtwa.h``); this package holds its ctypes binding and a quench
driver.  Build the library with ``python paper_2404_18594_amd/build.py``.
"""
from .binding import (EXPORTS, F32, F64, LAYOUT_FULL, LAYOUT_PACKED, LIB_PATH, MLP_IN, MLP_OUT,  # noqa: F401
                      MLP_PARAMS, MLP_WBF16, NOBS, PACKED_ELEMS, PACKED_TILE,
                      OBS_NAMES, Batch, CdtwaError, Mlp, Plan, Problem, cv_workspace_bytes, library,
                      new_cv_workspace)
from .driver import estimates, run_quench  # noqa: F401
