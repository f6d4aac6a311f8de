"""MI355X-native overlap-save coherent dedispersion (De & Gupta's method).

The computation runs in libcdd.so (hand-written HIP for gfx950) behind the C
ABI declared in include/cdd.h; this package is its Python binding.
"""
from ._binding import (CDD_CF32, autotune, CDD_CI8, PHASE_FP32, PHASE_FP64_REDUCED,  # noqa: F401
                       CddError, LIB_PATH, Plan, Server, dedisperse, dedisperse_noalloc, fold, fullband,
                       fullband_query, gsb_inverse, incoherent, lib, profile_enable,
                       profile_read, query)

__all__ = ["dedisperse", "dedisperse_noalloc", "incoherent", "fold", "gsb_inverse", "fullband", "fullband_query",
           "autotune", "query", "Plan", "Server", "CddError",
           "CDD_CI8", "CDD_CF32",
           "PHASE_FP64_REDUCED", "PHASE_FP32", "lib", "LIB_PATH", "profile_enable",
           "profile_read"]
