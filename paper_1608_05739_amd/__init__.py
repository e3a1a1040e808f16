"""MI355X-native PSATD field step (arXiv:1608.05739, Sec. III.B item 2).

The compute path is the HIP library ``libpsatd.so`` (C ABI in
``include/psatd.h``); this package is its Python binding.  There is no CPU
fallback: if the library is not built, loading it raises.
"""

from ._binding import (  # noqa: F401
    Domain,
    EXPORTED_SYMBOLS,
    Fdtd,
    LIBRARY_PATH,
    Patch,
    Plan,
    PsatdError,
    as_patch,
    describe_plan,
    load_library,
)
