"""DartMinHash (arXiv 2005.11547) for AMD Instinct MI355X: HIP kernels behind a
C ABI (include/dms.h) and a thin ctypes binding (``dms``)."""
from . import dms  # noqa: F401
from .dms import (Context, DMSError, LshIndex, Server, SketchDB, SketchInfo, lib, spec_constants,  # noqa: F401
                  spec_tabulation, t_of_k, to_device)
