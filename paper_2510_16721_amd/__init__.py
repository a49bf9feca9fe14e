"""MI355X (gfx950) cell-filter nudged elastic band: HIP kernels behind a C ABI.

The package holds the HIP sources (csrc/), their build script and a thin ctypes
binding (cfneb.py) of include/cfneb.h.  Nothing here falls back to CPU code: the
binding raises if libcfneb.so is missing.
"""
from . import cfneb  # noqa: F401
from .cfneb import Band, Params, FireState, CfnebError, default_params, band_bytes  # noqa: F401
