"""xkp: cross-matrix Krylov projection on MI355X (gfx950).

The solver is the HIP library libxkp.so (C ABI in include/xkp.h); `xkp` is its ctypes binding and
`driver` chains the calls over timesteps.  Importing this package loads nothing native; the
binding loads the library on first use and raises if it is missing.
"""
__all__ = ["xkp", "driver", "build"]
