"""MI355X (gfx950) tau-preconditioned GMRES for Riesz fractional NLS systems.

The compute path is the HIP library libfnls.so (built from csrc/), reached
through the C ABI declared in include/fnls.h; `fnls` is the thin ctypes
binding.  Importing this package loads nothing: the library is opened on the
first use of `paper_2410_03643_amd.fnls`.
"""
__all__ = ["fnls", "inputs"]
