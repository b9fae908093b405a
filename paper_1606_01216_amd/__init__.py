"""MI355X (gfx950) library for the shifted SPAI-preconditioned CG solves of
AIRGA model reduction (arXiv 1606.01216).

The compute path is ``libairga.so`` (HIP kernels behind the C ABI in
``include/airga.h``); ``airga`` is its thin ctypes binding.  Importing this
package loads nothing; the library is loaded on first use.
"""
__all__ = ["airga"]
