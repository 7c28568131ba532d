"""MI355X-native hybrid MFMA / vector SpMM (C = A*B, A in CSR).

The compute path lives in ``libspmm.so`` (HIP for gfx950, behind the C ABI in
``include/spmm.h``); :mod:`paper_2606_22482_amd.api` is a thin ctypes binding
over it.  Importing the package does not load the library; the first call does,
and fails loudly when the library has not been built.
"""
__all__ = ["api", "synth"]
