"""MI355X-native inexact GMRES policy iteration (arXiv:2211.04299).

The compute path is a HIP library (``libigmres.so``, C-ABI in
``include/igmres.h``); ``paper_2211_04299_amd.igmres`` is its thin ctypes
binding.  Importing this package does not load the library; the binding does,
and raises if it is missing.
"""
__all__ = ["synth"]
