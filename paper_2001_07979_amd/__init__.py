"""MI355X-native multi-matrix syndrome belief propagation (MBP) decoder.

The decoder is the HIP library ``libmbp.so`` behind the C-ABI declared in
``include/mbp.h``; ``paper_2001_07979_amd.mbp`` is its Python binding.
Importing this package loads nothing native.
"""
__all__ = ["mbp", "inputs"]
