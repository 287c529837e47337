"""MI355X-native Ewald-RPY Brownian dynamics (arXiv:1203.6208 hot path).

The compute path is the HIP C-ABI library ``librpy.so`` (see ``include/rpy.h``);
``paper_1203_6208_amd.rpy`` is its thin ctypes binding.  Importing this package
does not load the library; ``paper_1203_6208_amd.rpy`` does, and raises if it
has not been built.
"""
__all__ = ["inputs", "rpy"]
