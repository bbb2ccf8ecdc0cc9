"""MI355X-native randomized high-order t-SVT (HIP kernels behind a C ABI).

The compute path lives in libhtsvt.so (built by `build.py`); `htsvt` is the thin
ctypes binding.  Importing `paper_2506_09594_amd.htsvt` fails if the library
has not been built.
"""
__all__ = ["htsvt", "build"]
