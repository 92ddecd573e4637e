"""MI355X (gfx950) supernodal selected inversion of non-symmetric sparse matrices.

The compute path is the HIP library ``libselinv.so`` behind the C ABI in
``include/selinv.h``; ``paper_1708_04539_amd.selinv`` is its ctypes binding.
Importing the package itself loads nothing, so that the build step can run
before the library exists.
"""
__all__ = ["selinv", "build"]
