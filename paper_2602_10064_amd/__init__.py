"""MI355X-native TACAW hot path: frame-resolved multislice over a trajectory,
frame-mean subtraction and the time transform to I(k, w).

The compute lives in the HIP library ``libtacaw.so`` (C ABI declared in
``include/tacaw.h``); ``paper_2602_10064_amd.tacaw`` is its thin ctypes
binding.  ``paper_2602_10064_amd.workloads`` synthesizes seeded inputs.
Importing the package does not load the library.
"""
__all__ = ["workloads", "tacaw"]
