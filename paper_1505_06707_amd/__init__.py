"""MI355X-native SO-FFT + ECS propagation and FFT-preconditioned COCG.

The compute path is the HIP library ``libsofft.so`` built from ``csrc/`` (C ABI
declared in ``include/sofft.h``).  ``sofft`` is its thin Python binding: it
marshals torch device tensors and streams and calls the library; nothing is
computed in Python.  ``workloads`` holds the seeded synthetic inputs.
"""
__all__ = ["sofft", "workloads", "build"]
