"""MI355X-native decomposed-kernel (Mercer) Gaussian process.

The compute lives in the HIP library ``libmercergp.so`` (C ABI declared in
``include/gp.h``); ``binding`` wraps it with ctypes.  ``workloads`` holds the
seeded synthetic inputs.  Importing the package does not load the library.
"""

__all__ = ["binding", "workloads"]
