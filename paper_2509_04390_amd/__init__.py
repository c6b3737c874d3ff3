"""MI355X-native multichannel partitioned convolution (UPOLS / NUPC with a
frequency-domain delay line) behind the C ABI declared in include/rta.h.

``workloads`` holds the seeded input generators; ``rta`` is the ctypes
binding of librta.so (imported on demand: it fails loudly when the HIP
library has not been built).
"""
from . import workloads  # noqa: F401

__all__ = ["workloads"]
