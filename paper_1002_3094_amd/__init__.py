"""MI355X-native PCG for the axisymmetric variable-coefficient elliptic
operator with a separation-of-variables Laplace preconditioner
(Terekhov, arXiv:1002.3094).  The numerical path lives in the HIP library
``libaxipcg.so``; ``axipcg`` is its ctypes binding."""
from . import axipcg  # noqa: F401

__all__ = ["axipcg"]
