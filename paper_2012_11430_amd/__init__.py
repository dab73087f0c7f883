"""MI355X (gfx950) hot path of the multivariate matrix-pencil Prony method.

Layout:
  include/prony.h          C ABI (repository root)
  csrc/*.hip               HIP kernels and the ABI implementation (libprony.so)
  _lib.py                  ctypes loader of libprony.so
  api.py                   torch-tensor binding (samples, build_T, build_S, coeffs)
  host.py                  FP64 host steps assigned to the CPU by the paper
                           (reduced SVD, eigendecomposition of C_mu, LS solve)
  build.py                 hipcc build of libprony.so
"""
from . import _lib  # noqa: F401

__all__ = ["api", "host", "build"]
