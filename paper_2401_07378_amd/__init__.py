"""MI355X-native NNS-EMD (arXiv 2401.07378): hand-written HIP kernels for
gfx950 behind a small C ABI (include/nnsemd.h), with a thin ctypes binding.

Submodules:
  workloads  seeded synthetic inputs shaped like the paper's workloads
  binding    ctypes marshalling of libnnsemd.so (GPU only, no CPU path)
  build      hipcc build of libnnsemd.so
"""
__all__ = ["workloads", "binding", "build"]
