"""HOTRG coarse-graining step and its reverse-mode adjoint on AMD Instinct MI355X (gfx950).

Submodules (imported on demand, so that importing the package loads nothing):
  inputs    seeded synthetic input tensors (Ising model, symmetrised random tensors)
  binding   ctypes binding of libdtrg.so (the C ABI in include/dtrg.h)
  autograd  torch.autograd.Function wrapper
  build     hipcc build of libdtrg.so for gfx950
"""

__all__ = ["inputs", "binding", "autograd", "build"]
