"""MI355X (gfx950) sparse-pixel Gaussian rasterizer: error-guided sparse
training hot path of TurboGS (arXiv 2606.15924) as hand-written HIP kernels
behind a C ABI (``include/turbogs.h``, ``libturbogs.so``).

Modules:
  binding    ctypes binding with the C entry points' names
  pipeline   per-view buffers and the training-step driver
  autograd   torch.autograd.Function over the sparse forward/adjoint
  build      hipcc build of the library
"""
__all__ = ["binding", "pipeline", "autograd", "build"]
