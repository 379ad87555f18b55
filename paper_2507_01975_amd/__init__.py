"""MI355X (gfx950) implementation of the learnable-differentiable finite-volume
solver's hot path.  The numerical work runs in libldsv.so (HIP); ``ldsv`` is
its ctypes binding and ``autograd`` wraps the forward and adjoint entry points
as torch.autograd.Functions."""
