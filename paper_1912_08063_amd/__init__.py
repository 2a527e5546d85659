"""MI355X-native hot path of acoustic full-waveform inversion.

Forward modelling, adjoint propagation and the velocity gradient of the
constant-density acoustic wave equation (Huot et al., "High-resolution imaging
on TPUs", Eqs. 1-3), as hand-written HIP kernels for gfx950 behind a C ABI
(``include/fwi.h``, ``libfwi.so``).  Python here only marshals arguments:
torch supplies device memory and streams.

Submodules (imported lazily so that ``workloads`` works without torch):
    _lib       ctypes binding of libfwi.so (same entry-point names)
    api        forward() / gradient() on torch tensors
    autograd   FWIForward, a torch.autograd.Function with checkpointed backward
    serve      continuous-batching request server
    workloads  seeded synthetic inputs (no wave arithmetic)
"""
__all__ = ["api", "autograd", "serve", "workloads"]
