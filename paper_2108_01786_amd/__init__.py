"""MI355X-native boundary-integral water-wave solver (velocity-potential and
vortex-sheet normal velocity, arXiv 2108.01786, Secs. 3-4).

The compute path is the HIP library ``libwwbi.so`` behind the C ABI declared
in ``include/wwbi.h``; ``wwbi`` is its ctypes binding and ``autograd`` wraps
the forward solve and its hand-written adjoint as a torch.autograd.Function.
Importing the binding requires the built library; there is no fallback.
"""
__all__ = ["wwbi", "autograd", "build"]
