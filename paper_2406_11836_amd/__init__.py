"""MI355X-native partitioned 3D Gaussian splatting rasterizer (RetinaGS, arXiv 2406.11836).

The compute path is a C-ABI HIP library (``librgs.so``, declared in
``include/rgs.h``); ``_lib`` binds it with ctypes, ``raster`` drives one
forward/backward pass and wraps it in a ``torch.autograd.Function``, and
``serve`` is the continuous-batching render loop.  Importing the package does
not load the library; the first call that needs it does, and raises if it has
not been built.
"""
__all__ = ["scenes"]
