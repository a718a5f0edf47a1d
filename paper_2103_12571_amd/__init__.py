"""MI355X (gfx950) alpha-circulant preconditioned Richardson sweep.

The compute path lives in ``libaao.so`` (HIP kernels behind a C ABI declared
in ``include/aao.h``); ``binding`` wraps it with ctypes and uses PyTorch only
for device memory and streams.  Importing this package does not load the
library; ``binding.lib()`` does, and raises if it is missing.
"""
