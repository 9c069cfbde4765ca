"""MI355X-native (gfx950) engine for leading-order squared matrix elements.

The compute path is the C ABI in ``include/me.h`` backed by hand-written HIP
kernels in ``libme_mi355x.so``; ``binding`` marshals arguments to it and
``engine`` adds a small PyTorch convenience layer (device memory and streams
only).  Importing the package does not load the library.
"""
__all__ = ["binding", "engine", "inputs"]
