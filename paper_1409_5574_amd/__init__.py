"""MI355X (gfx950) implementation of the real-time synchrotron photon emission
method of Wallin, Gonoskov & Marklund (arXiv 1409.5574).

The emission path runs in hand-written HIP kernels inside ``libsr.so`` behind
the C ABI declared in ``include/sr.h``; ``api`` marshals torch tensors into it.
Importing the package does not load the library; ``api`` does, and fails
loudly when it is missing.
"""
