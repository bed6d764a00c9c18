"""MI355X (gfx950) Wilson-Dirac library: HIP kernels behind a C ABI
(include/wdirac.h), with a thin ctypes binding in ``wdirac``.

Importing the package does not load the shared library; ``from
paper_0810_5365_amd import wdirac`` does, and raises if it is not built.
"""
