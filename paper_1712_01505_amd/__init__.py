"""MI355X-native Wilson-Dirac stencil and Krylov solvers (HIP, gfx950).

The compute path is the C-ABI library ``libwilson.so`` built from ``csrc/``;
``wilson`` is its thin ctypes binding and ``autograd`` the differentiable
solve.  ``inputs`` generates seeded synthetic lattice fields.  Submodules are
imported on demand so that input generation works without the library.
"""
__all__ = ["inputs", "wilson", "autograd"]
