"""gltrsv: GrowLocal-scheduled sparse lower-triangular solve on AMD MI355X.

Submodules:
  ``gen``      seeded synthetic inputs (no solver arithmetic);
  ``binding``  ctypes binding of the HIP library ``libgltrsv.so``;
  ``build``    builds the library for gfx950.

Importing the package does not load the HIP library; ``binding.load()`` does.
"""
__version__ = "0.1.0"
