"""MI355X-native (gfx950) p-Laplacian hot path of p-spectral clustering on the Grassmann manifold.

The compute path is the HIP library ``libpspec.so`` (C ABI declared in ``include/pspec.h``);
``paper_2605_26975_amd.pspec`` is its thin ctypes binding.  Importing this package loads
nothing; the binding loads the library on first use and raises if it is missing.
"""
