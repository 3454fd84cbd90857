"""MI355X-native fast spectral collision operator for the multi-species
Boltzmann equation (DGFS), after arXiv:1903.04670.

The compute path is the HIP library ``libdgfs.so`` built from ``csrc/``;
``dgfs`` is its thin ctypes binding.  Importing this package does not load
the library; ``paper_1903_04670_amd.dgfs`` does, and raises if it is absent.
"""
