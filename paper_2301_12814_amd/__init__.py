"""MI355X-native lossy Gaussian boson sampling MPO simulator (arXiv 2301.12814).

The product is the C-ABI HIP library ``libgbsmpo.so`` (sources in ``csrc/``,
declarations in ``include/gbs_mpo.h``) and its thin ctypes binding
``paper_2301_12814_amd.gbsmpo``.  ``inputs`` holds only the seeded synthetic
input generators.  Importing the package loads nothing.
"""
