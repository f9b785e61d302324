"""MI355X-native integer convex-hull preconditioner (arXiv 1505.00914).

The product is the HIP library ``libhullprep.so`` (C ABI in
``include/hullprep.h``); this package is its thin Python binding plus the
seeded input generators and the serving loop.
"""
