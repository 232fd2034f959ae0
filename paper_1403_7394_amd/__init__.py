"""HAP on MI355X: a HIP library (libhap) for the Hierarchical Affinity Propagation sweep.

``paper_1403_7394_amd.hap`` is the ctypes binding of the C ABI declared in
``include/hap.h``; ``paper_1403_7394_amd.synth`` draws the seeded synthetic
inputs.  Importing the package loads nothing; the binding loads the shared
library on first use and raises if it has not been built.
"""
