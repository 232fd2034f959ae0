"""CPU oracle for Hierarchical Affinity Propagation (HAP).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import this package.  The product path (the
HIP library and its Python binding) never imports, links or calls anything
here, and nothing here imports the product path.

Contents
  hap_ref     plain FP64 NumPy HAP, Algorithm 1 run level by level
  literal     pure-Python HAP evaluated from the defining sums of Eq. 2.1-2.6,
              generic over the number type (fractions.Fraction gives exact rationals)
  ap_ref      plain Affinity Propagation (Frey and Dueck, 2007), written separately
  brute       exhaustive exemplar-set search for tiny inputs
  similarity  FP64 similarity, tie-break noise, median preference, net similarity
  warm        learned warm start: per-point features, FP64 perceptron with backpropagation
              and Adam, warm initial availabilities, warm run with cold fallback
"""
