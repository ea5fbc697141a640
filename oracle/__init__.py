"""CPU oracle for the Satellite System Graph method (arXiv 1907.06146).

TEST INFRASTRUCTURE ONLY. This package is the plain, slow, obviously correct
reference that the GPU search is checked against: only the tests, the smoke
check and the CPU-baseline leg of the benchmark may import it. The product
path never calls it and shares no code with it.

Contents:
  core      ctypes wrapper over ``ssg_oracle.c`` (FP64): brute-force kNN and
            ground truth, NSSG indexing (Alg. 3), Alg. 1 search, exact SSG
            (Alg. 2).
  pyref     an independent pure-Python Alg. 1 and SSG pruning for tiny inputs.
  cache     writer of the graph cache files that tests and benchmarks load.
  build_cache  command-line script that builds the caches of each workload.

Parity status of each function is stated in its docstring. Every function
here has at least one pin in ``tests/test_oracle_*.py`` that does not reuse
its own code path.
"""
