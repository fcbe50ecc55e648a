"""CPU oracle for replica-exchange Wang-Landau -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg import
this package.  ``oracle.core`` wraps the plain C oracle (rewl_oracle.c);
``oracle.exact`` holds the exact densities of states it is pinned against.
Nothing here imports the GPU package, and the GPU package never imports this.
"""
