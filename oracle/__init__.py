"""CPU oracle of DB-TSDF scan integration (test infrastructure only).

Only the test suite, the package smoke check and the benchmark's CPU-baseline
leg use this package. The GPU library never imports it, and it never imports
the GPU library.

- ``oracle.oracle``: ctypes front of the plain single-threaded C oracle
  (``dbtsdf_oracle.c``), which integrates scans step by step as Section III
  of the paper describes them.
- ``oracle.brute``: the closed-form definition of the integrated grid, in
  numpy, evaluated voxel by voxel on tiny grids (and on sampled voxels of big
  ones), used to pin the C oracle.
"""
