"""CPU FP64 oracle for the multidimensional butterfly factorization.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only the test-suite, the smoke check and the CPU
baseline leg of the benchmark use it.  It shares no code with the GPU
library; both sides receive the same seeded inputs (``mbf_workloads``) and
compute everything else independently.

Contents (Li, Yang, Ying, "Multidimensional Butterfly Factorization"):

* ``kernels``  -- kernel entries: 2D DFT and the generalized Radon FIO of
  Example 1 (Section 3.3, eq. (example1phi)).
* ``direct``   -- the plain definition u = K g (Section 1.1, eq. (kernel)),
  by direct O(N^2) summation in FP64, and FFT closed forms.
* ``trees``    -- quadtrees with Z-order numbering (Section 2.2, Fig. 1),
  the polar map (Section 3.1, eq. (polar)) and the corona split
  (Section 4.1, eq. (domaindecomp)).
* ``lowrank``  -- truncated SVD and the three low-rank forms
  (Section 2.1, eq. (lowrank1)-(lowrank3)); SVD via random sampling.
* ``butterfly`` -- BF / PBF / MSBF build, apply and adjoint apply
  (Sections 2.3-2.5, 3.2, 4.2).

Every function's pins live in ``tests/test_oracle_*.py``.  Parity unpinned:
exact factor entries (several factorizations are correct: random samples,
SVD phase freedom, rank ties) -- only operator outputs are compared.
"""

from . import kernels, direct, trees, lowrank, butterfly  # noqa: F401
