"""FP64 CPU oracle for the FMM-accelerated Laplace-Beltrami hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only the tests, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
library (``paper_2111_10743_amd``) and imports nothing from it.

What it computes is the plain discrete definition of the method of Agarwal,
O'Neil & Rachh, "FMM-accelerated solvers for the Laplace-Beltrami problem on
complex surfaces in three dimensions" (arXiv 2111.10743):

* Section 4 (discretization): order-k curved triangular patches sampled at
  interpolation nodes, smooth weights, an oversampled far rule, Near/Far split,
  and locally corrected quadrature, eq. (nys-lcq2): the far part is the plain
  O(N * N_over) sum over the oversampled sources (no FMM), the near part the
  stored corrections.
* Section 3 / Section 4.3: the layer potentials S, grad S, S', S''+D' and the
  second-kind operator A3 of eq. (ie-dis2), applied right to left.
* Section 6 (numerical examples): un-restarted GMRES, at most 100 iterations,
  relative Euclidean residual stopping rule.

Pins (each tested against something other than this code) live in
``tests/test_oracle_*.py``.  Functions without such a pin say "parity unpinned"
in their docstring.
"""
