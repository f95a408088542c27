"""Plain FP64 CPU oracle for HPS leaf-level static condensation.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call,
link or execute anything in this package; only the test suite, the smoke
check and the CPU-baseline leg of the benchmark use it.  It shares no code
with the HIP path (no kernels, headers, tables, helpers or pre/post
processing); the only module both sides read is the seeded problem
definition in ``paper_2211_14969_amd.inputs``, which holds no solver
arithmetic.

What it computes, and where in the paper (arxiv 2211.14969) each step comes
from:

* ``cheb``      - the p x p tensor grid of Chebyshev points on a leaf and the
                  spectral differentiation matrix (Sec. 2, the description of
                  the HPS discretisation).
* ``leaf``      - the dense p^2 x p^2 leaf interaction matrix: the PDE
                  (eqs. (bvp), (var_helm), and the general operator with a
                  mixed term of Sec. 3.2, eq. (chain_rule)) collocated at
                  interior nodes and the outward normal derivative (flux) on
                  the leaf edges; with a mixed term the corner values come
                  from the edges' extrapolants (a reading);
                  static condensation of the interior nodes (Sec. 2, the
                  paragraph before eq. (hps_reduced)), done with a plain
                  LAPACK LU with partial pivoting and matrix products (the
                  leaf operations of Sec. 2, cost paragraph); and the
                  per-leaf recovery of interior values (Sec. 3, after
                  eq. (constant_coeff_helm)).
* ``mixed``     - leaves of different orders in one problem (Sec. 2: p from a
                  fixed set): edge unknowns at the lower order's nodes,
                  interpolation of traces and fluxes (a reading), the
                  reduced system, its solve and the full system;
* ``interface`` - the reduced system on the leaf edges (eq. (hps_reduced)),
                  its sparse direct solve (Sec. 3.1: SciPy SuperLU with the
                  COLAMD ordering), the full unreduced collocation system for
                  brute-force checks, and the error measures of
                  eq. (accuracy_formula).

Every floating-point step is IEEE binary64.  Parity pins: each function is
pinned by the CPU tests in ``tests/test_oracle_*.py`` against closed forms,
exact solutions, brute force and the spectral convergence rate; none is
"parity unpinned".
"""
