"""CPU oracle for the matrix-free Q_p Laplacian: TEST INFRASTRUCTURE ONLY.

This package is a plain, slow, obviously-correct FP64 implementation of what the
GPU path computes.  It exists to check the GPU path, and only the test suite
(``tests/``), ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import it.  The product path (``paper_1910_13247_amd``) never
imports, links or executes anything here, and nothing here imports the product
path: the two share no code.  Random inputs come from ``synthetic`` and are
passed in as arrays.

What it computes (section numbers refer to the deal.II paper, arXiv 1910.13247):

* the weak Laplacian of eq. (1), generalised to a variable coefficient
  a(x) * grad u . grad v, integrated cell by cell with shape-function gradients
  and JxW at quadrature points, exactly as the step-4 cell loop of Sec. 2.4
  describes (``element.py``, ``assemble.py``);
* the global sparse matrix built from those cell matrices, Dirichlet rows, and
  its action on a vector (Sec. 3.6 states that the matrix-free operator is
  the action of exactly this operator) (``assemble.py``, ``ebe.py``);
* the right-hand side l(v) = int f v dx of the same cell loop (``rhs.py``);
* conjugate gradients and direct solves (``solve.py``);
* the pieces of the geometric multigrid of Sec. 3.5 / Sec. 6.1: level
  transfer by interpolation between nested meshes, Jacobi diagonal, Chebyshev
  smoothing, V-cycle (``gmg.py``);
* the symmetric interior penalty DG discretisation of the Laplacian used in the
  paper's multigrid experiment (Sec. 6.1): cell and face matrices, assembly, the
  action on sampled rows (``dg.py``).

Readings of points the paper leaves open (node family, quadrature rule,
geometry, Dirichlet treatment, numbering, Chebyshev constants) are fixed in
each module's docstring.

Parity status: every function is pinned by the ``-m "not gpu"`` tests in
``tests/test_oracle_*.py`` against closed forms, invariants, independent
constructions or brute force, except where a docstring says "parity unpinned".
"""
