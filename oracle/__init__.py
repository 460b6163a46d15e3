"""Plain FP64 CPU oracle for the batched tensor-product operators.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code, table or
helper with the HIP library in ``paper_2609_04534_amd/``.

What it computes (paper: "Adaptive Multilevel Discontinuous Galerkin Methods
on GPUs", arXiv 2609.04534):

* ``basis``  -- the 1D Gauss-Lobatto Lagrange basis on [0, 1], its exact mass
  and stiffness matrices, and the SIPG face-coupling blocks of
  eq. (face_coupling), Sec. 3.
* ``dense``  -- the per-block operators written out as dense Kronecker
  matrices: the volume operator of eq. (eval_pipeline), Sec. 3.1, and the
  cell block of eq. (cell_block), Sec. 5.2, with apply = dense mat-vec and
  inverse = dense LAPACK solve refined with a long-double residual.
* ``sipg``   -- the coupled SIPG operator of eq. (sipg) on a uniform
  Cartesian box mesh with Nitsche (homogeneous Dirichlet) boundary faces,
  A = A^vol + A^face of eq. (operator_split), assembled as a sparse matrix
  from dense cell-row blocks built from the bilinear form.
* ``hermite`` -- the Hermite-type 1D basis of Sec. 3.1 (eq. (hermite_conditions))
  with its mass and stiffness matrices, endpoint data, change of basis to the
  Lagrange basis and level transfers; ``sipg`` and ``mg`` take the basis as a
  parameter (``bname``).
* ``patch``  -- vertex-patch blocks: the operator of the 2 x 2 x 2 cells
  around a vertex as one tensor-product block of 2(p+1) points per
  direction (1D patch factors from the cell block and the coupling blocks).
* ``mg``     -- geometric multigrid for it: Chebyshev-accelerated
  block-Jacobi smoothing (eq. (chebyshev_weights), eq. (chebyshev_richardson)),
  polynomial-embedding transfers, a dense coarse solve, CG preconditioned by
  one V-cycle.

The oracle never uses sum factorization or fast diagonalization: those are
the method under test.  Every function cites the passage it follows.

Pins (tests/test_oracle_pins.py) tie every function to closed forms,
textbook values, printed stencils and brute-force quadrature; see the header
of each module for what pins it.
"""
