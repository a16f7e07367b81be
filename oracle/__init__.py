"""Plain FP64 CPU oracle for the ORAS-FGMRES Helmholtz path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product (the HIP library and its
Python binding) may import, call, link or execute anything in this package;
only the tests, the smoke check and the CPU-baseline leg of the benchmark use
it.  It shares no code with the HIP path: every formula here is written from
the paper (arXiv 2110.15113) and from the operator reading documented in each
module, in plain NumPy/SciPy, FP64, with no blocking or fusion beyond what the
definitions state.

Modules
  stencil_table  -- lambda-adaptive weight table (paper sec. 2.3, FDFD
                    discretisation; dispersion analysis)
  operator       -- discrete Helmholtz operator A (eq. 1 and eq. 1.1) with PML,
                    and the subdomain matrices B_j with Robin interfaces
                    (sec. 2.1, the ORAS definition)
  direct         -- the plain definition u = A^{-1} b by a block-tridiagonal
                    (z-plane) direct LU with LAPACK partial pivoting
  oras           -- overlapping cuboid partition, Boolean partition of unity,
                    M^{-1} = sum_j R_j^T D_j B_j^{-1} R_j with SuperLU local
                    factors (sec. 2.1, sec. 2.2)
  krylov         -- right-preconditioned flexible GMRES, CGS, complex Givens,
                    pseudo-block over columns (sec. 2.1, sec. 2.2 notes)
  adjoint        -- receiver sampling, adjoint solve and the gradient of a
                    least-squares misfit w.r.t. squared slowness (sec. 4 / FWI
                    motivation)
  metrics        -- the paper's gain-weighted l1 error Err (eq. eqerror)
  pivots         -- pivots of the plane Schur complements of a local matrix
                    without row exchanges, their ratio to the plane's largest
                    entry, and detection of a singular B_j (sec. 2.2)

Parity status of every function is stated in its module docstring.
"""
