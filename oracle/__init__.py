"""Plain FP64 CPU oracle for deflated multi-shift, multi-RHS GMRES.

TEST INFRASTRUCTURE ONLY. This package is the slow, obviously correct
reference that the GPU library is checked against. Only the test suite, the
smoke check and the benchmark's CPU-baseline leg may import it; the product
library never does, and it never imports the product library. Both sides
share only the seeded input generators in ``synth``.

Every routine is written in complex128 NumPy, step by step in the paper's
order and notation, with library primitives (matmul, lstsq, solve, eig, qr)
as single steps:

* ``lattice``  -- lexicographic / even-odd indexing and neighbour tables,
* ``wilson``   -- the Wilson-Dirac matrix A = I - kappa D of Example 7,
* ``kappa``    -- kappa_c from the rightmost eigenvalue of D,
* ``gmres``    -- GMRES-Sh (Sec. 2.1), GMRES-DR-Sh (Sec. 3), the minres
                  projection and GMRES-Proj-Sh with the v_{k+1} tracking,
                  extra right-hand side and correction (Sec. 4), the
                  related-RHS projection (Sec. 5).

The paper writes real transposes; the operator here is complex, so every
transpose is read as the conjugate transpose and inner products are u^H w.
"""
