"""Plain FP64 CPU oracle of the coupled velocity-pressure-force solve.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or links
this package: only the test-suite, the smoke check and the benchmark's CPU
baseline leg use it.  It shares no code with the HIP library.

The oracle follows the paper (Yovel, Treister, Feldman, "A SIMPLE-based
preconditioned solver for the direct-forcing immersed boundary method"):

  * mac.py      staggered-grid operators G, D = -G^T, L = G^T G, the momentum
                (Helmholtz) operator and the explicit convection term
                (Sec. 3.1, eqs. ustar / modified_poisson), as explicit
                scipy.sparse matrices, plus an independent stencil formulation;
  * delta.py    the discrete delta kernels and the regularization matrix
                R (here W) and its transpose (Sec. 2.3, eqs. delta,
                interpolation, regularization);
  * poisson.py  exact pseudo-inverse of L by fast diagonalisation (the
                uniform-grid equivalent of the direct solver of Sec. 4.2);
  * krylov.py   right-preconditioned GMRES;
  * schur.py    the lumped primal Schur complement solve
                (Sec. 4.1, eqs. tildeSp, ApproxSchurPrimalP, ApproxSchurPrimalF);
  * bodies.py   rigid-body kinematics, the rotation update and the discrete
                Newton-Euler equations (Sec. 2.2, Sec. 3.2.1);
  * step.py     one-way and two-way time steps (Sec. 3.1, Sec. 3.2.1);
  * adjoint.py  the transposed time step and point-position gradients.

Readings of the paper where it is silent or inconsistent are stated in the
docstrings of the functions that take them.
"""
