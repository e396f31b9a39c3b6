"""CPU FP64 oracle for the explicit order-2k generalized-alpha method with the
Kronecker-preconditioned mass solve (Behnoudfar, Loli, Reali, Sangalli, Calo,
"Explicit high-order generalized-alpha methods for isogeometric analysis of
structural dynamics").

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call, link
or execute anything in this package: only ``tests/``, ``__graft_entry__.smoke``
and the ``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the
HIP library (no kernels, headers, helpers, tables or constant generators).

Every routine is the plain definition of what the paper computes, in FP64,
with sparse-matrix library calls as the only building blocks:

* ``bspline``   -- open knot vectors, Cox-de Boor recursion, Gauss rule (Sec. 5.1)
* ``operators`` -- mass (eq. mass_matrix) and stiffness (eq. mp / pde) matrices
                   by Gauss quadrature, Dirichlet elimination, sampled rows
* ``precond``   -- the diagonally scaled Kronecker preconditioner (Sec. 5.4)
* ``solvers``   -- preconditioned CG and direct Cholesky mass solves (Sec. 5.6, 6)
* ``galpha``    -- parameters, predictor/stage/update step and initialisation of
                   the order-2k scheme (Sec. 3-4, eqs. ho1-ho3), and the scalar
                   amplification matrix used by the pins.
* ``convnet``   -- the learned initial guess (an addition, not in the paper):
                   network definition, crop loss and its gradient, Adam.
* ``multipatch``-- C0-glued patches and the additive Schwarz preconditioner
                   (Sec. 5.3, 5.5).
* ``dispersion``-- the 1-D dispersion study of Sec. 6.2 (omega = 1/j).

Readings of passages that are silent, ambiguous or garbled are listed in the
module docstrings where they apply.  Parity status: every function is pinned
by a ``-m "not gpu"`` test against closed forms, library routines, printed
matrices or brute force, except where a docstring says "parity unpinned".
"""
