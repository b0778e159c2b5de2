"""FP64 CPU oracle for the low-rank IgA optimal-control method (Buenger, Dolgov, Stoll).

TEST INFRASTRUCTURE ONLY. Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import or call anything here. The GPU
library never calls it and shares no code with it.

What it computes is the plain definition of what the GPU path computes
approximately or in another order:

* ``bspline``   -- open knot vectors, the Cox-de Boor recursion and its
                   derivative, Gauss-Legendre rules per element (Section 2).
* ``geometry``  -- the geometry map G = C:B, its Jacobian, omega = |det grad G|
                   and Q = (grad G^T grad G)^{-1} omega (Section 2).
* ``assembly``  -- full 3-D Galerkin mass and stiffness matrices by tensor
                   Gauss quadrature, element by element, in two modes: exact
                   weights, or weights interpolated in the higher-degree space
                   of Section 3 (the integrand the Kronecker form reproduces);
                   Dirichlet trimming; a matrix-free element-loop apply and
                   row sampling for large n; 1-D factor matrices.
* ``kkt``       -- the stationary KKT system of the control problem
                   (Section 4, time dropped), direct solve, objective.
* ``parabolic`` -- the time-dependent KKT system of Section 4 (implicit
                   Euler, rectangle rule, y_0 = 0): block matrix with the
                   time-difference matrix C, direct solve, objective.
* ``tt``        -- TT/TT-matrix expansion, TT-SVD, the frame matrix of
                   Section 5 and the projected local operator by its
                   definition F^T A F.

Pins tying each function to the paper or to mathematics live in
``tests/test_oracle_*.py``. Functions without such a pin say so.
"""
