"""CPU FP64 oracle for the derivative (and adjoint) of a QCP solution map.

TEST INFRASTRUCTURE ONLY. Only the tests, the package smoke check and the CPU-baseline leg
of the benchmark may import this package. The GPU library never calls it and shares no
code with it; both sides only share the seeded input generator (qcpgen), which holds none
of the method's arithmetic.

Contents
  cones       -- projections onto the dual cones and their Jacobians (Appendix A)
  embedding   -- Q, the residual map R, the normalised residual N, D_theta N and its
                 adjoint, D_z N (= F), phi and D phi (Sec. 2.1 - 2.4)
  lsqr        -- Paige & Saunders LSQR with optional right (column) scaling
  derivative  -- JVP and VJP by the paper's steps (Sec. 3.1, 3.2) with LSQR;
                 the dense implicit-function-theorem reference on the reduced KKT matrix;
                 the textbook active-set QP derivative; a semismooth Newton re-solve used
                 for finite differences.

Everything is numpy/scipy in float64. Library routines used as single steps: sparse
matrix-vector products, numpy.linalg.eigh, numpy.linalg.solve/inv.
"""
