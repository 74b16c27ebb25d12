"""Seeded synthetic inputs shared by the CPU oracle, the tests and the benchmark.

This module holds no arithmetic of the LapH method itself: it only draws the
inputs both sides receive (gauge links, orthonormal colour vectors, random
spinors, random gauge transforms) and the table of workload parameters.  The
method (Dirac operator, solves, projection) lives separately in ``oracle/``
(CPU reference) and in the HIP library; neither is imported here.

Array conventions (C order, complex128):

* gauge links      ``U[t][z][y][x][mu][a][b]``      mu = 0,1,2,3 <-> x,y,z,t
* spinor field     ``psi[t][z][y][x][s][a]``        spin s in 0..3, colour a in 0..2
* LapH vectors     ``V[t][l][z][y][x][a]``          l in 0..nev-1 (column l of the
  per-timeslice orthonormal basis, flat index ``a + 3*(x + L*(y + L*z))``)

The paper generates its gauge ensembles by Markov-chain Monte Carlo in an
earlier step (Sec. "Performance Measurement Method"); those ensembles are not
available, so the links here are rough synthetic SU(3) fields
``U = exp(i*eps*H)`` with ``H`` a Gaussian traceless Hermitian 3x3 matrix.
"""
from .generators import (  # noqa: F401
    gauge_field,
    unit_gauge,
    orthonormal_laph_vectors,
    random_spinor,
    random_su3,
    spinor_shape,
    gauge_shape,
)
from .configs import CONFIGS, rhs_masses  # noqa: F401
