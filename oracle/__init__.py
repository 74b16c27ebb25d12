"""CPU oracle for the LapH perambulator path -- TEST INFRASTRUCTURE ONLY.

A plain, slow, FP64 implementation of what the GPU library computes:
the Wilson-clover Dirac matrix, plain BiCGStab / dense solves of D x = b on the
full lattice, LapH Laplacian eigenvectors, spin-diluted sources, the
perambulator projection tau = V^dagger D^-1 V and its gradients, and the meson
doublets and baryon triplets of the LapH vectors.  It shares no
code with the HIP library and neither imports the other.  Only ``tests/``,
``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may use
it; the product path never routes through it.

Parity status: every function here is pinned by the CPU tests in
``tests/test_oracle_pins.py`` (dense inverse, free-field propagator in closed
form, constant-flux clover eigenvalues, gamma5-hermiticity, gauge covariance,
Schur identity, perambulator reciprocity, free Laplacian spectrum, free-field
perambulator and its mass derivative, finite differences, codec bound;
plane-wave closed forms, zero-momentum identity, gauge invariance, the
determinant form and antisymmetry of the doublets and triplets).
"""
from . import codec, dirac, laph, solvers  # noqa: F401
from ._cref import build_oracle_c  # noqa: F401
