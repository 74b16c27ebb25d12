"""Workload parameters of the five synthetic workloads.

The paper's production workload is a 64^3 x 192 ensemble split over 32 GPUs
(Sec. "Performance Measurement Method" and "Performance Results"); one GPU's
share is about 1.6M sites, which the 32^3 x 64 headline case (2.1M sites)
stands in for.  The smaller cases are correctness and feature cases:

* ``dense_4x4x4x4``: 4^4, FP64 throughout, LapH vectors = lowest eigenvectors of the 3-D
  Laplacian, checked against a dense inverse.
* ``single_rhs_16x16x16x32``: 16^3 x 32, single-RHS solves with FP32 / FP16-with-norm inner precision.
* ``multimass_24x24x24x48``: 24^3 x 48, one batched solve of 256 RHS over four masses (40/72/64/80).
* ``gradients_8x8x8x8``: differentiation (8^4 finite-difference check, 16^3 x 32 timing).
* ``perambulator_32x32x32x64``: 32^3 x 64 headline: 4 source times x 256 RHS, projection on all sinks.

Dims are ``(Lx, Ly, Lz, Lt)``; time is antiperiodic for the fermions in every case.
"""

CONFIGS = {
    "dense_4x4x4x4": dict(dims=(4, 4, 4, 4), seed_u=1000, nev=8, v_kind="laplacian",
               masses=(0.1,), split=(32,), t0s=(0,), csw=1.0, tol=1e-12),
    "single_rhs_16x16x16x32": dict(dims=(16, 16, 16, 32), seed_u=1001, nev=32, seed_v=2001,
               masses=(0.05,), split=(128,), t0s=(0,), csw=1.0, tol=1e-10),
    "multimass_24x24x24x48": dict(dims=(24, 24, 24, 48), seed_u=1002, nev=64, seed_v=2002,
               masses=(0.02, 0.05, 0.1, 0.2), split=(40, 72, 64, 80), t0s=(0,),
               csw=1.0, tol=1e-10),
    "gradients_8x8x8x8": dict(dims=(8, 8, 8, 8), dims_timing=(16, 16, 16, 32), seed_u=1003,
               nev=16, seed_v=2003, masses=(0.05,), split=(64,), t0s=(0,),
               t_sink=4, t_sink_timing=8, csw=1.0, tol=1e-10, fd_h=1e-4,
               seed_fd=4000),
    "perambulator_32x32x32x64": dict(dims=(32, 32, 32, 64), seed_u=1004, nev=64, seed_v=2004,
               masses=(0.02,), split=(256,), t0s=(0, 16, 32, 48), csw=1.0,
               tol=1e-10),
}

GAUGE_EPS = 0.3
SEED_GAUGE_TRANSFORM = 3000
SEED_DSLASH_SPINOR = 5000


def rhs_masses(cfg):
    """Per-RHS mass index for a config: contiguous ranges in RHS order r = 4k + alpha."""
    out = []
    for i, n in enumerate(cfg["split"]):
        out += [i] * n
    return out
