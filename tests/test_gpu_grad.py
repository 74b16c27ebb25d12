"""GPU gradients of the perambulator loss (8^4 gradient workload) against the FP64 oracle.

8^4 lattice, m0 = 0.05, c_sw = 1, N_ev = 16 seeded orthonormal LapH vectors,
64 spin-diluted sources at t0 = 0, L = sum |tau[t_sink = 4]|^2.  The GPU
gradients with respect to the sources and to m0 come from the differentiable
wrappers (adjoint solve = the library's dagger solve, inner FP32 or FP16-norm
iterations with FP64 reliable updates).  Reference numbers -- the oracle's
adjoint-formula gradients and its central differences at h = 1e-4 -- are in
tests/golden/gradients_8x8x8x8.json, written by tests/golden/make_gradients_8x8x8x8.py
(oracle only).  Tolerance 1e-5 relative (per checked scalar, floored at 1e-3 of
the largest gradient entry for components).
"""
import json
import os

import numpy as np
import pytest
import torch

import laph_synth as ls
from gpu_common import dev, host, log_case, make_lattice, require_gpu

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "gradients_8x8x8x8.json")


@pytest.fixture(scope="module")
def grad_case():
    require_gpu()
    from golden.make_gradients_8x8x8x8 import directions, single_components  # noqa: F401
    ref = json.load(open(GOLDEN))
    cfg = ls.CONFIGS["gradients_8x8x8x8"]
    dims = cfg["dims"]
    U = ls.gauge_field(dims, cfg["seed_u"])
    V = ls.orthonormal_laph_vectors(dims, cfg["nev"], cfg["seed_v"])
    return dict(cfg=cfg, ref=ref, U=U, V=V)


def _close(a, b, tol, floor=0.0):
    return abs(a - b) <= tol * max(abs(b), floor)


@pytest.mark.parametrize("prec", ["f32", "f16n"])
def test_gradients_vs_oracle_and_fd(grad_case, prec):
    import paper_2510_26313_amd as pl
    from golden.make_gradients_8x8x8x8 import directions
    cfg, ref = grad_case["cfg"], grad_case["ref"]
    log_case("gradients", prec=prec)
    lat = make_lattice(cfg["dims"], grad_case["U"], masses=cfg["masses"], csw=cfg["csw"])
    Vd = dev(grad_case["V"])
    B = lat.make_sources(Vd, 0).requires_grad_(True)
    m0 = torch.tensor(cfg["masses"][0], dtype=torch.float64, requires_grad=True)
    X = pl.solve(lat, B, m0, tol=1e-10, inner_prec=prec)
    tau = pl.project(lat, X, Vd)
    L = (tau[cfg["t_sink"]].abs() ** 2).sum()
    L.backward()
    gB = host(B.grad)
    gm = float(m0.grad)
    assert _close(float(L), ref["L"], 1e-8)
    assert _close(gm, ref["grad_m0"], 1e-6)
    assert _close(gm, ref["fd_m0"], 1e-5)
    assert _close(float(np.linalg.norm(gB)), ref["grad_b_norm"], 1e-6)
    gmax = np.abs(gB).max()
    for d, r in zip(directions(gB.shape, cfg["seed_fd"]), ref["directions"]):
        an = float(np.real(np.vdot(gB, d)))
        assert _close(an, r["adjoint"], 1e-6, 1e-3 * gmax)
        assert _close(an, r["fd"], 1e-5, 1e-3 * gmax)
    for c in ref["components"]:
        an = float(np.real(gB[tuple(c["index"])]))
        assert _close(an, c["fd"], 1e-5, 1e-3 * gmax)


def test_perambulator_autograd_matches_fused(grad_case):
    """The composed differentiable perambulator equals the fused library call."""
    import paper_2510_26313_amd as pl
    cfg, ref = grad_case["cfg"], grad_case["ref"]
    lat = make_lattice(cfg["dims"], grad_case["U"], masses=cfg["masses"], csw=cfg["csw"])
    Vd = dev(grad_case["V"])
    log_case("perambulator_autograd")
    m0 = torch.tensor(cfg["masses"][0], dtype=torch.float64, requires_grad=True)
    tau_g = pl.perambulator(lat, Vd, 0, m0, tol=1e-10, csw=cfg["csw"], inner_prec="f32")
    with torch.no_grad():
        tau_f = pl.perambulator(lat, Vd, 0, cfg["masses"][0], tol=1e-10, csw=cfg["csw"], inner_prec="f32")
    t1, t2 = host(tau_g), host(tau_f)
    assert np.linalg.norm(t1 - t2) <= 1e-8 * np.linalg.norm(t2)
    (tau_g[cfg["t_sink"]].abs() ** 2).sum().backward()
    assert _close(float(m0.grad), ref["grad_m0"], 1e-6)


@pytest.mark.parametrize("dims,nrhs", [((6, 4, 4, 10), 3), ((16, 16, 16, 32), 1)])
def test_mass_gradient_reduction_vs_fsum(dims, nrhs):
    """The library's FP64 reduction -sum_r Re<Z_r, X_r> against an exactly rounded sum
    (math.fsum) of the same products, on seeded random fields."""
    import math
    require_gpu()
    U = ls.gauge_field(dims, 81)
    lat = make_lattice(dims, U)
    Z = ls.random_spinor(ls.spinor_shape(dims, nrhs), 8100)
    X = ls.random_spinor(ls.spinor_shape(dims, nrhs), 8101)
    log_case("mass_gradient", dims=dims, nrhs=nrhs)
    g = lat.mass_gradient(dev(Z), dev(X))
    terms = np.concatenate([(Z.real * X.real).ravel(), (Z.imag * X.imag).ravel()])
    exact = -math.fsum(terms)
    assert abs(g - exact) <= 1e-13 * math.fsum(np.abs(terms))
    # fixed summation order: the same call gives the same bits
    assert lat.mass_gradient(dev(Z), dev(X)) == g
