"""Perambulator columns of the two large workloads against stored oracle values.

``tests/golden/tau_columns_*.npz`` hold columns tau[:, :, k, :, alpha] (every sink
timeslice, LapH vector and sink spin) of single RHS r = 4k + alpha, written by
``tests/golden/make_tau_columns.py`` from the FP64 oracle alone (full-system
BiCGStab to 1e-13, plain projection).  The library computes them in the
configuration the benchmark times (FP16-with-norm inner iterations, FP64 reliable
updates, batches of 128 RHS, tolerance 1e-10) and they must agree per column to a
relative L2 error of 1e-8:

* the perambulator workload (32^3 x 64, nev 64, m0 0.02): one column per source
  time t0 in {0, 16, 32, 48}, each from the full 256-RHS perambulator of that t0;
* the multi-mass workload (24^3 x 48): two columns per mass from one batched solve
  of all 256 RHS over four masses (40/72/64/80), projected by the library.
"""
import gc
import os

import numpy as np
import pytest
import torch

import laph_synth as ls
from gpu_common import dev, host, log_case, make_lattice, require_gpu

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _load(name):
    path = os.path.join(GOLDEN, "tau_columns_%s.npz" % name)
    if not os.path.exists(path):
        pytest.skip("golden file %s not generated" % path)
    with np.load(path, allow_pickle=False) as z:
        return {k: z[k] for k in z.files}


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_perambulator_32x32x32x64_columns_vs_oracle():
    import paper_2510_26313_amd as pl
    require_gpu()
    gc.collect()
    torch.cuda.empty_cache()
    g = _load("32x32x32x64")
    cfg = ls.CONFIGS["perambulator_32x32x32x64"]
    dims = cfg["dims"]
    U = ls.gauge_field(dims, cfg["seed_u"])
    V = ls.orthonormal_laph_vectors(dims, cfg["nev"], cfg["seed_v"])
    lat = make_lattice(dims, U, masses=cfg["masses"], csw=cfg["csw"])
    Vd = dev(V)
    del V
    p = pl.default_params(inner_prec="f16n", chunk=128, rhs_tile=16, stencil=2, traversal=2)
    for i, (t0, r) in enumerate(zip(g["t0"], g["rhs"])):
        log_case("32^3x64 perambulator vs golden", t0=int(t0), rhs=int(r))
        tau, st = lat.perambulator_raw(Vd, int(t0), 0, 1e-10, p)
        assert all(s["status"] == "converged" and s["true_res"] <= 1e-10 for s in st)
        k, al = divmod(int(r), 4)
        col = host(tau[:, :, k, :, al])
        err = _rel(col, g["tau"][i])
        print("t0 %d rhs %d: relative L2 error of the tau column %.3e" % (t0, r, err), flush=True)
        assert err <= 1e-8
        del tau
    lat.release_scratch()


def test_multimass_24x24x24x48_columns_vs_oracle():
    import paper_2510_26313_amd as pl
    require_gpu()
    gc.collect()
    torch.cuda.empty_cache()
    g = _load("24x24x24x48")
    cfg = ls.CONFIGS["multimass_24x24x24x48"]
    dims = cfg["dims"]
    U = ls.gauge_field(dims, cfg["seed_u"])
    V = ls.orthonormal_laph_vectors(dims, cfg["nev"], cfg["seed_v"])
    lat = make_lattice(dims, U, masses=cfg["masses"], csw=cfg["csw"])
    mi = ls.rhs_masses(cfg)
    Vd = dev(V)
    B = lat.make_sources(Vd, 0)
    log_case("24^3x48 batched four-mass solve vs golden", nrhs=len(mi))
    X, st = lat.solve_raw(B, mi, 1e-10, pl.default_params(inner_prec="f16n", rhs_tile=16, stencil=2))
    assert all(s["status"] == "converged" and s["true_res"] <= 1e-10 for s in st)
    del B
    for i, r in enumerate(g["rhs"]):
        r = int(r)
        assert abs(cfg["masses"][mi[r]] - float(g["mass"][i])) < 1e-15
        k, al = divmod(r, 4)
        # the library's projection of this solution: a spin quartet with only slot alpha set
        X4 = torch.zeros(lat.spinor_shape(4), dtype=torch.complex128, device="cuda")
        X4[al] = X[r]
        tau = lat.project_raw(X4, Vd)
        col = host(tau[:, :, 0, :, al])
        err = _rel(col, g["tau"][i])
        print("m0 %g rhs %d: relative L2 error of the tau column %.3e" % (g["mass"][i], r, err), flush=True)
        assert err <= 1e-8
    del X
    lat.release_scratch()
