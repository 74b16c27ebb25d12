"""GPU stochastic LapH (noise-diluted sources), against the oracle.

* the diluted noise sources against the oracle's, on a ragged lattice;
* the fused stochastic perambulator on 4^4 ( Laplacian eigenvectors, Z4 noise,
  3 interlaced groups) against the oracle's dense-inverse result, FP64 and FP16N inner;
* full dilution with unit noise reproduces the GPU perambulator;
* invalid dilution raises.
"""
import numpy as np
import pytest

import laph_synth as ls
from gpu_common import dev, host, log_case, make_lattice, rel, require_gpu
from oracle import laph

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _z4(nev, seed):
    rng = np.random.default_rng(seed)
    return np.ascontiguousarray(np.exp(0.5j * np.pi * rng.integers(0, 4, size=(4, nev))))


def test_noise_sources_vs_oracle():
    dims = (6, 4, 4, 6)
    U = ls.gauge_field(dims, 71)
    V = ls.orthonormal_laph_vectors(dims, 5, 72)
    rho = _z4(5, 73)
    lat = make_lattice(dims, U)
    log_case("noise_sources", dims=dims, nev=5, n_dil=2)
    B = host(lat.make_noise_sources(dev(V), 3, dev(rho), 2))
    ref = laph.noise_sources(V, 3, rho, 2)
    assert B.shape == ref.shape
    assert np.abs(B - ref).max() <= 1e-15 * np.abs(ref).max()


def test_stochastic_perambulator_4x4x4x4():
    import paper_2510_26313_amd as pl
    cfg = ls.CONFIGS["dense_4x4x4x4"]
    U = ls.gauge_field(cfg["dims"], cfg["seed_u"])
    V, _, _ = laph.laplacian_eigvecs(U, cfg["nev"])
    rho = _z4(cfg["nev"], 74)
    phi_ref, _ = laph.stochastic_perambulator(U, V, 1, cfg["masses"][0], rho, 3, method="dense")
    lat = make_lattice(cfg["dims"], U, masses=cfg["masses"])
    for prec in ("f64", "f16n"):
        log_case("stochastic_perambulator_4x4x4x4", prec=prec)
        phi, st = lat.stochastic_perambulator_raw(dev(V), 1, dev(rho), 3, 0, 1e-12 if prec == "f64" else 1e-10,
                                                  pl.default_params(inner_prec=prec))
        assert len(st) == 12 and all(s["status"] == "converged" for s in st)
        assert rel(host(phi), phi_ref) < 1e-8


def test_full_dilution_unit_noise_is_perambulator():
    import paper_2510_26313_amd as pl
    dims, nev = (4, 4, 4, 6), 4
    U = ls.gauge_field(dims, 75)
    V = ls.orthonormal_laph_vectors(dims, nev, 76)
    lat = make_lattice(dims, U)
    p = pl.default_params(inner_prec="f32")
    log_case("full dilution")
    tau = host(lat.perambulator_raw(dev(V), 2, 0, 1e-11, p)[0])
    phi = host(lat.stochastic_perambulator_raw(dev(V), 2, dev(np.ones((4, nev), dtype=np.complex128)), nev, 0,
                                               1e-11, p)[0])
    assert rel(phi, tau) < 1e-13


def test_invalid_dilution():
    import paper_2510_26313_amd as pl
    dims, nev = (4, 4, 4, 4), 3
    U = ls.gauge_field(dims, 77)
    V = dev(ls.orthonormal_laph_vectors(dims, nev, 78))
    lat = make_lattice(dims, U)
    rho = dev(_z4(nev, 79))
    for n_dil in (0, nev + 1):
        with pytest.raises(pl.LaphError):
            lat.make_noise_sources(V, 0, rho, n_dil)
    with pytest.raises(pl.LaphError):
        lat.stochastic_perambulator_raw(V, 0, rho, 0)
