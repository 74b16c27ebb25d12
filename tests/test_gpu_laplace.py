"""GPU LapH vectors: -Delta on every timeslice and its lowest eigenpairs, against the oracle.

* (-Delta) X against the oracle's stencil on a ragged lattice and on one whose x
  extent is a block row (1e-13);
* the nev lowest eigenpairs against the oracle's dense eigendecomposition per
  timeslice (4^4 with nev 8, 8^3 x 4 with nev 16, a non-cubic 6x4x4x6 with an odd
  nev 5 and 4^4 with a single vector): eigenvalues within 1e-10,
  eigenvectors (both sides in the same phase convention) within 1e-8; the same at
  8^3 x 4 with the orthonormalisation forced through either of its two paths;
* 16^3 x 4, nev 32: eigenvalues of timeslice 0 against ARPACK (scipy eigsh on the
  oracle's stencil), residuals of every pair with the oracle's stencil;
* 32^3 x 64, nev 64 (the perambulator lattice): residuals with the oracle's stencil
  and orthonormality on sampled timeslices.
"""
import numpy as np
import pytest

import laph_synth as ls
from gpu_common import dev, host, log_case, make_lattice, require_gpu
from oracle import laph as olaph

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _lattice(dims, seed):
    U = ls.gauge_field(dims, seed)
    return U, make_lattice(dims, U)


def _colour_fields(dims, n, seed):
    lx, ly, lz, lt = dims
    rng = np.random.default_rng(seed)
    shape = (lt, n, lz, ly, lx, 3)
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def _residuals(U3, V, lam):
    """||(-Delta) v - lambda v|| per vector of one timeslice, with the oracle's stencil."""
    r = olaph.neg_laplacian_apply(U3, V) - lam[:, None, None, None, None] * V
    return np.linalg.norm(r.reshape(V.shape[0], -1), axis=1)


@pytest.mark.parametrize("dims", [(6, 4, 4, 10), (32, 8, 4, 4)])
def test_apply_laplacian_vs_oracle(dims):
    """(6, 4, 4, 10): blocks of 32 sites that straddle x rows; (32, 8, 4, 4): one x row
    per block, rows visited in tiles of (y, z)."""
    U, lat = _lattice(dims, 61)
    X = _colour_fields(dims, 5, 62)
    log_case("apply_laplacian", dims=dims)
    got = host(lat.apply_laplacian(dev(X)))
    for t in range(dims[3]):
        ref = olaph.neg_laplacian_apply(U[t], X[t])
        assert np.abs(got[t] - ref).max() <= 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("dims,nev,seed", [((4, 4, 4, 4), 8, 1000), ((8, 8, 8, 4), 16, 1001),
                                            ((6, 4, 4, 6), 5, 1002), ((4, 4, 4, 4), 1, 1003)])
def test_eigvecs_vs_dense_oracle(dims, nev, seed):
    U, lat = _lattice(dims, seed)
    Vref, lamref, gap = olaph.laplacian_eigvecs(U, nev)
    log_case("laplacian_eigvecs", dims=dims, nev=nev)
    V, lam, info = lat.laplacian_eigvecs(nev, tol=1e-12)
    V = host(V)
    assert info["residual"] <= 1e-12
    assert np.abs(lam - lamref).max() <= 1e-10
    # eigenvector error <~ residual / gap to the rest of the spectrum
    err = np.linalg.norm((V - Vref).reshape(dims[3], nev, -1), axis=2)
    assert err.max() <= 1e-8, (err.max(), gap.min())


@pytest.mark.parametrize("tiny", ["2", "1e-300"])
def test_eigvecs_orthonormalisation_paths(monkeypatch, tiny):
    """The Cholesky breakdown threshold forced both ways: every timeslice through the
    Gram eigendecomposition (2), or none however close to breakdown (1e-300)."""
    dims, nev, seed = (8, 8, 8, 4), 16, 1001
    U, lat = _lattice(dims, seed)
    Vref, lamref, _ = olaph.laplacian_eigvecs(U, nev)
    monkeypatch.setenv("LAPH_EIG_CHOL_TINY", tiny)
    log_case("laplacian_eigvecs orthonormalisation", dims=dims, nev=nev, chol_tiny=tiny)
    V, lam, info = lat.laplacian_eigvecs(nev, tol=1e-12)
    V = host(V)
    assert info["residual"] <= 1e-12
    assert np.abs(lam - lamref).max() <= 1e-10
    err = np.linalg.norm((V - Vref).reshape(dims[3], nev, -1), axis=2)
    assert err.max() <= 1e-8


def test_eigvecs_16cubed_vs_arpack():
    from scipy.sparse.linalg import LinearOperator, eigsh
    dims, nev = (16, 16, 16, 4), 32
    U, lat = _lattice(dims, 1001)
    log_case("laplacian_eigvecs", dims=dims, nev=nev)
    V, lam, info = lat.laplacian_eigvecs(nev, tol=1e-10)
    V = host(V)
    lx, ly, lz, lt = dims
    n = 3 * lx * ly * lz
    op = LinearOperator((n, n), matvec=lambda v: olaph.neg_laplacian_apply(
        U[0], v.reshape(lz, ly, lx, 3)).reshape(-1), dtype=np.complex128)
    w = np.sort(eigsh(op, k=nev, which="SA", tol=1e-12, return_eigenvectors=False))
    assert np.abs(lam[0] - w).max() <= 1e-9
    for t in range(lt):
        assert _residuals(U[t], V[t], lam[t]).max() <= 1e-9
        g = V[t].reshape(nev, -1).conj() @ V[t].reshape(nev, -1).T
        assert np.abs(g - np.eye(nev)).max() <= 1e-12


def test_eigvecs_full_lattice_residuals():
    cfg = ls.CONFIGS["perambulator_32x32x32x64"]
    dims, nev = cfg["dims"], cfg["nev"]
    U, lat = _lattice(dims, cfg["seed_u"])
    log_case("laplacian_eigvecs", dims=dims, nev=nev)
    V, lam, info = lat.laplacian_eigvecs(nev, tol=1e-10)
    print("eigvecs 32^3x64 nev 64:", info, flush=True)
    assert np.all(np.diff(lam, axis=1) >= 0)
    for t in (0, 37):
        Vt = host(V[t])
        assert _residuals(U[t], Vt, lam[t]).max() <= 1e-9
        g = Vt.reshape(nev, -1).conj() @ Vt.reshape(nev, -1).T
        assert np.abs(g - np.eye(nev)).max() <= 1e-12


def test_perambulator_from_gpu_laph_vectors():
    """The whole pipeline on the 4^4 workload: LapH vectors from the GPU eigensolver, then the fused
    perambulator, against the oracle's dense-inverse perambulator on the oracle's vectors."""
    import paper_2510_26313_amd as pl
    cfg = ls.CONFIGS["dense_4x4x4x4"]
    dims = cfg["dims"]
    U = ls.gauge_field(dims, cfg["seed_u"])
    lat = make_lattice(dims, U, masses=cfg["masses"], csw=cfg["csw"])
    log_case("pipeline", dims=dims, nev=cfg["nev"])
    V, lam, info = lat.laplacian_eigvecs(cfg["nev"], tol=1e-12)
    tau, st = lat.perambulator_raw(V, 0, 0, 1e-12, pl.default_params(inner_prec="f64"))
    Vref, _, _ = olaph.laplacian_eigvecs(U, cfg["nev"])
    ref, _ = olaph.perambulator(U, Vref, 0, cfg["masses"][0], method="dense")
    assert np.linalg.norm(host(tau) - ref) <= 1e-9 * np.linalg.norm(ref)
