"""GPU parity: every HIP entry point against the CPU oracle on the same seeded inputs.

Sizes are chosen so the oracle finishes in seconds while the kernels still
span several 256-site blocks with a ragged tail (6x4x4x10: 480 sites per
parity), plus the 4^4 configuration of the dense-inverse check.
"""
import numpy as np
import pytest
import torch

import laph_synth as ls
from gpu_common import dev, host, log_case, make_lattice, parity_mask, per_rhs_rel, rel, require_gpu
from oracle import codec, dirac, laph, solvers

pytestmark = pytest.mark.gpu

DIMS_RAGGED = (6, 4, 4, 10)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


@pytest.fixture(scope="module")
def ragged():
    U = ls.gauge_field(DIMS_RAGGED, 42)
    lat = make_lattice(DIMS_RAGGED, U, masses=(0.1, 0.05))
    return U, lat


# ---------------------------------------------------------------------------
# layouts
# ---------------------------------------------------------------------------

def test_pack_unpack_roundtrip(ragged):
    U, lat = ragged
    psi = ls.random_spinor(ls.spinor_shape(DIMS_RAGGED, 3), 5003)
    log_case("pack_unpack", dims=DIMS_RAGGED)
    t = dev(psi)
    back = host(lat.unpack(lat.pack(t, "f64"), 3, "f64"))
    assert np.array_equal(back, psi)
    back32 = host(lat.unpack(lat.pack(t, "f32"), 3, "f32"))
    exp32 = psi.real.astype(np.float32).astype(np.float64) + 1j * psi.imag.astype(np.float32).astype(np.float64)
    assert np.array_equal(back32, exp32)
    back16 = host(lat.unpack(lat.pack(t, "f16n"), 3, "f16n"))
    v = np.stack([psi.real, psi.imag], axis=-1).reshape(psi.shape[:5] + (24,))
    q, n = codec.encode(v)
    d = codec.decode(q, n).astype(np.float64).reshape(psi.shape[:5] + (12, 2))
    exp16 = (d[..., 0] + 1j * d[..., 1]).reshape(psi.shape)
    assert np.array_equal(back16, exp16)


# ---------------------------------------------------------------------------
# stencil and clover
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("prec,tol", [("f64", 1e-14), ("f32", 1e-6), ("f16n", 3e-3)])
@pytest.mark.parametrize("dagger", [False, True])
def test_apply_dslash(ragged, prec, tol, dagger):
    U, lat = ragged
    par = parity_mask(DIMS_RAGGED)[..., None, None]
    psi = ls.random_spinor(ls.spinor_shape(DIMS_RAGGED, 2), 5002)
    for out_p in (0, 1):
        log_case("apply_dslash", prec=prec, dagger=dagger, out_parity=out_p)
        src = psi * (par == 1 - out_p)
        buf = lat.pack(dev(src), prec, parity=1 - out_p)
        out = lat.apply_dslash(buf, 2, out_p, prec, dagger)
        got = host(lat.unpack(out, 2, prec, parity=out_p))
        exp = dirac.hop(U, src, True, dagger) * (par == out_p)
        assert rel(got, exp) < tol


@pytest.mark.parametrize("prec,tol", [("f64", 1e-14), ("f32", 1e-6)])
def test_apply_clover(ragged, prec, tol):
    U, lat = ragged
    par = parity_mask(DIMS_RAGGED)[..., None, None]
    psi = ls.random_spinor(ls.spinor_shape(DIMS_RAGGED, 2), 5004)
    for mi, m0 in enumerate((0.1, 0.05)):
        A = dirac.clover_matrix(U, m0, 1.0)
        Ai = dirac.clover_inverse(A)
        for p in (0, 1):
            for inv, M in ((False, A), (True, Ai)):
                log_case("apply_clover", prec=prec, mass=m0, parity=p, inverse=inv)
                src = psi * (par == p)
                out = lat.apply_clover(lat.pack(dev(src), prec, parity=p), 2, p, mi, inv, prec)
                got = host(lat.unpack(out, 2, prec, parity=p))
                exp = dirac.apply_site_matrix(M, src)
                assert rel(got, exp) < tol


@pytest.mark.parametrize("dagger", [False, True])
def test_apply_D(ragged, dagger):
    U, lat = ragged
    psi = ls.random_spinor(ls.spinor_shape(DIMS_RAGGED, 2), 5005)
    D = dirac.WilsonClover(U, 0.05, 1.0)
    log_case("apply_D", dagger=dagger)
    got = host(lat.apply_D(dev(psi), mass_idx=1, dagger=dagger))
    exp = D.apply_dagger(psi) if dagger else D.apply(psi)
    assert rel(got, exp) < 1e-14


def test_clover_flux_closed_form():
    """P3(b) on the GPU clover: the lambda_8 flux field gives an exactly diagonal A."""
    L, lt = 4, 4
    dims = (L, L, L, lt)
    U = ls.unit_gauge(dims)
    B = 2 * np.pi / L ** 2

    def E(phi):
        return np.diag([np.exp(2j * phi), np.exp(-1j * phi), np.exp(-1j * phi)])
    for x in range(L):
        U[:, :, :, x, 1] = E(B * x)
    for y in range(L):
        U[:, :, y, L - 1, 0] = E(-B * L * y)
    lat = make_lattice(dims, U, masses=(0.1,))
    s = np.sin(2 * B) + np.sin(B)
    f = np.array([2 * s / 3, -s / 3, -s / 3])
    diag = 4.1 - 0.5 * np.outer([1, -1, 1, -1], f)
    par = parity_mask(dims)[..., None, None]
    psi = ls.random_spinor(ls.spinor_shape(dims, 1), 7)
    for p in (0, 1):
        log_case("clover_flux", parity=p)
        src = psi * (par == p)
        got = host(lat.unpack(lat.apply_clover(lat.pack(dev(src), "f64", parity=p), 1, p, 0, False), 1, "f64", p))
        assert rel(got, diag * src) < 1e-14


# ---------------------------------------------------------------------------
# projection (MFMA GEMM)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("nev,nsrc", [(5, 3), (64, 2), (17, 33)])
def test_project(ragged, nev, nsrc):
    U, lat = ragged
    V = ls.orthonormal_laph_vectors(DIMS_RAGGED, nev, 2000 + nev)
    X = ls.random_spinor(ls.spinor_shape(DIMS_RAGGED, 4 * nsrc), 6000 + nsrc)
    log_case("project", nev=nev, nsrc=nsrc)
    got = host(lat.project_raw(dev(X), dev(V)))
    exp = laph.project(V, X, nsrc)
    assert rel(got, exp) < 1e-14
    # adjoint
    G = ls.random_spinor((DIMS_RAGGED[3], nev, nsrc, 4, 4), 6100)
    got_a = host(lat.project_adjoint_raw(dev(G), dev(V)))
    exp_a = laph.tau_cotangent_to_X(V, G[0], 0, X.shape)
    for t in range(1, DIMS_RAGGED[3]):
        exp_a = exp_a + laph.tau_cotangent_to_X(V, G[t], t, X.shape)
    assert rel(got_a, exp_a) < 1e-14


def test_make_sources(ragged):
    U, lat = ragged
    V = ls.orthonormal_laph_vectors(DIMS_RAGGED, 3, 77)
    log_case("make_sources")
    got = host(lat.make_sources(dev(V), 7))
    assert np.array_equal(got, laph.laph_sources(V, 7))


# ---------------------------------------------------------------------------
# solves
# ---------------------------------------------------------------------------

def test_solve_4x4x4x4_dense():
    """4^4, LapH sources of the lowest Laplacian eigenvectors, FP64 solve to 1e-12 vs dense LU."""
    import paper_2510_26313_amd as pl
    cfg = ls.CONFIGS["dense_4x4x4x4"]
    U = ls.gauge_field(cfg["dims"], cfg["seed_u"])
    V, _, _ = laph.laplacian_eigvecs(U, cfg["nev"])
    b = laph.laph_sources(V, 0)
    D = dirac.WilsonClover(U, cfg["masses"][0], cfg["csw"])
    x_ref = solvers.dense_solve(D, b)
    lat = make_lattice(cfg["dims"], U, masses=cfg["masses"])
    for batched in (1, 0):
        log_case("solve_4x4x4x4", batched=batched)
        X, st = lat.solve_raw(dev(b), 0, 1e-12, pl.default_params(inner_prec="f64", batched=batched))
        e = per_rhs_rel(host(X), x_ref)
        assert e.max() < 1e-10, e.max()
        assert all(s["status"] == "converged" and s["true_res"] <= 1e-12 for s in st)


@pytest.fixture(scope="module")
def ragged_ref(ragged):
    U, lat = ragged
    b = ls.random_spinor(ls.spinor_shape(DIMS_RAGGED, 6), 5010)
    D = dirac.WilsonClover(U, 0.05, 1.0)
    x_ref, info = solvers.bicgstab(D.apply, b, tol=1e-13)
    return b, x_ref


@pytest.fixture(scope="module")
def f64_iters(ragged, ragged_ref):
    """Iterations of the plain FP64 even-odd BiCGStab (no reliable updates) per RHS."""
    import paper_2510_26313_amd as pl
    U, lat = ragged
    b, _ = ragged_ref
    log_case("solve f64 reference iterations")
    _, st = lat.solve_raw(dev(b), 1, 1e-10, pl.default_params(inner_prec="f64", batched=1, rhs_tile=1, stencil=1,
                                                                traversal=1))
    return [s["iters"] for s in st]


@pytest.mark.parametrize("prec", ["f64", "f32", "f16n"])
@pytest.mark.parametrize("batched,tile,stencil,trav", [(1, 0, 0, 0), (1, 2, 1, 2), (1, 4, 2, 1), (1, 8, 2, 2),
                                                      (0, 1, 1, 1)])
@pytest.mark.parametrize("graph", [1, 0])
def test_solve_mixed_precision(ragged, ragged_ref, f64_iters, prec, batched, tile, stencil, trav, graph):
    import paper_2510_26313_amd as pl
    U, lat = ragged
    b, x_ref = ragged_ref
    log_case("solve", prec=prec, batched=batched, tile=tile, stencil=stencil, graph=graph)
    p = pl.default_params(inner_prec=prec, batched=batched, rhs_tile=tile, stencil=stencil, traversal=trav,
                          use_graph=graph, graph_iters=4)
    X, st = lat.solve_raw(dev(b), 1, 1e-10, p)
    e = per_rhs_rel(host(X), x_ref)
    assert e.max() < 1e-8, (e.max(), st)
    assert all(s["status"] == "converged" and s["true_res"] <= 1e-10 for s in st), st
    # an error in the inner operator would cost iterations (the FP64 reliable updates
    # would still correct the solution): bound them by the FP64 solver's count
    iters = [s["iters"] for s in st]
    assert all(i <= j + 3 for i, j in zip(iters, f64_iters)), (iters, f64_iters)
    if prec != "f64":
        assert all(s["updates"] >= 2 for s in st)


@pytest.mark.parametrize("prec", ["f32", "f16n"])
@pytest.mark.parametrize("stencil64,tile64", [(1, 1), (1, 4), (2, 4), (2, 8), (2, 16)])
def test_solve_fp64_update_shapes(ragged, ragged_ref, prec, stencil64, tile64):
    """The FP64 reliable-update stages in each form (they act on the flagged RHS only)."""
    import paper_2510_26313_amd as pl
    U, lat = ragged
    b, x_ref = ragged_ref
    log_case("solve_fp64_updates", prec=prec, stencil64=stencil64, tile64=tile64)
    p = pl.default_params(inner_prec=prec, rhs_tile=4, stencil=2, traversal=1, stencil64=stencil64,
                          rhs_tile64=tile64, graph_iters=4)
    X, st = lat.solve_raw(dev(b), 1, 1e-10, p)
    assert per_rhs_rel(host(X), x_ref).max() < 1e-8, st
    assert all(s["status"] == "converged" and s["true_res"] <= 1e-10 and s["updates"] >= 2 for s in st), st


@pytest.mark.parametrize("stencil64,tile64", [(1, 4), (2, 8)])
def test_reported_true_residual_matches_oracle(ragged, ragged_ref, stencil64, tile64):
    """The per-RHS |B - D X| / |B| the solver reports (the LDS form takes the odd part in
    the pass that reconstructs x_o, the register form in a separate clover pass) equals
    the oracle's full-lattice residual of the returned X."""
    import paper_2510_26313_amd as pl
    U, lat = ragged
    b, _ = ragged_ref
    log_case("true_residual", stencil64=stencil64, tile64=tile64)
    p = pl.default_params(inner_prec="f16n", rhs_tile=4, stencil=2, traversal=1, stencil64=stencil64,
                          rhs_tile64=tile64)
    X, st = lat.solve_raw(dev(b), 1, 1e-10, p)
    X = host(X)
    R = b - dirac.WilsonClover(U, 0.05, 1.0).apply(X)
    for i, s in enumerate(st):
        ref = np.linalg.norm(R[i]) / np.linalg.norm(b[i])
        assert abs(s["true_res"] - ref) <= 1e-2 * ref + 1e-14, (i, s["true_res"], ref)


# 16 x 8 x 4 x 4: 64 sites per parity are whole y rows, so the LDS-form stages run
# their site blocks in 4-D tiles (4 z-planes x 4 timeslices, FP64 2 x 2)
DIMS_TILED = (16, 8, 4, 4)


@pytest.mark.parametrize("prec,stencil64", [("f16n", 2), ("f32", 1), ("f64", 0)])
def test_solve_tiled_block_order(prec, stencil64):
    import paper_2510_26313_amd as pl
    U = ls.gauge_field(DIMS_TILED, 43)
    lat = make_lattice(DIMS_TILED, U, masses=(0.05,))
    b = ls.random_spinor(ls.spinor_shape(DIMS_TILED, 8), 5030)
    x_ref, _ = solvers.bicgstab(dirac.WilsonClover(U, 0.05, 1.0).apply, b, tol=1e-13)
    log_case("solve_tiled", prec=prec, stencil64=stencil64)
    kw = dict(inner_prec=prec, rhs_tile=8, stencil=2, traversal=2)
    if prec != "f64":
        kw.update(stencil64=stencil64, rhs_tile64=4 if stencil64 == 1 else 8)
    X, st = lat.solve_raw(dev(b), 0, 1e-10, pl.default_params(**kw))
    assert per_rhs_rel(host(X), x_ref).max() < 1e-8, st
    assert all(s["status"] == "converged" and s["true_res"] <= 1e-10 for s in st), st


def test_solve_dagger(ragged, ragged_ref):
    import paper_2510_26313_amd as pl
    U, lat = ragged
    b, _ = ragged_ref
    D = dirac.WilsonClover(U, 0.05, 1.0)
    x_ref, _ = solvers.bicgstab(D.apply_dagger, b, tol=1e-13)
    log_case("solve_dagger")
    X, st = lat.solve_raw(dev(b), 1, 1e-10, pl.default_params(inner_prec="f16n", dagger=1))
    assert per_rhs_rel(host(X), x_ref).max() < 1e-8


def test_solve_multimass_batched(ragged):
    """Uneven mass split in one batched solve (the 40/72/64/80 pattern, scaled down)."""
    import paper_2510_26313_amd as pl
    U, _ = ragged
    masses = (0.02, 0.05, 0.1, 0.2)
    split = (3, 5, 2, 6)
    lat = make_lattice(DIMS_RAGGED, U, masses=masses)
    mi = [i for i, n in enumerate(split) for _ in range(n)]
    b = ls.random_spinor(ls.spinor_shape(DIMS_RAGGED, len(mi)), 5020)
    log_case("solve_multimass")
    X, st = lat.solve_raw(dev(b), mi, 1e-10, pl.default_params(inner_prec="f16n", rhs_tile=4, stencil=1))
    X = host(X)
    for m, m0 in enumerate(masses):
        idx = [r for r in range(len(mi)) if mi[r] == m]
        x_ref, _ = solvers.bicgstab(dirac.WilsonClover(U, m0, 1.0).apply, b[idx], tol=1e-13)
        assert per_rhs_rel(X[idx], x_ref).max() < 1e-8


def test_solve_multimass_lds(ragged):
    """Uneven mass split with the LDS-staged stencil (tiles of 8 RHS of one mass)."""
    import paper_2510_26313_amd as pl
    U, _ = ragged
    masses = (0.02, 0.2)
    mi = [0] * 5 + [1] * 11
    lat = make_lattice(DIMS_RAGGED, U, masses=masses)
    b = ls.random_spinor(ls.spinor_shape(DIMS_RAGGED, len(mi)), 5021)
    log_case("solve_multimass_lds")
    X, st = lat.solve_raw(dev(b), mi, 1e-10, pl.default_params(inner_prec="f32", rhs_tile=8, stencil=2))
    X = host(X)
    for m, m0 in enumerate(masses):
        idx = [r for r in range(len(mi)) if mi[r] == m]
        x_ref, _ = solvers.bicgstab(dirac.WilsonClover(U, m0, 1.0).apply, b[idx], tol=1e-13)
        assert per_rhs_rel(X[idx], x_ref).max() < 1e-8


@pytest.mark.parametrize("prec,stencil,tile,trav", [("f16n", 2, 16, 2), ("f16n", 1, 4, 1), ("f32", 2, 8, 1),
                                                   ("f64", 1, 2, 2), ("f64", 2, 8, 1)])
def test_time_stages_runs(ragged, prec, stencil, tile, trav):
    U, lat = ragged
    log_case("time_stages", prec=prec, stencil=stencil, tile=tile, traversal=trav)
    ms1, ms2 = lat.time_stages(prec, 16, tile, 0, reps=2, stencil=stencil, traversal=trav)
    assert ms1 > 0 and ms2 > 0


def test_autotune_and_auto_solve(ragged, ragged_ref):
    """The autotuner returns a valid shape, and an automatic solve (tuning on first use) converges."""
    import paper_2510_26313_amd as pl
    U, lat = ragged
    b, x_ref = ragged_ref
    log_case("autotune")
    t = lat.autotune("f16n", 6, 1)
    assert (t["stencil"], t["rhs_tile"]) in [(1, 1), (1, 2), (1, 4), (2, 4), (2, 8), (2, 16)] and t["ms"] > 0
    assert t["traversal"] in (1, 2)
    X, st = lat.solve_raw(dev(b), 1, 1e-10, pl.default_params(inner_prec="f32", stencil=0, rhs_tile=0))
    assert per_rhs_rel(host(X), x_ref).max() < 1e-8


def test_solve_x0_warm_start(ragged, ragged_ref):
    import paper_2510_26313_amd as pl
    U, lat = ragged
    b, x_ref = ragged_ref
    x0 = x_ref + 1e-3 * ls.random_spinor(x_ref.shape, 5030)
    log_case("solve_x0")
    X, st = lat.solve_raw(dev(b), 1, 1e-10, pl.default_params(inner_prec="f32"), X0=dev(x0))
    assert per_rhs_rel(host(X), x_ref).max() < 1e-8
    X2, st2 = lat.solve_raw(dev(b), 1, 1e-10, pl.default_params(inner_prec="f32"))
    assert max(s["iters"] for s in st) < max(s["iters"] for s in st2)


# ---------------------------------------------------------------------------
# perambulators
# ---------------------------------------------------------------------------

def test_perambulator_4x4x4x4():
    import paper_2510_26313_amd as pl
    cfg = ls.CONFIGS["dense_4x4x4x4"]
    U = ls.gauge_field(cfg["dims"], cfg["seed_u"])
    V, _, _ = laph.laplacian_eigvecs(U, cfg["nev"])
    tau_ref, _ = laph.perambulator(U, V, 0, cfg["masses"][0], method="dense")
    lat = make_lattice(cfg["dims"], U, masses=cfg["masses"])
    for prec in ("f64", "f16n"):
        log_case("perambulator_c0", prec=prec)
        tau, st = lat.perambulator_raw(dev(V), 0, 0, 1e-12 if prec == "f64" else 1e-10,
                                       pl.default_params(inner_prec=prec))
        assert rel(host(tau), tau_ref) < 1e-8


@pytest.mark.parametrize("t0", [3, 9])
def test_perambulator_ragged_chunks(ragged, t0):
    """nev = 5 (20 RHS) in chunks of 8: chunk boundaries cut a spin quartet.  The source
    preparation works on the timeslices around t0 only; t0 = 9 (the last of 10) takes
    that slab across the periodic boundary."""
    import paper_2510_26313_amd as pl
    U, lat = ragged
    V = ls.orthonormal_laph_vectors(DIMS_RAGGED, 5, 2100)
    tau_ref, _ = laph.perambulator(U, V, t0, 0.1, tol=1e-13)
    log_case("perambulator_chunks", t0=t0)
    tau, st = lat.perambulator_raw(dev(V), t0, 0, 1e-10, pl.default_params(inner_prec="f16n", chunk=8))
    assert rel(host(tau), tau_ref) < 1e-8
    assert len(st) == 20 and all(s["status"] == "converged" for s in st)


def test_perambulator_reciprocity_gpu(ragged):
    """P7 on the GPU result: tau(src 0)[t=4] vs tau(src 4)[t=0]."""
    import paper_2510_26313_amd as pl
    U, lat = ragged
    V = ls.orthonormal_laph_vectors(DIMS_RAGGED, 4, 2200)
    p = pl.default_params(inner_prec="f32")
    log_case("reciprocity")
    tA = host(lat.perambulator_raw(dev(V), 0, 0, 1e-11, p)[0])
    tB = host(lat.perambulator_raw(dev(V), 4, 0, 1e-11, p)[0])
    g5 = np.array([1, 1, -1, -1])
    exp = np.einsum("b,a,klab->lkba", g5, g5, np.conj(tB[0]))
    assert rel(tA[4], exp) < 1e-8


# ---------------------------------------------------------------------------
# failure handling (forced from the host; every kernel exits normally)
# ---------------------------------------------------------------------------

def test_nonfinite_source_only_that_rhs(ragged):
    import paper_2510_26313_amd as pl
    U, lat = ragged
    b = ls.random_spinor(ls.spinor_shape(DIMS_RAGGED, 3), 5040)
    b[1, 0, 0, 0, 0, 0, 0] = np.nan
    log_case("nonfinite_source")
    with pytest.raises(pl.LaphError) as ei:
        lat.solve_raw(dev(b), 0, 1e-10, pl.default_params(inner_prec="f32"))
    st = ei.value.stats
    assert st[1]["status"] == "nonfinite"
    assert st[0]["status"] == "converged" and st[2]["status"] == "converged"


def test_maxiter_noconv_and_zero_source(ragged):
    import paper_2510_26313_amd as pl
    U, lat = ragged
    b = ls.random_spinor(ls.spinor_shape(DIMS_RAGGED, 2), 5050)
    b[0] = 0
    log_case("maxiter")
    X, st = lat.solve_raw(dev(b), 0, 1e-10, pl.default_params(inner_prec="f32", maxiter=3),
                          raise_on_noconv=False)
    assert st[0]["status"] == "converged" and np.abs(host(X)[0]).max() == 0
    assert st[1]["status"] == "noconv" and st[1]["iters"] <= 3 + 8
    with pytest.raises(pl.LaphNoConvergence):
        lat.solve_raw(dev(b), 0, 1e-10, pl.default_params(inner_prec="f32", maxiter=3))


def test_invalid_gauge_rejected():
    import paper_2510_26313_amd as pl
    dims = (4, 4, 4, 4)
    U = ls.gauge_field(dims, 3)
    U[1, 2, 3, 0, 2] *= 1.0 + 1e-6
    lat = pl.Lattice(dims)
    log_case("invalid_gauge")
    with pytest.raises(pl.LaphError):
        lat.load_gauge(dev(U))


def test_tune_cache_reuse_and_key(tmp_path, monkeypatch):
    """A tuned choice written to the cache is reused by a new context without timing;
    cache lines of another architecture or stencil build are ignored; and the tuned
    shape is no slower than the library's default shape for that batch."""
    import paper_2510_26313_amd as pl
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("LAPH_TUNE_CACHE", str(cache))
    dims = (16, 8, 8, 8)
    U = ls.gauge_field(dims, 44)
    lat = make_lattice(dims, U, masses=(0.05,))
    assert lat.tuned_choice("f16n", 32) is None
    log_case("autotune for the cache", dims=dims)
    t = lat.autotune("f16n", 32, 0)
    lines = cache.read_text().splitlines()
    assert len(lines) == 1 and lines[0].split()[0] == "laph-tune-2" and lines[0].split()[1].startswith("gfx")
    lat2 = make_lattice(dims, U, masses=(0.05,))
    assert lat2.tuned_choice("f16n", 32) == dict(stencil=t["stencil"], rhs_tile=t["rhs_tile"],
                                                 traversal=t["traversal"])
    # the same line with another architecture or another stencil digest is not taken
    f = lines[0].split()
    other = [" ".join(["laph-tune-2", "gfx000"] + f[2:]), " ".join(f[:2] + ["0000000000000000"] + f[3:])]
    cache.write_text("\n".join(other) + "\n")
    lat3 = make_lattice(dims, U, masses=(0.05,))
    assert lat3.tuned_choice("f16n", 32) is None
    # tuned vs the default shape of a 32-RHS F16N batch (LDS links, 16 RHS per load, tile-major)
    best = lambda **kw: min(sum(lat.time_stages("f16n", 32, mass_idx=0, reps=10, **kw)) for _ in range(3))
    log_case("tuned vs default shape")
    tuned = best(rhs_tile=t["rhs_tile"], stencil=t["stencil"], traversal=t["traversal"])
    default = best(rhs_tile=16, stencil=2, traversal=1)
    assert tuned <= 1.05 * default, (tuned, default)
