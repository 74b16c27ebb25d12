"""Pins of the CPU oracle against facts fixed by mathematics, not by the oracle.

Each test names the identity it checks.  Together they are chosen so that a
plausible slip anywhere in the oracle (hop sign or projector, gamma basis,
boundary phase, mass normalisation, a mis-oriented clover leaf, the clover
normalisation or sign, the trace removal, Laplacian sign, projection index
order, sink/source roles, the adjoint used by the gradients, the codec) fails
at least one of them.
"""
import numpy as np
import pytest

import laph_synth as ls
from oracle import codec, dirac, laph, solvers

GAM_LIT = {
    0: np.array([[0, 0, 0, 1j], [0, 0, 1j, 0], [0, -1j, 0, 0], [-1j, 0, 0, 0]]),
    1: np.array([[0, 0, 0, -1], [0, 0, 1, 0], [0, 1, 0, 0], [-1, 0, 0, 0]]),
    2: np.array([[0, 0, 1j, 0], [0, 0, 0, -1j], [-1j, 0, 0, 0], [0, 1j, 0, 0]]),
    3: np.array([[0, 0, 1, 0], [0, 0, 0, 1], [1, 0, 0, 0], [0, 1, 0, 0]]),
}


def _rel(a, b):
    return np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(np.ravel(b)), 1e-300)


# ---------------------------------------------------------------------------
# gamma algebra
# ---------------------------------------------------------------------------

def test_gamma_algebra():
    """Clifford algebra, hermiticity, gamma5 = diag(1,1,-1,-1), sigma block structure."""
    g = dirac.GAMMA
    for mu in range(4):
        assert np.array_equal(g[mu], GAM_LIT[mu])
        assert np.allclose(g[mu], g[mu].conj().T)
        for nu in range(4):
            ac = g[mu] @ g[nu] + g[nu] @ g[mu]
            assert np.allclose(ac, 2 * np.eye(4) * (mu == nu))
    assert np.allclose(dirac.GAMMA5, np.diag([1, 1, -1, -1]))
    for mu, nu in dirac.PLANES:
        s = dirac.sigma(mu, nu)
        assert np.allclose(s, s.conj().T)
        assert np.allclose(s[:2, 2:], 0) and np.allclose(s[2:, :2], 0)
        assert np.allclose(np.sort(np.linalg.eigvalsh(s)), [-1, -1, 1, 1])
    # sigma_xy worked out by hand in this basis
    assert np.allclose(dirac.sigma(0, 1), np.diag([1, -1, 1, -1]))


def test_hop_c_matches_numpy():
    """The C site loop and the whole-field numpy form of H agree (both directions)."""
    dims = (4, 6, 4, 8)
    U = ls.gauge_field(dims, 7)
    psi = ls.random_spinor(ls.spinor_shape(dims, 2), 8)
    for dg in (False, True):
        for ap in (False, True):
            a = dirac.hop(U, psi, ap, dg)
            b = dirac.hop_numpy(U, psi, ap, dg)
            assert _rel(a, b) < 1e-14


# ---------------------------------------------------------------------------
# P2: free field in momentum space
# ---------------------------------------------------------------------------

def _momenta(dims, antiperiodic_t=True):
    lx, ly, lz, lt = dims
    px = 2 * np.pi * np.arange(lx) / lx
    py = 2 * np.pi * np.arange(ly) / ly
    pz = 2 * np.pi * np.arange(lz) / lz
    pt = (2 * np.arange(lt) + (1 if antiperiodic_t else 0)) * np.pi / lt
    return px, py, pz, pt


def _dp(p, m0):
    """D(p) = M(p) + i sum gamma_mu sin p_mu, M(p) = m0 + sum (1 - cos p_mu) (literal gammas)."""
    m = m0 + sum(1 - np.cos(pm) for pm in p)
    return m * np.eye(4) + 1j * sum(GAM_LIT[mu] * np.sin(p[mu]) for mu in range(4))


def test_free_field_plane_wave():
    """At U = 1, D e^{ipx} u = e^{ipx} D(p) u for allowed momenta (non-cubic lattice)."""
    dims = (4, 6, 2, 8)
    lx, ly, lz, lt = dims
    U = ls.unit_gauge(dims)
    m0 = 0.1
    D = dirac.WilsonClover(U, m0, csw=1.0)
    px, py, pz, pt = _momenta(dims)
    t, z, y, x = np.meshgrid(np.arange(lt), np.arange(lz), np.arange(ly), np.arange(lx), indexing="ij")
    rng = np.random.default_rng(0)
    for (ix, iy, iz, it) in [(1, 2, 1, 0), (3, 5, 0, 7), (0, 1, 1, 3)]:
        p = (px[ix], py[iy], pz[iz], pt[it])
        phase = np.exp(1j * (p[0] * x + p[1] * y + p[2] * z + p[3] * t))
        u = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
        psi = phase[..., None, None] * u
        lhs = D.apply(psi[None])[0]
        rhs = phase[..., None, None] * (_dp(p, m0) @ u)
        assert _rel(lhs, rhs) < 1e-13


def test_free_field_propagator_closed_form():
    """P2: x = D^-1 delta (BiCGStab) equals (1/V) sum_p e^{ipx} D(p)^-1 at U = 1."""
    dims = (4, 4, 2, 6)
    lx, ly, lz, lt = dims
    vol = lx * ly * lz * lt
    m0 = 0.1
    D = dirac.WilsonClover(ls.unit_gauge(dims), m0, csw=1.0)
    b = np.zeros(ls.spinor_shape(dims, 12), dtype=np.complex128)
    for s in range(4):
        for a in range(3):
            b[3 * s + a, 0, 0, 0, 0, s, a] = 1.0
    x, info = solvers.bicgstab(D.apply, b, tol=1e-13)
    assert info["true_res"].max() < 1e-12
    px, py, pz, pt = _momenta(dims)
    prop = np.zeros((lt, lz, ly, lx, 4, 4), dtype=np.complex128)
    T, Z, Y, X = np.meshgrid(np.arange(lt), np.arange(lz), np.arange(ly), np.arange(lx), indexing="ij")
    for a in px:
        for bb in py:
            for c in pz:
                for d in pt:
                    sinv = np.linalg.inv(_dp((a, bb, c, d), m0))
                    ph = np.exp(1j * (a * X + bb * Y + c * Z + d * T))
                    prop += ph[..., None, None] * sinv
    prop /= vol
    # x[3*s+a] is column (s, a): x[(s,a)][t,z,y,x][beta, c] = prop[...,beta,s] delta_{ac}
    for s in range(4):
        for a in range(3):
            exp = np.zeros((lt, lz, ly, lx, 4, 3), dtype=np.complex128)
            exp[..., :, a] = prop[..., :, s]
            assert _rel(x[3 * s + a], exp) < 1e-11


# ---------------------------------------------------------------------------
# P3: constant abelian flux -> clover eigenvalues in closed form
# ---------------------------------------------------------------------------

def _flux_field(L, lt, n, diag_phase):
    dims = (L, L, L, lt)
    U = ls.unit_gauge(dims)
    B = 2 * np.pi * n / L ** 2
    for x in range(L):
        U[:, :, :, x, 1] = diag_phase(B * x)
    for y in range(L):
        U[:, :, y, L - 1, 0] = diag_phase(-B * L * y)
    return U, B


def test_clover_constant_flux_eigenvalues():
    """P3(a): E = diag(e^{i phi}, e^{-i phi}, 1) -> eig A = 4+m0 +- (csw/2) sin B (x4), 4+m0 (x4)."""
    def E(phi):
        return np.diag([np.exp(1j * phi), np.exp(-1j * phi), 1.0])
    m0, csw = 0.1, 1.0
    U, B = _flux_field(4, 4, 1, E)
    A = dirac.clover_matrix(U, m0, csw)
    exp = np.sort([4 + m0 + 0.5 * csw * np.sin(B)] * 4 + [4 + m0 - 0.5 * csw * np.sin(B)] * 4
                  + [4 + m0] * 4)
    ev = np.linalg.eigvalsh(A.reshape(-1, 12, 12))
    assert np.abs(np.sort(ev, axis=-1) - exp).max() < 1e-13


def test_clover_constant_flux_traceless_and_sign():
    """P3(b): E = diag(e^{2i phi}, e^{-i phi}, e^{-i phi}) -> A = 4+m0 - (csw/2) sigma_xy (x) diag(f)."""
    def E(phi):
        return np.diag([np.exp(2j * phi), np.exp(-1j * phi), np.exp(-1j * phi)])
    m0, csw = 0.1, 1.0
    U, B = _flux_field(4, 4, 1, E)
    A = dirac.clover_matrix(U, m0, csw)
    s = np.sin(2 * B) + np.sin(B)
    f = np.array([2 * s / 3, -s / 3, -s / 3])
    sig_xy = np.array([1, -1, 1, -1])
    exp = np.diag((4 + m0 - 0.5 * csw * np.outer(sig_xy, f)).ravel())
    assert np.abs(A - exp).max() < 1e-14


def test_clover_chiral_blocks_hermitian():
    """A is Hermitian and chirally block-diagonal for a rough field; A(m0) = A(0) + m0."""
    dims = (4, 4, 4, 4)
    U = ls.gauge_field(dims, 11)
    A = dirac.clover_matrix(U, 0.1, 1.0)
    assert np.abs(A - np.conj(np.swapaxes(A, -1, -2))).max() < 1e-14
    _, _, off = dirac.clover_blocks(A)
    assert off < 1e-15
    A0 = dirac.clover_matrix(U, 0.0, 1.0)
    assert np.abs(A - A0 - 0.1 * np.eye(12)).max() < 1e-14


# ---------------------------------------------------------------------------
# P4: gamma5-hermiticity;  P5: gauge covariance
# ---------------------------------------------------------------------------

def test_gamma5_hermiticity():
    dims = (4, 4, 4, 6)
    U = ls.gauge_field(dims, 12)
    D = dirac.WilsonClover(U, 0.1, 1.0)
    phi = ls.random_spinor(ls.spinor_shape(dims, 1), 13)
    psi = ls.random_spinor(ls.spinor_shape(dims, 1), 14)
    g5 = np.diag(dirac.GAMMA5).real.reshape(4, 1)
    lhs = np.vdot(phi, D.apply(psi))
    rhs = np.vdot(g5 * D.apply(g5 * phi), psi)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)
    # the dagger flag of the hop is gamma5 H gamma5
    assert _rel(D.hop(psi, dagger=True), g5 * D.hop(g5 * psi)) < 1e-15
    # and <phi, D psi> = <D^dagger phi, psi>
    assert abs(np.vdot(D.apply_dagger(phi), psi) - lhs) < 1e-12 * abs(lhs)


def _gauge_transform(U, g):
    Ug = np.empty_like(U)
    for mu in range(4):
        Ug[..., mu, :, :] = g @ U[..., mu, :, :] @ dirac.dag(dirac.site_shift(g, mu, +1))
    return Ug


def test_gauge_covariance_of_D_and_laplacian():
    """P5: U' = g U g(x+mu)^dagger  =>  D' (g psi) = g (D psi); -Delta spectrum invariant."""
    dims = (4, 4, 4, 6)
    U = ls.gauge_field(dims, 15)
    lx, ly, lz, lt = dims
    g = ls.random_su3(lx * ly * lz * lt, 3000).reshape(lt, lz, ly, lx, 3, 3)
    Ug = _gauge_transform(U, g)
    psi = ls.random_spinor(ls.spinor_shape(dims, 1), 16)
    D = dirac.WilsonClover(U, 0.1, 1.0)
    Dg = dirac.WilsonClover(Ug, 0.1, 1.0)
    gpsi = np.matmul(g[:, :, :, :, None], psi[..., None])[..., 0]
    lhs = Dg.apply(gpsi)
    rhs = np.matmul(g[:, :, :, :, None], D.apply(psi)[..., None])[..., 0]
    assert _rel(lhs, rhs) < 1e-13
    w1 = np.linalg.eigvalsh(laph.neg_laplacian_dense(U[2]))
    w2 = np.linalg.eigvalsh(laph.neg_laplacian_dense(Ug[2]))
    assert np.abs(w1 - w2).max() < 1e-12


def test_perambulator_gauge_invariance():
    """P5 on tau: V' = g V, U' = g U g^dagger leave tau unchanged."""
    dims = (4, 4, 4, 4)
    lx, ly, lz, lt = dims
    U = ls.gauge_field(dims, 17)
    V = ls.orthonormal_laph_vectors(dims, 3, 18)
    g = ls.random_su3(lx * ly * lz * lt, 3000).reshape(lt, lz, ly, lx, 3, 3)
    Ug = _gauge_transform(U, g)
    Vg = np.matmul(g[:, None], V[..., None])[..., 0]
    tau, _ = laph.perambulator(U, V, 1, 0.1, tol=1e-13)
    taug, _ = laph.perambulator(Ug, Vg, 1, 0.1, tol=1e-13)
    assert _rel(taug, tau) < 1e-11


# ---------------------------------------------------------------------------
# P1: dense inverse;  P6: Schur identity
# ---------------------------------------------------------------------------

def test_dense_inverse_c0():
    """P1: BiCGStab on the 4^4 lattice and LapH sources agrees with LU of the dense 3072^2 D."""
    cfg = ls.CONFIGS["dense_4x4x4x4"]
    U = ls.gauge_field(cfg["dims"], cfg["seed_u"])
    V, lam, gap = laph.laplacian_eigvecs(U, cfg["nev"])
    assert gap.min() > 0
    D = dirac.WilsonClover(U, cfg["masses"][0], cfg["csw"])
    b = laph.laph_sources(V, 0)
    x_dense = solvers.dense_solve(D, b)
    x_it, info = solvers.bicgstab(D.apply, b, tol=1e-13)
    assert info["true_res"].max() < 1e-12
    for r in range(b.shape[0]):
        assert _rel(x_it[r], x_dense[r]) < 1e-12
    assert _rel(D.apply(x_dense), b) < 1e-13


def test_schur_identity():
    """P6: even-odd route (M_hat x_e = b_hat, then x_o) reproduces the full solve."""
    dims = (4, 4, 4, 4)
    U = ls.gauge_field(dims, 19)
    D = dirac.WilsonClover(U, 0.05, 1.0)
    eo = dirac.EvenOdd(D)
    b = ls.random_spinor(ls.spinor_shape(dims, 2), 20)
    x_full, _ = solvers.bicgstab(D.apply, b, tol=1e-13)
    bh = eo.prepare(b)
    xe, info = solvers.bicgstab(eo.M_hat, bh, tol=1e-14)
    x = eo.reconstruct(b, xe)
    assert _rel(x, x_full) < 1e-12
    # and the operator identity on an arbitrary even field:
    # e * D(x_e + x_o(x_e)) = A_ee M_hat x_e (with b = 0 reconstruction)
    ve = eo.e * ls.random_spinor(ls.spinor_shape(dims, 1), 21)
    full = eo.reconstruct(np.zeros_like(ve), ve)
    lhs = eo.e * D.apply(full)
    rhs = eo.e * dirac.apply_site_matrix(D.A, eo.M_hat(ve))
    assert _rel(lhs, rhs) < 1e-13


# ---------------------------------------------------------------------------
# P7: perambulator gamma5 reciprocity
# ---------------------------------------------------------------------------

def test_perambulator_reciprocity():
    """tau^(src t0)[t][l][k][b][a] = g5_b g5_a conj(tau^(src t)[t0][k][l][a][b])."""
    dims = (4, 4, 4, 4)
    U = ls.gauge_field(dims, 1000)
    V, _, _ = laph.laplacian_eigvecs(U, 8)
    tauA, _ = laph.perambulator(U, V, 0, 0.1, method="dense")
    tauB, _ = laph.perambulator(U, V, 2, 0.1, method="dense")
    g5 = np.diag(dirac.GAMMA5).real
    lhs = tauA[2]                                        # source t0=0, sink t=2
    rhs = np.einsum("b,a,klab->lkba", g5, g5, np.conj(tauB[0]))
    assert _rel(lhs, rhs) < 1e-12


# ---------------------------------------------------------------------------
# P8: free Laplacian spectrum;  LapH eigenvector conventions
# ---------------------------------------------------------------------------

def test_free_laplacian_spectrum():
    dims = (4, 6, 2, 2)
    lx, ly, lz, lt = dims
    U = ls.unit_gauge(dims)
    w = np.linalg.eigvalsh(laph.neg_laplacian_dense(U[0]))
    ks = [2 * np.pi * np.arange(n) / n for n in (lx, ly, lz)]
    lam = [sum(2 - 2 * np.cos(k) for k in (a, b, c)) for a in ks[0] for b in ks[1] for c in ks[2]]
    exp = np.sort(np.repeat(lam, 3))
    assert np.abs(w - exp).max() < 1e-12
    # the spectrum alone is blind to p -> p + pi; the eigenvectors are not:
    # a plane wave e^{ipx} has eigenvalue sum_k (2 - 2 cos p_k), the constant field 0
    Z, Y, X = np.meshgrid(np.arange(lz), np.arange(ly), np.arange(lx), indexing="ij")
    for (a, b, c) in [(0, 0, 0), (1, 2, 1), (3, 5, 0)]:
        p = (ks[0][a], ks[1][b], ks[2][c])
        f = np.zeros((lz, ly, lx, 3), dtype=np.complex128)
        f[..., 1] = np.exp(1j * (p[0] * X + p[1] * Y + p[2] * Z))
        lam_p = sum(2 - 2 * np.cos(k) for k in p)
        assert np.abs(laph.neg_laplacian_apply(U[0], f) - lam_p * f).max() < 1e-12


def test_laplacian_eigvecs_c0():
    """Orthonormal, eigen-residual small, ascending, phase convention applied."""
    cfg = ls.CONFIGS["dense_4x4x4x4"]
    U = ls.gauge_field(cfg["dims"], cfg["seed_u"])
    V, lam, gap = laph.laplacian_eigvecs(U, cfg["nev"])
    lt = U.shape[0]
    for t in range(lt):
        q = V[t].reshape(cfg["nev"], -1)
        assert np.abs(q.conj() @ q.T - np.eye(cfg["nev"])).max() < 1e-13
        assert np.all(np.diff(lam[t]) >= -1e-14)
        res = laph.neg_laplacian_apply(U[t], V[t]) - lam[t][:, None, None, None, None] * V[t]
        assert np.abs(res).max() < 1e-12
        for l in range(cfg["nev"]):
            v = q[l]
            i = np.argmax(np.abs(v))
            assert abs(v[i].imag) < 1e-14 and v[i].real > 0


# ---------------------------------------------------------------------------
# P9: free-field perambulator with plane-wave LapH vectors, and d tau / d m0
# ---------------------------------------------------------------------------

def test_free_field_perambulator_and_mass_derivative():
    dims = (4, 4, 2, 6)
    lx, ly, lz, lt = dims
    m0 = 0.2
    t0 = 1
    U = ls.unit_gauge(dims)
    px, py, pz, pt = _momenta(dims)
    moms = [(0, 0, 0), (1, 1, 1), (3, 1, 0)]   # nonzero sin p_y makes tau complex
    Z, Y, X = np.meshgrid(np.arange(lz), np.arange(ly), np.arange(lx), indexing="ij")
    vecs = []
    for (a, b, c) in moms:
        ph = np.exp(1j * (px[a] * X + py[b] * Y + pz[c] * Z)) / np.sqrt(lx * ly * lz)
        for col in range(3):
            f = np.zeros((lz, ly, lx, 3), dtype=np.complex128)
            f[..., col] = ph
            vecs.append(f)
    nev = len(vecs)
    V = np.broadcast_to(np.array(vecs)[None], (lt, nev, lz, ly, lx, 3)).copy()
    tau, Xs = laph.perambulator(U, V, t0, m0, method="dense")
    D = dirac.WilsonClover(U, m0, 1.0)
    dX = solvers.dense_solve(D, -Xs)                        # dX/dm0 = -D^-1 X
    dtau = laph.project(V, dX, nev)
    for t in range(lt):
        for i, (a, b, c) in enumerate(moms):
            S = [np.linalg.inv(_dp((px[a], py[b], pz[c], p4), m0)) for p4 in pt]
            ex = sum(np.exp(1j * p4 * (t - t0)) * s for p4, s in zip(pt, S)) / lt
            dex = -sum(np.exp(1j * p4 * (t - t0)) * s @ s for p4, s in zip(pt, S)) / lt
            for col in range(3):
                l = 3 * i + col
                assert np.abs(tau[t, l, l] - ex).max() < 1e-11
                assert np.abs(dtau[t, l, l] - dex).max() < 1e-11
        # off-diagonal (momentum or colour mismatch) vanishes
        mask = ~np.eye(nev, dtype=bool)
        assert np.abs(tau[t][mask]).max() < 1e-11


# ---------------------------------------------------------------------------
# P10: adjoint gradients against central finite differences
# ---------------------------------------------------------------------------

def test_adjoint_gradients_vs_fd():
    dims = (4, 4, 4, 4)
    U = ls.gauge_field(dims, 1003)
    V = ls.orthonormal_laph_vectors(dims, 3, 2003)
    m0, csw, ts = 0.05, 1.0, 2
    D = dirac.WilsonClover(U, m0, csw)
    b = laph.laph_sources(V, 0)
    L, gb, gm, _ = laph.adjoint_gradients(D, V, b, ts)
    fd_m = laph.fd_mass(U, V, b, m0, csw, ts)
    assert abs(gm - fd_m) <= 1e-5 * abs(fd_m)
    rng = np.random.default_rng(4000)
    d = rng.standard_normal(b.shape) + 1j * rng.standard_normal(b.shape)
    d /= np.linalg.norm(d)
    fd_b = laph.fd_source(D, V, b, d, ts)
    an_b = float(np.real(np.vdot(gb, d)))
    assert abs(an_b - fd_b) <= 1e-5 * max(abs(fd_b), 1e-3 * np.abs(gb).max())


# ---------------------------------------------------------------------------
# P11: projection index order against a brute-force loop
# ---------------------------------------------------------------------------

def test_projection_bruteforce():
    dims = (2, 2, 2, 4)
    lx, ly, lz, lt = dims
    nev = 2
    V = ls.orthonormal_laph_vectors(dims, nev, 5)
    X = ls.random_spinor(ls.spinor_shape(dims, 4 * nev), 6)
    tau = laph.project(V, X, nev)
    for t in range(lt):
        for l in range(nev):
            for k in range(nev):
                for be in range(4):
                    for al in range(4):
                        acc = 0
                        for z in range(lz):
                            for y in range(ly):
                                for x in range(lx):
                                    for a in range(3):
                                        acc += np.conj(V[t, l, z, y, x, a]) * X[4 * k + al, t, z, y, x, be, a]
                        assert abs(tau[t, l, k, be, al] - acc) < 1e-14


def test_sources_layout():
    dims = (2, 2, 2, 4)
    V = ls.orthonormal_laph_vectors(dims, 2, 5)
    b = laph.laph_sources(V, 3)
    assert b.shape == (8, 4, 2, 2, 2, 4, 3)
    assert np.allclose(np.linalg.norm(b.reshape(8, -1), axis=1), 1.0)
    assert np.array_equal(b[4 * 1 + 2, 3, :, :, :, 2, :], V[3, 1])
    assert np.abs(b[4 * 1 + 2, :3]).max() == 0 and np.abs(b[4 * 1 + 2, 3, ..., 0, :]).max() == 0


# ---------------------------------------------------------------------------
# meson doublets and baryon triplets of the LapH vectors
# ---------------------------------------------------------------------------

# eps_abc written out: even permutations of (0, 1, 2) +1, odd ones -1
EPS_LIT = {(0, 1, 2): 1, (1, 2, 0): 1, (2, 0, 1): 1, (0, 2, 1): -1, (2, 1, 0): -1, (1, 0, 2): -1}

PW_MODES = [((0, 0, 0), 0), ((1, 0, 0), 1), ((0, 1, 0), 2), ((1, 1, 0), 0), ((3, 0, 0), 1), ((0, 0, 1), 2),
            ((2, 3, 1), 1), ((0, 0, 0), 2), ((3, 3, 3), 0)]
PW_MOMS = [(0, 0, 0), (1, 0, 0), (1, 1, 0), (0, 3, 1), (-1, 0, 2), (3, 2, 1)]


def _plane_wave_vectors(dims, modes):
    """V_j(x, t) = exp(+2 pi i k_j . x / L) e_{c_j} / sqrt(Lx Ly Lz) on every timeslice."""
    lx, ly, lz, lt = dims
    z, y, x = np.meshgrid(np.arange(lz), np.arange(ly), np.arange(lx), indexing="ij")
    V = np.zeros((lt, len(modes), lz, ly, lx, 3), dtype=np.complex128)
    for j, ((kx, ky, kz), c) in enumerate(modes):
        V[:, j, :, :, :, c] = np.exp(2j * np.pi * (kx * x / lx + ky * y / ly + kz * z / lz)) / np.sqrt(lx * ly * lz)
    return V


def test_doublets_triplets_free_plane_waves():
    """Plane-wave colour vectors give closed forms (momenta mod L):
    Phi_p[j][j'] = delta_{c c'} delta(k' - k = p),
    B_p[j1][j2][j3] = eps_{c1 c2 c3} (L^3)^(-1/2) delta(k1 + k2 + k3 = p)."""
    L = 4
    dims = (L, L, L, 2)
    V = _plane_wave_vectors(dims, PW_MODES)
    phi = laph.meson_doublets(V, PW_MOMS)
    B = laph.baryon_triplets(V, PW_MOMS)
    assert phi.shape == (len(PW_MOMS), 2, len(PW_MODES), len(PW_MODES))
    assert B.shape == (len(PW_MOMS), 2) + (len(PW_MODES),) * 3

    def same(q, r):
        return all((q[d] - r[d]) % L == 0 for d in range(3))

    for ip, p in enumerate(PW_MOMS):
        for j, (k, c) in enumerate(PW_MODES):
            for jj, (kk, cc) in enumerate(PW_MODES):
                want = float(c == cc and same([kk[d] - k[d] for d in range(3)], p))
                assert np.abs(phi[ip, :, j, jj] - want).max() < 1e-13
        for j1, (k1, c1) in enumerate(PW_MODES):
            for j2, (k2, c2) in enumerate(PW_MODES):
                for j3, (k3, c3) in enumerate(PW_MODES):
                    ksum = [k1[d] + k2[d] + k3[d] for d in range(3)]
                    want = EPS_LIT.get((c1, c2, c3), 0) / L ** 1.5 if same(ksum, p) else 0.0
                    assert np.abs(B[ip, :, j1, j2, j3] - want).max() < 1e-13


def test_doublets_zero_momentum_identity():
    """Phi at p = 0 of orthonormal vectors is the identity on every timeslice."""
    dims = (4, 4, 2, 3)
    lx, ly, lz, lt = dims
    rng = np.random.default_rng(52)
    V = np.empty((lt, 6, lz, ly, lx, 3), dtype=np.complex128)
    for t in range(lt):
        q, _ = np.linalg.qr(rng.standard_normal((3 * lx * ly * lz, 6)) + 1j * rng.standard_normal((3 * lx * ly * lz, 6)))
        V[t] = q.T.reshape(6, lz, ly, lx, 3)
    phi = laph.meson_doublets(V, [(0, 0, 0)])
    assert np.abs(phi[0] - np.eye(6)[None]).max() < 1e-13


def test_doublets_triplets_gauge_invariance():
    """V -> g V with g(x) in SU(3): doublets (g^dagger g = 1) and triplets (det g = 1) unchanged."""
    dims = (4, 2, 2, 3)
    lx, ly, lz, lt = dims
    V = ls.random_spinor((lt, 5, lz, ly, lx, 3), 53)
    g = ls.random_su3(lx * ly * lz * lt, 54).reshape(lt, lz, ly, lx, 3, 3)
    Vg = np.matmul(g[:, None], V[..., None])[..., 0]
    moms = [(0, 0, 0), (1, 0, 1), (0, -1, 0)]
    assert _rel(laph.meson_doublets(Vg, moms), laph.meson_doublets(V, moms)) < 1e-13
    assert _rel(laph.baryon_triplets(Vg, moms), laph.baryon_triplets(V, moms)) < 1e-13


def test_triplet_integrand_is_determinant():
    """eps_abc u_a v_b w_c = det[u v w]: the triplet against numpy's determinant per site."""
    dims = (2, 4, 2, 2)
    lx, ly, lz, lt = dims
    V = ls.random_spinor((lt, 4, lz, ly, lx, 3), 55)
    mom = (1, 1, 1)
    B = laph.baryon_triplets(V, [mom])
    for t in range(lt):
        for l, m, n in ((0, 1, 2), (3, 1, 0), (2, 3, 1)):
            acc = 0
            for z in range(lz):
                for y in range(ly):
                    for x in range(lx):
                        ph = np.exp(-2j * np.pi * (x / lx + y / ly + z / lz))
                        acc += ph * np.linalg.det(np.stack([V[t, l, z, y, x], V[t, m, z, y, x], V[t, n, z, y, x]], 1))
            assert abs(B[0, t, l, m, n] - acc) < 1e-13 * max(1.0, abs(acc))


def test_doublets_momentum_reversal_and_triplet_antisymmetry():
    """Phi_{-p}[m][l] = conj(Phi_p[l][m]); B changes sign under any swap of two indices."""
    dims = (4, 2, 2, 2)
    lx, ly, lz, lt = dims
    V = ls.random_spinor((lt, 4, lz, ly, lx, 3), 56)
    phi = laph.meson_doublets(V, [(1, 0, 1), (-1, 0, -1)])
    assert _rel(phi[1], np.conj(phi[0]).transpose(0, 2, 1)) < 1e-14
    B = laph.baryon_triplets(V, [(0, 1, 0)])
    for perm in ((0, 1, 3, 2, 4), (0, 1, 2, 4, 3), (0, 1, 4, 3, 2)):
        assert _rel(B.transpose(perm), -B) < 1e-14


# ---------------------------------------------------------------------------
# stochastic LapH: noise-diluted sources
# ---------------------------------------------------------------------------

def test_noise_sources_full_dilution_are_laph_sources():
    """n_dil = nev and rho = 1: the diluted noise sources are the perambulator's sources."""
    dims = (2, 2, 2, 4)
    V = ls.orthonormal_laph_vectors(dims, 3, 61)
    b = laph.noise_sources(V, 2, np.ones((4, 3), dtype=np.complex128), 3)
    assert np.array_equal(b, laph.laph_sources(V, 2))


def test_stochastic_perambulator_is_noise_weighted_perambulator():
    """D^-1 is linear: phi[t][l][j][beta][alpha] = sum_{k = j mod n_dil} tau[t][l][k][beta][alpha] rho[alpha][k]
    (interlaced LapH dilution, full spin and time dilution; Z4 noise)."""
    dims = (4, 4, 4, 4)
    nev, n_dil, t0, m0 = 5, 2, 1, 0.1
    U = ls.gauge_field(dims, 62)
    V = ls.orthonormal_laph_vectors(dims, nev, 63)
    rng = np.random.default_rng(64)
    rho = np.exp(0.5j * np.pi * rng.integers(0, 4, size=(4, nev)))
    tau, _ = laph.perambulator(U, V, t0, m0, method="dense")
    phi, _ = laph.stochastic_perambulator(U, V, t0, m0, rho, n_dil, method="dense")
    assert phi.shape == (dims[3], nev, n_dil, 4, 4)
    want = np.zeros_like(phi)
    for j in range(n_dil):
        for k in range(nev):
            if k % n_dil == j:
                want[:, :, j] += tau[:, :, k] * rho[None, None, None, :, k]
    assert _rel(phi, want) < 1e-12


# ---------------------------------------------------------------------------
# spin basis of the perambulator
# ---------------------------------------------------------------------------

def test_spin_rotate_equals_rotating_sources_and_solutions():
    """tau in the basis psi' = S psi, two routes: S tau S^dagger, against sources built from
    the new basis vectors (old components conj(S[alpha'][alpha])), solved, their solutions
    rotated by S and projected."""
    dims = (4, 4, 4, 4)
    nev, t0, m0 = 2, 1, 0.1
    U = ls.gauge_field(dims, 81)
    V = ls.orthonormal_laph_vectors(dims, nev, 82)
    rng = np.random.default_rng(83)
    S, _ = np.linalg.qr(rng.standard_normal((4, 4)) + 1j * rng.standard_normal((4, 4)))
    tau, _ = laph.perambulator(U, V, t0, m0, method="dense")
    D = dirac.WilsonClover(U, m0, 1.0)
    b = np.zeros((4 * nev, dims[3], dims[2], dims[1], dims[0], 4, 3), dtype=np.complex128)
    for k in range(nev):
        for ap in range(4):
            for al in range(4):
                b[4 * k + ap, t0, :, :, :, al, :] = np.conj(S[ap, al]) * V[t0, k]
    X = solvers.dense_solve(D, b)
    Xs = np.einsum("ab,r...bc->r...ac", S, X)
    assert _rel(laph.spin_rotate(tau, S), laph.project(V, Xs, nev)) < 1e-12
    assert _rel(laph.spin_rotate(laph.spin_rotate(tau, S), np.conj(S.T)), tau) < 1e-14


# ---------------------------------------------------------------------------
# P13: FP16-with-norm codec
# ---------------------------------------------------------------------------

def test_codec_bound_and_zero():
    rng = np.random.default_rng(1)
    v = rng.standard_normal((1000, 24)) * np.exp(rng.uniform(-20, 20, (1000, 1)))
    v[3] = 0.0
    q, n = codec.encode(v)
    w = codec.decode(q, n)
    err = np.abs(v.astype(np.float32).astype(np.float64) - w.astype(np.float64))
    assert np.all(err <= codec.error_bound(n.astype(np.float64))[:, None])
    assert np.all(w[3] == 0) and n[3] == 0
    # the largest component is coded as +-1 exactly
    i = np.argmax(np.abs(v[0]))
    assert abs(float(q[0, i])) == 1.0


def test_sampled_sites_match_full_operator():
    """The one-site form of D (used for sampled checks at large sizes) equals the full operator."""
    dims = (4, 6, 4, 6)
    U = ls.gauge_field(dims, 23)
    psi = ls.random_spinor(ls.spinor_shape(dims, 2), 24)
    D = dirac.WilsonClover(U, 0.02, 1.0)
    full = D.apply(psi)
    fulld = D.apply_dagger(psi)
    sites = [(0, 0, 0, 0), (5, 3, 5, 3), (2, 1, 4, 0), (5, 0, 0, 3)]
    got = dirac.apply_at_sites(U, psi, sites, 0.02, 1.0)
    gotd = dirac.apply_at_sites(U, psi, sites, 0.02, 1.0, dagger=True)
    for i, (t, z, y, x) in enumerate(sites):
        assert np.abs(got[:, i] - full[:, t, z, y, x]).max() < 1e-13
        assert np.abs(gotd[:, i] - fulld[:, t, z, y, x]).max() < 1e-13


def test_sampled_hop_and_clover_inverse_match_full_fields():
    """The one-site hop (a Python loop over the 8 neighbours) equals the plain-C
    whole-field hop at every site, dagger included, with the antiperiodic wrap;
    the one-site clover inverse equals the whole-field inverse."""
    dims = (4, 6, 4, 6)
    U = ls.gauge_field(dims, 25)
    psi = ls.random_spinor(ls.spinor_shape(dims, 2), 26)
    lx, ly, lz, lt = dims
    sites = [(t, z, y, x) for t in range(lt) for z in range(lz) for y in range(ly) for x in range(lx)]
    for dag in (False, True):
        got = dirac.hop_at_sites(U, psi, sites, dagger=dag)
        full = dirac.hop(U, psi, True, dag)
        exp = np.stack([full[:, t, z, y, x] for (t, z, y, x) in sites], axis=1)
        assert np.abs(got - exp).max() < 1e-13
    Ai = dirac.clover_inverse(dirac.clover_matrix(U, 0.05, 1.0))
    for (t, z, y, x) in [(0, 0, 0, 0), (5, 3, 5, 3), (2, 1, 4, 0)]:
        assert np.abs(dirac.clover_inverse_at(U, (t, z, y, x), 0.05, 1.0) - Ai[t, z, y, x]).max() < 1e-14
