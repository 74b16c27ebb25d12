"""Plant plausible mistakes in the CPU oracle and check that a pin catches each.

Each case patches one oracle function with a wrong variant (wrong projector
sign, missing boundary phase, wrong mass normalisation, no trace removal,
flipped clover sign, a leaf built from the wrong links, a reversed leaf, a
Laplacian sign slip, a conjugate on the wrong factor of the projection, a
missing gamma5 in the adjoint, the doublets' conjugate or phase sign, a triplet
epsilon sign or a conjugated triplet factor, blocked instead of interlaced noise
dilution, noise of the wrong spin, a spin rotation by S^T instead of S^dagger;
for the multigrid: a restriction without the conjugate, Gram-Schmidt without the
projections or across chiralities, a coarse matrix of D^dagger, a smoother that
reconstructs with the wrong sign, a coarse BiCGStab with a conjugated omega) and
asserts that the named pin now fails.
Everything runs on the CPU; nothing here touches the GPU library.
"""
import numpy as np
import pytest

from oracle import dirac, laph
from oracle import multigrid as omg
import test_oracle_mg as mgpins
import test_oracle_pins as pins

_orig_hop = dirac.hop
_orig_fs = dirac.field_strength
_orig_ps = dirac.plaquette_sum
_orig_ct = dirac.clover_term


def _hop_flipped(U, psi, antiperiodic_t=True, dagger=False):
    return _orig_hop(U, psi, antiperiodic_t, not dagger)


def _hop_periodic(U, psi, antiperiodic_t=True, dagger=False):
    return _orig_hop(U, psi, False, dagger)


def _fs_no_trace(U, mu, nu):
    q = dirac.plaquette_sum(U, mu, nu)
    return (q - dirac.dag(q)) / 8.0


def _ct_flipped(U, csw):
    return -_orig_ct(U, csw)


def _ps_wrong_link(U, mu, nu):
    um, un = U[..., mu, :, :], U[..., nu, :, :]
    s = dirac.site_shift
    dag = dirac.dag
    um_m = s(um, mu, -1)
    un_n = s(un, nu, -1)
    leaf1 = um @ s(un, mu, +1) @ dag(s(um, nu, +1)) @ dag(un)
    leaf2 = un @ dag(s(um, nu, +1)) @ dag(s(un, mu, -1)) @ um_m      # U_mu(x+nu): wrong site
    leaf3 = dag(um_m) @ dag(s(un_n, mu, -1)) @ s(um_m, nu, -1) @ un_n
    leaf4 = dag(un_n) @ s(um, nu, -1) @ s(un_n, mu, +1) @ dag(um)
    return leaf1 + leaf2 + leaf3 + leaf4


def _ps_reversed_leaf(U, mu, nu):
    um, un = U[..., mu, :, :], U[..., nu, :, :]
    s = dirac.site_shift
    dag = dirac.dag
    leaf1 = um @ s(un, mu, +1) @ dag(s(um, nu, +1)) @ dag(un)
    q = _orig_ps(U, mu, nu)
    return q - leaf1 + dag(leaf1)


class _WrongMass(dirac.WilsonClover):
    def __init__(self, U, m0, csw=1.0, antiperiodic_t=True):
        super().__init__(U, 2 * m0, csw, antiperiodic_t)


def _neg_lap_wrong_sign(U3, f):
    out = 6.0 * f
    for k in range(3):
        ax = -2 - k
        uk = U3[..., k, :, :]
        ub = np.roll(uk, +1, axis=-3 - k)
        out = out + np.matmul(uk, np.roll(f, -1, axis=ax)[..., None])[..., 0]
        out = out + np.matmul(dirac.dag(ub), np.roll(f, +1, axis=ax)[..., None])[..., 0]
    return out


def _project_conj_x(V, X, nev_src):
    lt, nev, lz, ly, lx, _ = V.shape
    Xr = X.reshape(nev_src, 4, lt, lz, ly, lx, 4, 3)
    return np.einsum("tlzyxa,kctzyxba->tlkbc", V, np.conj(Xr))


def _adjoint_no_g5(D, V, b, t_sink, tol=1e-13):
    from oracle.solvers import bicgstab
    L, X, tau = laph.loss_of_sources(D, V, b, t_sink, tol)
    gx = laph.tau_cotangent_to_X(V, 2.0 * tau[t_sink], t_sink, X.shape)
    Z, _ = bicgstab(D.apply, gx, tol=tol)
    return L, Z, -float(np.sum(np.real(np.conj(Z) * X))), X


def _doublets_no_conj(V, moms):
    lt, nev, lz, ly, lx, _ = V.shape
    ph = laph.momentum_phases((lx, ly, lz), moms)
    return np.einsum("pzyx,tlzyxa,tmzyxa->ptlm", ph, V, V)


def _doublets_phase_sign(V, moms):
    lt, nev, lz, ly, lx, _ = V.shape
    ph = np.conj(laph.momentum_phases((lx, ly, lz), moms))
    return np.einsum("pzyx,tlzyxa,tmzyxa->ptlm", ph, np.conj(V), V)


def _triplets_one_eps_sign(V, moms):
    lt, nev, lz, ly, lx, _ = V.shape
    ph = laph.momentum_phases((lx, ly, lz), moms)
    eps = laph.levi_civita()
    eps[2, 0, 1] = -1.0
    return np.einsum("pzyx,abc,tlzyxa,tmzyxb,tnzyxc->ptlmn", ph, eps, V, V, V)


def _triplets_conj_first(V, moms):
    lt, nev, lz, ly, lx, _ = V.shape
    ph = laph.momentum_phases((lx, ly, lz), moms)
    return np.einsum("pzyx,abc,tlzyxa,tmzyxb,tnzyxc->ptlmn", ph, laph.levi_civita(), np.conj(V), V, V)


def _noise_sources_blocked(V, t0, rho, n_dil):
    lt, nev, lz, ly, lx, _ = V.shape
    b = np.zeros((4 * n_dil, lt, lz, ly, lx, 4, 3), dtype=np.complex128)
    per = -(-nev // n_dil)
    for k in range(nev):
        for alpha in range(4):
            b[4 * (k // per) + alpha, t0, :, :, :, alpha, :] += rho[alpha, k] * V[t0, k]
    return b


def _noise_sources_wrong_spin(V, t0, rho, n_dil):
    lt, nev, lz, ly, lx, _ = V.shape
    b = np.zeros((4 * n_dil, lt, lz, ly, lx, 4, 3), dtype=np.complex128)
    for j in range(n_dil):
        for alpha in range(4):
            for k in range(j, nev, n_dil):
                b[4 * j + alpha, t0, :, :, :, alpha, :] += rho[0, k] * V[t0, k]
    return b


def _spin_rotate_transpose(tau, S):
    return np.einsum("ab,...bc,cd->...ad", S, tau, S.T)


def _restrict_no_conj(basis, f, dims, block):
    wb = omg._to_blocks(basis, dims, block)
    fb = omg._to_blocks(f, dims, block)
    return np.einsum("itzyxcm,ntzyxcm->ntzyxci", wb, fb)


def _orth_no_projection(vecs, dims, block):
    g = omg._to_blocks(np.asarray(vecs, dtype=np.complex128), dims, block)
    w = g / np.sqrt(np.sum(np.abs(g) ** 2, axis=-1, keepdims=True))
    return omg._from_blocks(w, dims, block)


def _orth_whole_spinor(vecs, dims, block):
    # Gram-Schmidt over both chiralities at once (a non-chiral basis)
    g = omg._to_blocks(np.asarray(vecs, dtype=np.complex128), dims, block)
    sh = g.shape
    h = g.reshape(sh[:-2] + (2 * sh[-1],))
    w = np.array(h)
    for i in range(w.shape[0]):
        for j in range(i):
            w[i] = w[i] - np.sum(np.conj(w[j]) * w[i], axis=-1, keepdims=True) * w[j]
        w[i] = w[i] / np.sqrt(np.sum(np.abs(w[i]) ** 2, axis=-1, keepdims=True))
    return omg._from_blocks(w.reshape(sh), dims, block)


class _DaggerD:
    def __init__(self, D):
        self.D = D
        self.dims = D.dims

    def apply(self, psi):
        return self.D.apply_dagger(psi)


_orig_coarse_dense = omg.coarse_dense


def _coarse_dense_dagger(D, basis, block):
    return _orig_coarse_dense(_DaggerD(D), basis, block)


def _smoother_wrong_reconstruction(D, r, iters):
    e, rho = _orig_smoother(D, r, iters)
    eo = dirac.EvenOdd(D)
    e_e = eo.e * e
    e_o = eo.o * eo.Ainv(eo.o * r - 0.5 * eo.o * D.hop(e_e))
    return e_e + e_o, rho


_orig_smoother = omg.smoother


def _coarse_bicgstab_conj_omega(Dc, b, iters, tol):
    x = np.zeros_like(b)
    r = b.copy()
    rh = b.copy()
    p = np.zeros_like(b)
    v = np.zeros_like(b)
    rho = alpha = omega = 1.0
    for _ in range(iters):
        rn = np.vdot(rh, r)
        beta = (rn / rho) * (alpha / omega)
        rho = rn
        p = r + beta * (p - omega * v)
        v = Dc @ p
        alpha = rho / np.vdot(rh, v)
        s = r - alpha * v
        t = Dc @ s
        omega = np.conj(np.vdot(t, s) / np.vdot(t, t).real)
        x = x + alpha * p + omega * s
        r = s - omega * t
    return x


CASES = [
    ("hop projector sign", dirac, "hop", _hop_flipped, pins.test_free_field_plane_wave),
    ("no antiperiodic phase", dirac, "hop", _hop_periodic, pins.test_free_field_propagator_closed_form),
    ("mass normalisation", dirac, "WilsonClover", _WrongMass, pins.test_free_field_plane_wave),
    ("no trace removal", dirac, "field_strength", _fs_no_trace, pins.test_clover_constant_flux_traceless_and_sign),
    ("clover sign", dirac, "clover_term", _ct_flipped, pins.test_clover_constant_flux_traceless_and_sign),
    ("leaf from wrong link", dirac, "plaquette_sum", _ps_wrong_link, pins.test_gauge_covariance_of_D_and_laplacian),
    ("reversed leaf", dirac, "plaquette_sum", _ps_reversed_leaf, pins.test_clover_constant_flux_eigenvalues),
    ("laplacian sign", laph, "neg_laplacian_apply", _neg_lap_wrong_sign, pins.test_free_laplacian_spectrum),
    ("projection conjugate", laph, "project", _project_conj_x, pins.test_free_field_perambulator_and_mass_derivative),
    ("adjoint without gamma5", laph, "adjoint_gradients", _adjoint_no_g5, pins.test_adjoint_gradients_vs_fd),
    ("doublet without conjugate", laph, "meson_doublets", _doublets_no_conj, pins.test_doublets_zero_momentum_identity),
    ("doublet phase sign", laph, "meson_doublets", _doublets_phase_sign, pins.test_doublets_triplets_free_plane_waves),
    ("triplet epsilon sign", laph, "baryon_triplets", _triplets_one_eps_sign,
     pins.test_doublets_triplets_gauge_invariance),
    ("triplet conjugated factor", laph, "baryon_triplets", _triplets_conj_first,
     pins.test_doublets_triplets_gauge_invariance),
    ("blocked instead of interlaced dilution", laph, "noise_sources", _noise_sources_blocked,
     pins.test_stochastic_perambulator_is_noise_weighted_perambulator),
    ("noise of the wrong spin", laph, "noise_sources", _noise_sources_wrong_spin,
     pins.test_stochastic_perambulator_is_noise_weighted_perambulator),
    ("spin rotation by S^T instead of S^dagger", laph, "spin_rotate", _spin_rotate_transpose,
     pins.test_spin_rotate_equals_rotating_sources_and_solutions),
    ("restriction without the conjugate", omg, "restrict", _restrict_no_conj, mgpins.test_restrict_is_adjoint_of_prolong),
    ("Gram-Schmidt without projections", omg, "block_orthonormalize", _orth_no_projection,
     mgpins.test_basis_orthonormal_and_spanning),
    ("Gram-Schmidt across chiralities", omg, "block_orthonormalize", _orth_whole_spinor,
     mgpins.test_basis_orthonormal_and_spanning),
    ("coarse matrix of D^dagger", omg, "coarse_dense", _coarse_dense_dagger,
     mgpins.test_galerkin_orthogonality_and_gamma5),
    ("smoother reconstructs with the wrong sign", omg, "smoother", _smoother_wrong_reconstruction,
     mgpins.test_smoother_residual_identity_and_monotone_mr),
    ("coarse BiCGStab with a conjugated omega", omg, "coarse_bicgstab", _coarse_bicgstab_conj_omega,
     mgpins.test_coarse_bicgstab_reaches_the_dense_solve),
]


@pytest.mark.parametrize("name,mod,attr,bad,pin", CASES, ids=[c[0] for c in CASES])
def test_pin_catches_planted_mistake(monkeypatch, name, mod, attr, bad, pin):
    monkeypatch.setattr(mod, attr, bad)
    with pytest.raises(AssertionError):
        pin()
