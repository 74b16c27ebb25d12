"""Pins of the oracle's multigrid pieces (``oracle/multigrid.py``) against facts
fixed by their definitions and by the free field, not by the oracle itself.

* the prolongator columns are orthonormal per aggregate and chirality and span the
  chiral halves of the near-null vectors there (a skipped projection, a lost
  normalisation or a chirality mix-up fails);
* restriction is the adjoint of prolongation (a missing conjugate fails);
* after an exact coarse correction the restricted residual vanishes (Galerkin
  orthogonality: D_c = P^dagger D P holds, whatever the routes of R, P and D);
* gamma5-hermiticity carries over to the coarse matrix with the chirality signs;
* the coarse matrix couples an aggregate only to itself and its 8 neighbours;
* on the free field with constant near-null vectors the coarse matrix is a Wilson
  matrix on the coarse lattice in closed form: self block (4 + m0) - sum_mu
  (b_mu - 1)/b_mu, hop to a + mu -1/2 eta (1 - gamma_mu)/b_mu, to a - mu
  -1/2 eta (1 + gamma_mu)/b_mu, eta = -1 across the antiperiodic time boundary.
"""
import numpy as np

import laph_synth as ls
from oracle import dirac
from oracle import multigrid as mg

DIMS = (6, 4, 4, 6)
BLOCK = (2, 2, 2, 3)
NV = 3


def _vecs(dims, nv, seed):
    return ls.random_spinor((nv,) + ls.spinor_shape(dims), seed)


def _chiral(f, chi):
    out = np.zeros_like(f)
    out[..., 2 * chi:2 * chi + 2, :] = f[..., 2 * chi:2 * chi + 2, :]
    return out


def test_basis_orthonormal_and_spanning():
    v = _vecs(DIMS, NV, 801)
    w = mg.block_orthonormalize(v, DIMS, BLOCK)
    xc, yc, zc, tc = mg.coarse_dims(DIMS, BLOCK)
    nc = xc * yc * zc * tc
    # coefficients of the columns against themselves: R applied to the columns
    for i in range(NV):
        c = mg.restrict(w, w[i:i + 1], DIMS, BLOCK)[0].reshape(nc, 2, NV)
        expect = np.zeros((nc, 2, NV), dtype=np.complex128)
        expect[:, :, i] = 1.0
        assert np.abs(c - expect).max() < 1e-13
    # each chiral half of each near-null vector lies in the span: v = P R v
    pv = mg.prolong(w, mg.restrict(w, v, DIMS, BLOCK), DIMS, BLOCK)
    assert np.abs(pv - v).max() < 1e-12 * np.abs(v).max()
    # a column is supported on one chirality: w = P_+ w + P_- w with each part from its own Gram-Schmidt
    for i in range(NV):
        for chi in range(2):
            part = _chiral(w[i], chi)
            n2 = mg.restrict(w, part[None], DIMS, BLOCK)[0].reshape(nc, 2, NV)
            assert np.abs(n2[:, 1 - chi, :]).max() < 1e-13


def test_restrict_is_adjoint_of_prolong():
    v = _vecs(DIMS, NV, 802)
    w = mg.block_orthonormalize(v, DIMS, BLOCK)
    xc, yc, zc, tc = mg.coarse_dims(DIMS, BLOCK)
    f = ls.random_spinor(ls.spinor_shape(DIMS, 2), 803)
    c = ls.random_spinor((2, tc, zc, yc, xc, 2, NV), 804)
    lhs = np.sum(np.conj(mg.prolong(w, c, DIMS, BLOCK)) * f)
    rhs = np.sum(np.conj(c) * mg.restrict(w, f, DIMS, BLOCK))
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_galerkin_orthogonality_and_gamma5():
    U = ls.gauge_field(DIMS, 805)
    D = dirac.WilsonClover(U, 0.1, 1.0)
    w = mg.block_orthonormalize(_vecs(DIMS, NV, 806), DIMS, BLOCK)
    Dc = mg.coarse_dense(D, w, BLOCK)
    r = ls.random_spinor(ls.spinor_shape(DIMS, 1), 807)
    rc = mg.restrict(w, r, DIMS, BLOCK)
    ec = np.linalg.solve(Dc, rc.reshape(-1)).reshape(rc.shape)
    r2 = r - D.apply(mg.prolong(w, ec, DIMS, BLOCK))
    assert np.abs(mg.restrict(w, r2, DIMS, BLOCK)).max() < 1e-12 * np.abs(rc).max()
    g5 = mg.coarse_gamma5(DIMS, BLOCK, NV)
    H = g5[:, None] * Dc
    assert np.abs(H - H.conj().T).max() < 1e-13 * np.abs(Dc).max()


def test_coarse_stencil_is_nearest_neighbour():
    dims, block = (6, 6, 6, 6), (2, 2, 2, 2)
    U = ls.gauge_field(dims, 808)
    D = dirac.WilsonClover(U, 0.1, 1.0)
    nv = 2
    w = mg.block_orthonormalize(_vecs(dims, nv, 809), dims, block)
    Dc = mg.coarse_dense(D, w, block)
    m = 2 * nv
    nc = Dc.shape[0] // m
    blocks = Dc.reshape(nc, m, nc, m)
    for a in range(nc):
        nb = {a} | {mg.coarse_neighbour(dims, block, a, mu, k) for mu in range(4) for k in (1, -1)}
        for b in range(nc):
            n = np.abs(blocks[a, :, b, :]).max()
            if b in nb:
                assert n > 1e-3
            else:
                assert n == 0.0


def test_free_field_closed_form():
    dims, block = (6, 6, 6, 6), (2, 2, 2, 2)
    m0 = 0.07
    U = ls.unit_gauge(dims)
    D = dirac.WilsonClover(U, m0, 1.0)
    # v_i = e_(s, a) + e_(s + 2, a), s = i // 3, a = i % 3: chirality halves e_(s, a) and e_(s + 2, a)
    v = np.zeros((6,) + ls.spinor_shape(dims), dtype=np.complex128)
    for i in range(6):
        v[i, ..., i // 3, i % 3] = 1.0
        v[i, ..., 2 + i // 3, i % 3] = 1.0
    w = mg.block_orthonormalize(v, dims, block)
    Dc = mg.coarse_dense(D, w, block)
    xc, yc, zc, tc = mg.coarse_dims(dims, block)
    nc = xc * yc * zc * tc
    # coarse index (chi, i) is fine spin-colour index 6 chi + i
    G = [np.kron(dirac.GAMMA[mu], np.eye(3)) for mu in range(4)]
    one = np.eye(12)
    expect = np.zeros((nc, 12, nc, 12), dtype=np.complex128)
    ext = (xc, yc, zc, tc)
    for a in range(nc):
        expect[a, :, a, :] += (4 + m0 - sum((b - 1) / b for b in block)) * one
        co = [a % xc, (a // xc) % yc, (a // (xc * yc)) % zc, a // (xc * yc * zc)]
        for mu in range(4):
            for k, sgn in ((1, -1.0), (-1, 1.0)):
                eta = 1.0
                if mu == 3 and (co[3] + k) % ext[3] != co[3] + k:
                    eta = -1.0
                b = mg.coarse_neighbour(dims, block, a, mu, k)
                expect[a, :, b, :] += -0.5 * eta * (one + sgn * G[mu]) / block[mu]
    assert np.abs(Dc - expect.reshape(Dc.shape)).max() < 1e-13


def _relaxed_setup(dims, block, m0, nv, seed):
    U = ls.gauge_field(dims, seed)
    D = dirac.WilsonClover(U, m0, 1.0)
    V = _vecs(dims, nv, seed + 1)
    from oracle import solvers
    for _ in range(2):
        V, _ = solvers.bicgstab(D.apply, V, tol=1e-2)
    w = mg.block_orthonormalize(V, dims, block)
    return D, w, mg.coarse_dense(D, w, block)


def test_smoother_residual_identity_and_monotone_mr():
    """After the smoother the odd residual vanishes and the even one is A_ee times the
    last MR residual; each MR step cannot increase that residual."""
    U = ls.gauge_field(DIMS, 810)
    D = dirac.WilsonClover(U, 0.1, 1.0)
    r = ls.random_spinor(ls.spinor_shape(DIMS), 811)
    last = np.inf
    for it in range(1, 5):
        e, rho = mg.smoother(D, r, it)
        res = r - D.apply(e)
        expect = dirac.apply_site_matrix(D.A, rho)
        assert np.linalg.norm(res - expect) < 1e-12 * np.linalg.norm(r)
        odd = 1.0 - dirac.parity_mask(DIMS)
        assert np.linalg.norm(odd * res) < 1e-12 * np.linalg.norm(r)
        n = np.linalg.norm(rho)
        assert n <= last * (1 + 1e-12)
        last = n


def test_coarse_bicgstab_reaches_the_dense_solve():
    D, w, Dc = _relaxed_setup(DIMS, BLOCK, 0.1, NV, 812)
    b = ls.random_spinor((Dc.shape[0],), 813)
    x = mg.coarse_bicgstab(Dc, b, 500, 1e-14)
    ref = np.linalg.solve(Dc, b)
    assert np.linalg.norm(x - ref) < 1e-10 * np.linalg.norm(ref)


def test_cycle_contracts_the_residual():
    """With near-null vectors from two inverse-iteration passes the cycle is a good
    approximate inverse: |r - D K r| well below |r| (a two-grid property)."""
    D, w, Dc = _relaxed_setup(DIMS, BLOCK, 0.1, NV, 814)
    r = ls.random_spinor(ls.spinor_shape(DIMS), 815)
    e = mg.cycle(D, w, BLOCK, Dc, r, 4, 16, 0.1)
    assert np.linalg.norm(r - D.apply(e)) < 0.2 * np.linalg.norm(r)
