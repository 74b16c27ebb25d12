"""Oracle: LapH vectors, sources, perambulators and their gradients, in FP64.

Test infrastructure only (see ``oracle/__init__.py``).

* LapH smearing projects quark fields onto the lowest eigenvectors of the
  gauge-covariant 3-D Laplacian on each timeslice (Sec. "Current
  state-of-the-art", Sec. "LapH").  ``laplacian_eigvecs`` computes them densely.
* Sources are the LapH vectors of the source timeslice, diluted in spin; the
  propagators are the Dirac solves from those sources, and the perambulator is
  their projection onto the LapH vectors of every sink timeslice (Sec.
  "QUDA", Sec. "Eigenvector Projection"):

      tau[t][l][k][beta][alpha] = sum_{x, a} conj(V_l(x, t)_a) X^(4k+alpha)(x, t)_(beta, a)
      X^(r) = D^-1 b^(r),   b^(4k+alpha)(x, t)_(s, a) = delta_{t,t0} delta_{s,alpha} V_k(x, t0)_a

* Gradients of L = sum |tau[t_s]|^2 with respect to the sources and to m0 use
  D^dagger = gamma5 D gamma5 and dD/dm0 = 1 (the mass enters A only):
      Z^(r) = gamma5 D^-1 (gamma5 G_X^(r)),   grad_b = Z,   grad_m0 = -sum_r Re<Z^(r), X^(r)>
  with PyTorch's convention grad_z = dL/dRe z + i dL/dIm z.
"""
import numpy as np

from .dirac import GAMMA5, WilsonClover, dag
from .solvers import bicgstab, dense_solve


# --- the 3-D gauge-covariant Laplacian ------------------------------------------

def neg_laplacian_apply(U3, f):
    """(-Delta f)(x) = sum_k [2 f(x) - U_k(x) f(x+k) - U_k(x-k)^dagger f(x-k)].

    U3: links of one timeslice, shape (z, y, x, 4, 3, 3) (only k = 0, 1, 2 used);
    f: colour field (..., z, y, x, 3).  Periodic, no boundary phase."""
    out = 6.0 * f
    for k in range(3):
        ax = -2 - k                      # x: -2, y: -3, z: -4 for f[..., z, y, x, a]
        uk = U3[..., k, :, :]
        fwd = np.roll(f, -1, axis=ax)
        bwd = np.roll(f, +1, axis=ax)
        ub = np.roll(uk, +1, axis=-3 - k)  # U_k(x - k), link field axes (z, y, x, a, b)
        out = out - np.matmul(uk, fwd[..., None])[..., 0]
        out = out - np.matmul(dag(ub), bwd[..., None])[..., 0]
    return out


def neg_laplacian_dense(U3):
    """Dense (3 L^3) x (3 L^3) matrix of -Delta on one timeslice."""
    lz, ly, lx = U3.shape[:3]
    n = 3 * lx * ly * lz
    eye = np.eye(n, dtype=np.complex128).reshape(n, lz, ly, lx, 3)
    return neg_laplacian_apply(U3, eye).reshape(n, n).T.copy()


def fix_phase(v, tol=1e-12):
    """Make the largest-modulus component real positive (lowest index on ties)."""
    mags = np.abs(v)
    big = mags.max()
    idx = int(np.nonzero(mags >= big - tol)[0][0])
    return v * (np.conj(v[idx]) / np.abs(v[idx]))


def laplacian_eigvecs(U, nev):
    """Lowest ``nev`` eigenvectors of -Delta on every timeslice.

    Returns (V[t][l][z][y][x][a], eigenvalues[t][nev], gap[t] = lambda_{nev} - lambda_{nev-1})."""
    lt, lz, ly, lx = U.shape[:4]
    V = np.empty((lt, nev, lz, ly, lx, 3), dtype=np.complex128)
    lam = np.empty((lt, nev))
    gap = np.empty(lt)
    for t in range(lt):
        w, q = np.linalg.eigh(neg_laplacian_dense(U[t]))
        lam[t] = w[:nev]
        gap[t] = w[nev] - w[nev - 1] if nev < len(w) else np.inf
        for l in range(nev):
            V[t, l] = fix_phase(q[:, l]).reshape(lz, ly, lx, 3)
    return V, lam, gap


# --- sources and projection -------------------------------------------------------

def laph_sources(V, t0, nev=None):
    """Spin-diluted LapH sources b[r][t][z][y][x][s][a] with r = 4k + alpha."""
    lt, nv, lz, ly, lx, _ = V.shape
    nev = nv if nev is None else nev
    b = np.zeros((4 * nev, lt, lz, ly, lx, 4, 3), dtype=np.complex128)
    for k in range(nev):
        for alpha in range(4):
            b[4 * k + alpha, t0, :, :, :, alpha, :] = V[t0, k]
    return b


def project(V, X, nev_src):
    """tau[t][l][k][beta][alpha] = sum_{x,a} conj(V_l(x,t)_a) X^(4k+alpha)(x,t)_(beta,a)."""
    lt, nev, lz, ly, lx, _ = V.shape
    Xr = X.reshape(nev_src, 4, lt, lz, ly, lx, 4, 3)     # [k][alpha][t][z][y][x][beta][a]
    return np.einsum("tlzyxa,kctzyxba->tlkbc", np.conj(V), Xr)


def perambulator(U, V, t0, m0, csw=1.0, tol=1e-13, method="bicgstab", antiperiodic_t=True):
    """tau = V^dagger D(m0)^-1 V for all sink timeslices; returns (tau, X)."""
    D = WilsonClover(U, m0, csw, antiperiodic_t)
    b = laph_sources(V, t0)
    if method == "dense":
        X = dense_solve(D, b)
    else:
        X, _ = bicgstab(D.apply, b, tol=tol)
    return project(V, X, V.shape[1]), X


# --- stochastic LapH: noise-diluted sources ---------------------------------------
#
# The stochastic variant of LapH (Sec. "Current state-of-the-art": the earlier CPU
# NN work used it) replaces the full set of 4 nev sources per source time by noise in the
# LapH x spin space, diluted: the noise rho[alpha][k] of the source time is split
# by spin (full spin dilution) and by LapH index into n_dil interlaced groups
# {k : k mod n_dil = j}.  Source j, alpha carries the noise of its group and spin:
#
#     b^(4j+alpha)(x, t)_(beta, a) = delta_{t,t0} delta_{beta,alpha} sum_{k = j mod n_dil} rho[alpha][k] V_k(x, t0)_a
#
# and its solution is projected onto the LapH vectors of every sink time exactly
# like the perambulator (phi[t][l][j][beta][alpha]).  With n_dil = nev and
# rho = 1 the sources are the perambulator's.

def noise_sources(V, t0, rho, n_dil):
    """Diluted noise sources b[r][t][z][y][x][s][a], r = 4 j + alpha, j < n_dil."""
    lt, nev, lz, ly, lx, _ = V.shape
    b = np.zeros((4 * n_dil, lt, lz, ly, lx, 4, 3), dtype=np.complex128)
    for j in range(n_dil):
        for alpha in range(4):
            for k in range(j, nev, n_dil):
                b[4 * j + alpha, t0, :, :, :, alpha, :] += rho[alpha, k] * V[t0, k]
    return b


def stochastic_perambulator(U, V, t0, m0, rho, n_dil, csw=1.0, tol=1e-13, method="bicgstab", antiperiodic_t=True):
    """phi[t][l][j][beta][alpha] = sum_{x,a} conj(V_l(x,t)_a) (D^-1 b^(4j+alpha))(x,t)_(beta,a); returns (phi, X)."""
    D = WilsonClover(U, m0, csw, antiperiodic_t)
    b = noise_sources(V, t0, rho, n_dil)
    if method == "dense":
        X = dense_solve(D, b)
    else:
        X, _ = bicgstab(D.apply, b, tol=tol)
    return project(V, X, n_dil), X


# --- spin basis of the perambulator ---------------------------------------------------
#
# The driver side of the paper's workflow introduces a further Dirac spin basis
# (Sec. "Quda_laph"), without saying which.  A change of basis psi' = S psi (S unitary)
# turns the propagator's spin matrix M into S M S^dagger, so for the perambulator
#     tau'[t][l][k][beta'][alpha'] = sum_{beta, alpha} S[beta'][beta] tau[t][l][k][beta][alpha] conj(S[alpha'][alpha])

def spin_rotate(tau, S):
    """tau' = S tau S^dagger on the last two (sink spin, source spin) indices."""
    return np.einsum("ab,...bc,dc->...ad", S, tau, np.conj(S))


# --- loss and gradients -------------------------------------------------------------

def loss_from_tau(tau, t_sink, nblk=None):
    """L = sum_{l, k < nblk; beta, alpha} |tau[t_sink][l][k][beta][alpha]|^2."""
    blk = tau[t_sink] if nblk is None else tau[t_sink, :nblk, :nblk]
    return float(np.sum(np.abs(blk) ** 2))


def loss_of_sources(D, V, b, t_sink, tol=1e-13):
    """L(b, m0) = sum |tau[t_sink]|^2 with X = D^-1 b (b has the 4*nev RHS)."""
    X, _ = bicgstab(D.apply, b, tol=tol)
    tau = project(V, X, b.shape[0] // 4)
    return loss_from_tau(tau, t_sink), X, tau


def tau_cotangent_to_X(V, g_tau_t, t_sink, shape):
    """G_X^(4k+alpha)(x, t_sink)_(beta, a) = sum_l V_l(x, t_sink)_a G_tau[l][k][beta][alpha]."""
    lt, nev, lz, ly, lx, _ = V.shape
    nk = g_tau_t.shape[1]
    gx = np.zeros(shape, dtype=np.complex128).reshape(nk, 4, lt, lz, ly, lx, 4, 3)
    gx[:, :, t_sink] = np.einsum("lzyxa,lkbc->kczyxba", V[t_sink], g_tau_t)
    return gx.reshape(shape)


def adjoint_gradients(D, V, b, t_sink, tol=1e-13):
    """(L, grad_b, grad_m0) by the adjoint formula with D^dagger = gamma5 D gamma5."""
    L, X, tau = loss_of_sources(D, V, b, t_sink, tol)
    g_tau = 2.0 * tau[t_sink]
    gx = tau_cotangent_to_X(V, g_tau, t_sink, X.shape)
    g5 = np.diag(GAMMA5).real.reshape(4, 1)
    Zg, _ = bicgstab(D.apply, g5 * gx, tol=tol)
    Z = g5 * Zg
    grad_m0 = -float(np.sum(np.real(np.conj(Z) * X)))
    return L, Z, grad_m0, X


def fd_mass(U, V, b, m0, csw, t_sink, h=1e-4, tol=1e-13, antiperiodic_t=True):
    """Central difference (L(m0+h) - L(m0-h)) / 2h."""
    lp = loss_of_sources(WilsonClover(U, m0 + h, csw, antiperiodic_t), V, b, t_sink, tol)[0]
    lm = loss_of_sources(WilsonClover(U, m0 - h, csw, antiperiodic_t), V, b, t_sink, tol)[0]
    return (lp - lm) / (2 * h)


def fd_source(D, V, b, d, t_sink, h=1e-4, tol=1e-13):
    """Central difference (L(b + h d) - L(b - h d)) / 2h  (~ Re<grad_b, d>)."""
    lp = loss_of_sources(D, V, b + h * d, t_sink, tol)[0]
    lm = loss_of_sources(D, V, b - h * d, t_sink, tol)[0]
    return (lp - lm) / (2 * h)


# --- meson doublets and baryon triplets of the LapH vectors ----------------------
#
# The LapH vectors also build the quark-antiquark doublets and three-quark triplets
# that enter the Wick contractions of meson and baryon correlators (Sec. "QUDA").
# The paper names them only; the definitions below are the standard momentum-
# projected, undisplaced forms, with p = 2 pi (nx / Lx, ny / Ly, nz / Lz):
#
#     Phi_p[t][l][m]     = sum_x exp(-i p.x) sum_a conj(V_l(x, t)_a) V_m(x, t)_a
#     B_p[t][l][m][n]    = sum_x exp(-i p.x) sum_{a,b,c} eps_abc V_l(x, t)_a V_m(x, t)_b V_n(x, t)_c

def levi_civita():
    """eps_abc of three colours: +1 on even permutations of (0, 1, 2), -1 on odd ones."""
    eps = np.zeros((3, 3, 3))
    for a, b, c in ((0, 1, 2), (1, 2, 0), (2, 0, 1)):
        eps[a, b, c] = 1.0
        eps[a, c, b] = -1.0
    return eps


def momentum_phases(dims3, moms):
    """exp(-i p.x) on one timeslice, [n_mom][z][y][x], for integer momenta (nx, ny, nz)."""
    lx, ly, lz = dims3
    z, y, x = np.meshgrid(np.arange(lz), np.arange(ly), np.arange(lx), indexing="ij")
    return np.array([np.exp(-2j * np.pi * (nx * x / lx + ny * y / ly + nz * z / lz)) for nx, ny, nz in moms])


def meson_doublets(V, moms):
    """Phi[p][t][l][m] = sum_x exp(-i p.x) sum_a conj(V_l(x, t)_a) V_m(x, t)_a."""
    lt, nev, lz, ly, lx, _ = V.shape
    ph = momentum_phases((lx, ly, lz), moms)
    return np.einsum("pzyx,tlzyxa,tmzyxa->ptlm", ph, np.conj(V), V, optimize=True)


def baryon_triplets(V, moms):
    """B[p][t][l][m][n] = sum_x exp(-i p.x) eps_abc V_l(x, t)_a V_m(x, t)_b V_n(x, t)_c."""
    lt, nev, lz, ly, lx, _ = V.shape
    ph = momentum_phases((lx, ly, lz), moms)
    return np.einsum("pzyx,abc,tlzyxa,tmzyxb,tnzyxc->ptlmn", ph, levi_civita(), V, V, V, optimize=True)
