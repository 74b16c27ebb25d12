"""Oracle: the pieces of a two-level aggregation multigrid for D(m0), in FP64.

Test infrastructure only (see ``oracle/__init__.py``).

The paper's production solver is an adaptive geometric multigrid (Sec. "QUDA"
calls it the workhorse of the Dirac-matrix solves; Sec. "Performance Measurement
Method" names a mixed-precision multigrid solve as the kernel of the whole
computation) and, batched, motivates batching by the small parallelism of the
coarse grids (Sec. "Batched Linear Solves").  It does not spell the method out;
the reading used here is the standard aggregation form of that method:

* aggregates: blocks of b = (bx, by, bz, bt) fine sites; the coarse lattice has
  extents L_mu / b_mu and the aggregate of x is floor(x_mu / b_mu);
* near-null vectors v_1 .. v_nv (fine spinor fields) are split by chirality with
  P_+/- = (1 +/- gamma5)/2, gamma5 = diag(1, 1, -1, -1): spins 0, 1 and 2, 3;
* on every aggregate and chirality the nv restricted halves are made orthonormal
  by Gram-Schmidt in the order v_1, v_2, ... (each vector has the projections on
  the earlier, already normalised ones subtracted one after another, then is
  normalised); the results w_(a, chi, i) are the columns of the prolongator P;
* coarse vectors c[a][chi][i] (complex, chi = 0 for +, 1 for -):
  (P c)(x) = sum_(chi, i) c[a(x)][chi][i] w_(a(x), chi, i)(x), restriction R = P^dagger;
* coarse operator D_c = P^dagger D P (Galerkin).  D couples nearest neighbours, so
  D_c couples an aggregate with itself and its 8 neighbouring aggregates.

A solve preconditioned with these pieces still returns x = D^-1 b, so the GPU's
multigrid solutions are checked against the oracle's plain solvers; this module
gives the quantities with a definition of their own (basis, R, P, D_c) that the
GPU builds.

Coarse index order: c[..., tc, zc, yc, xc, chi, i]; a dense coarse matrix uses the
flat index ((((tc * Zc + zc) * Yc + yc) * Xc + xc) * 2 + chi) * nv + i.
"""
import numpy as np


def coarse_dims(dims, block):
    """(Xc, Yc, Zc, Tc) for fine dims (Lx, Ly, Lz, Lt) and aggregate extents."""
    for L, b in zip(dims, block):
        if b <= 0 or L % b:
            raise ValueError("aggregate extent %d does not divide %d" % (b, L))
    return tuple(L // b for L, b in zip(dims, block))


def _to_blocks(f, dims, block):
    """f[..., t, z, y, x, 4, 3] -> [..., Tc, Zc, Yc, Xc, 2 (chirality), (bt bz by bx 2 3)]."""
    lx, ly, lz, lt = dims
    bx, by, bz, bt = block
    xc, yc, zc, tc = coarse_dims(dims, block)
    lead = f.shape[:-6]
    g = f.reshape(lead + (tc, bt, zc, bz, yc, by, xc, bx, 2, 2, 3))
    k = len(lead)
    # move the coarse axes first, chirality next, the in-aggregate axes last
    order = list(range(k)) + [k + 0, k + 2, k + 4, k + 6, k + 8, k + 1, k + 3, k + 5, k + 7, k + 9, k + 10]
    g = np.transpose(g, order)
    return g.reshape(lead + (tc, zc, yc, xc, 2, bt * bz * by * bx * 6))


def _from_blocks(g, dims, block):
    """Inverse of _to_blocks."""
    lx, ly, lz, lt = dims
    bx, by, bz, bt = block
    xc, yc, zc, tc = coarse_dims(dims, block)
    lead = g.shape[:-6]
    k = len(lead)
    g = g.reshape(lead + (tc, zc, yc, xc, 2, bt, bz, by, bx, 2, 3))
    # axes now: tc zc yc xc chi bt bz by bx s a  ->  tc bt zc bz yc by xc bx chi s a
    order = list(range(k)) + [k + 0, k + 5, k + 1, k + 6, k + 2, k + 7, k + 3, k + 8, k + 4, k + 9, k + 10]
    f = np.transpose(g, order)
    return f.reshape(lead + (lt, lz, ly, lx, 4, 3))


def block_orthonormalize(vecs, dims, block):
    """Prolongator columns from near-null vectors vecs[nv][t][z][y][x][4][3].

    Returns w[nv][t][z][y][x][4][3]: on each aggregate, w[i] restricted to the
    spins of chirality chi is the i-th Gram-Schmidt vector of the chirality-chi
    halves of vecs[0..nv-1] there.  Raises if a half is (numerically) in the span
    of the earlier ones."""
    nv = vecs.shape[0]
    g = _to_blocks(np.asarray(vecs, dtype=np.complex128), dims, block)   # [nv][Tc..Xc][2][m]
    w = np.array(g)
    for i in range(nv):
        for j in range(i):
            d = np.sum(np.conj(w[j]) * w[i], axis=-1, keepdims=True)
            w[i] = w[i] - d * w[j]
        n = np.sqrt(np.sum(np.abs(w[i]) ** 2, axis=-1, keepdims=True))
        if np.any(n <= 1e-12 * np.sqrt(np.sum(np.abs(g[i]) ** 2, axis=-1, keepdims=True))):
            raise ValueError("near-null vector %d is linearly dependent on an aggregate" % i)
        w[i] = w[i] / n
    return _from_blocks(w, dims, block)


def restrict(basis, f, dims, block):
    """(R f)[n][tc][zc][yc][xc][chi][i] = sum over the aggregate of <w_(a, chi, i), f>."""
    wb = _to_blocks(basis, dims, block)            # [nv][Tc][Zc][Yc][Xc][2][m]
    fb = _to_blocks(f, dims, block)                # [n][Tc][Zc][Yc][Xc][2][m]
    return np.einsum("itzyxcm,ntzyxcm->ntzyxci", np.conj(wb), fb)


def prolong(basis, c, dims, block):
    """(P c)(x) = sum_(chi, i) c[a(x)][chi][i] w_(a(x), chi, i)(x); c[n][tc][zc][yc][xc][2][nv]."""
    wb = _to_blocks(basis, dims, block)
    fb = np.einsum("itzyxcm,ntzyxci->ntzyxcm", wb, c)
    return _from_blocks(fb, dims, block)


def coarse_dense(D, basis, block):
    """The Galerkin coarse matrix P^dagger D P as a dense matrix, column by column:
    column q is R D P e_q for the coarse unit vector e_q."""
    dims = D.dims
    nv = basis.shape[0]
    xc, yc, zc, tc = coarse_dims(dims, block)
    nq = tc * zc * yc * xc * 2 * nv
    out = np.zeros((nq, nq), dtype=np.complex128)
    chunk = 64
    for q0 in range(0, nq, chunk):
        q1 = min(nq, q0 + chunk)
        e = np.zeros((q1 - q0, nq), dtype=np.complex128)
        e[np.arange(q1 - q0), np.arange(q0, q1)] = 1.0
        c = e.reshape((q1 - q0, tc, zc, yc, xc, 2, nv))
        col = restrict(basis, D.apply(prolong(basis, c, dims, block)), dims, block)
        out[:, q0:q1] = col.reshape(q1 - q0, nq).T
    return out


def coarse_gamma5(dims, block, nv):
    """The coarse chirality sign (+1 for chi = 0, -1 for chi = 1) per coarse index."""
    xc, yc, zc, tc = coarse_dims(dims, block)
    s = np.ones((tc, zc, yc, xc, 2, nv))
    s[..., 1, :] = -1.0
    return s.ravel()


def coarse_neighbour(dims, block, a, mu, k):
    """Coarse site index of the aggregate next to a in direction k * mu (periodic)."""
    xc, yc, zc, tc = coarse_dims(dims, block)
    ext = (xc, yc, zc, tc)
    co = [a % xc, (a // xc) % yc, (a // (xc * yc)) % zc, a // (xc * yc * zc)]
    co[mu] = (co[mu] + k) % ext[mu]
    return ((co[3] * zc + co[2]) * yc + co[1]) * xc + co[0]


# ---------------------------------------------------------------------------
# the cycle (the reading of the method's steps used by the library)
# ---------------------------------------------------------------------------
# The multigrid-preconditioned solve returns D^-1 b whatever the cycle does, and is
# checked against the plain solvers.  The cycle itself is this project's reading of
# the method (the paper names the solver class only); its pieces are pinned below by
# identities of their own (tests/test_oracle_mg.py), not by values the paper gives.

def _dot(a, b):
    return np.sum(np.conj(a) * b)


def smoother(D, r, iters):
    """Approximate D^-1 r through the even-odd Schur system: b^ = A_ee^-1 (r_e + 1/2
    H_eo A_oo^-1 r_o); `iters` minimal-residual steps on M^ e_e = b^ from e_e = 0
    (rho <- b^ - M^ e_e, alpha = <M^ rho, rho> / |M^ rho|^2); e_o = A_oo^-1 (r_o +
    1/2 H_oe e_e).  Returns (e, rho): the full-lattice e and the last MR residual."""
    from .dirac import EvenOdd
    eo = EvenOdd(D)
    rho = eo.prepare(r)
    e_e = np.zeros_like(r)
    for _ in range(iters):
        t = eo.M_hat(rho)
        tt = _dot(t, t).real
        a = _dot(t, rho) / tt if tt > 0 else 0.0
        e_e = e_e + a * rho
        rho = rho - a * t
    return eo.reconstruct(r, e_e), rho


def coarse_bicgstab(Dc, b, iters, tol):
    """BiCGStab on the dense coarse matrix from x = 0, r^ = r = b, for at most `iters`
    iterations, stopping once |r| <= tol |b| (checked after each iteration)."""
    x = np.zeros_like(b)
    r = b.copy()
    rh = b.copy()
    p = np.zeros_like(b)
    v = np.zeros_like(b)
    rho = alpha = omega = 1.0
    b2 = _dot(b, b).real
    if not b2 > 0:
        return x
    for _ in range(iters):
        rn = _dot(rh, r)
        if rn == 0:
            break
        beta = (rn / rho) * (alpha / omega)
        rho = rn
        p = r + beta * (p - omega * v)
        v = Dc @ p
        sg = _dot(rh, v)
        if sg == 0:
            break
        alpha = rho / sg
        s = r - alpha * v
        t = Dc @ s
        tt = _dot(t, t).real
        omega = _dot(t, s) / tt if tt > 0 else 0.0
        x = x + alpha * p + omega * s
        r = s - omega * t
        if _dot(r, r).real <= tol * tol * b2:
            break
    return x


def cycle(D, basis, block, Dc, r, smooth_iters, coarse_iters, coarse_tol):
    """One two-level cycle for D e = r: pre-smoother, coarse correction of its
    residual (restrict, coarse BiCGStab, prolong), post-smoother on what remains."""
    from .dirac import apply_site_matrix
    dims = D.dims
    e1, rho = smoother(D, r, smooth_iters)
    res = apply_site_matrix(D.A, rho)          # r - D e1: A_ee times the MR residual (odd part 0)
    rc = restrict(basis, res[None], dims, block)[0]
    ec = coarse_bicgstab(Dc, rc.ravel(), coarse_iters, coarse_tol).reshape(rc.shape)
    q = prolong(basis, ec[None], dims, block)[0]
    res2 = res - D.apply(q)
    e3, _ = smoother(D, res2, smooth_iters)
    return e1 + q + e3


def gcr(D, basis, block, Dc, b, tol, smooth_iters, coarse_iters, coarse_tol, restart, maxiter, directions=False):
    """Flexible GCR(restart) for D x = b preconditioned by one cycle per iteration,
    from x = 0: z_k = cycle(r), w_k = D z_k, w_k and z_k made orthogonal to the
    earlier w_j of the cycle (coefficients <w_j, w_k> of the normalised w_j, all from
    the unmodified w_k), then x += g z_k, r -= g w_k with g = <w_k, r> / |w_k|^2 and
    w_k, z_k normalised by |w_k|.  Every `restart` iterations, or once |r| <= tol |b| / 2,
    the residual is recomputed as b - D x; the solve stops when that is <= tol |b| or
    after maxiter iterations.  Returns (x, iterations), and with directions=True also
    the normalised z and w of the last restart cycle."""
    x = np.zeros_like(b)
    r = b.copy()
    b2 = _dot(b, b).real
    it = 0
    while it < maxiter and _dot(r, r).real > tol * tol * b2:
        Z, W = [], []
        for _ in range(restart):
            if it >= maxiter:
                break
            z = cycle(D, basis, block, Dc, r, smooth_iters, coarse_iters, coarse_tol)
            w = D.apply(z)
            betas = [_dot(wj, w) for wj in W]
            for bj, zj, wj in zip(betas, Z, W):
                w = w - bj * wj
                z = z - bj * zj
            n2 = _dot(w, w).real
            g = _dot(w, r) / n2
            x = x + g * z
            r = r - g * w
            W.append(w / np.sqrt(n2))
            Z.append(z / np.sqrt(n2))
            it += 1
            if _dot(r, r).real <= 0.25 * tol * tol * b2:
                break
        r = b - D.apply(x)
    if directions:
        return x, it, Z, W
    return x, it
