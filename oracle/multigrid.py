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
