"""Oracle: the Wilson-clover Dirac matrix D(m0), written out in FP64.

Test infrastructure only (see ``oracle/__init__.py``).

The paper's quark propagators are the inverse of the lattice Dirac matrix
applied to LapH sources (Sec. "Current state-of-the-art"; Sec. "QUDA": the
Dirac-matrix linear solver is the workhorse).  The paper does not write the
matrix down; this module implements the reading used throughout the project:

    (D psi)(x) = A(x) psi(x) - 1/2 (H psi)(x)
    (H psi)(x) = sum_mu [ eta+ (1 - gamma_mu) U_mu(x) psi(x+mu)
                         + eta- (1 + gamma_mu) U_mu(x-mu)^dagger psi(x-mu) ]
    A(x)       = (4 + m0) 1 + c_sw (i/2) sum_{mu<nu} sigma_munu (x) F_munu(x)
    sigma_munu = (i/2) [gamma_mu, gamma_nu]
    F_munu     = (Q_munu - Q_munu^dagger)/8 with its trace removed,
                 Q_munu = sum of the four oriented plaquettes at x in the mu-nu plane

DeGrand-Rossi chiral gamma basis, periodic links, fermion hops across the time
boundary carry -1 when the time direction is antiperiodic.

Field layouts: ``psi[..., t, z, y, x, s, a]`` and ``U[t, z, y, x, mu, a, b]``.
"""
import numpy as np

from ._cref import hop_c

# DeGrand-Rossi chiral basis (rows); gamma5 = gx gy gz gt = diag(1, 1, -1, -1).
GAMMA = np.array([
    [[0, 0, 0, 1j], [0, 0, 1j, 0], [0, -1j, 0, 0], [-1j, 0, 0, 0]],
    [[0, 0, 0, -1], [0, 0, 1, 0], [0, 1, 0, 0], [-1, 0, 0, 0]],
    [[0, 0, 1j, 0], [0, 0, 0, -1j], [-1j, 0, 0, 0], [0, 1j, 0, 0]],
    [[0, 0, 1, 0], [0, 0, 0, 1], [1, 0, 0, 0], [0, 1, 0, 0]],
], dtype=np.complex128)
GAMMA5 = GAMMA[0] @ GAMMA[1] @ GAMMA[2] @ GAMMA[3]
PLANES = [(mu, nu) for mu in range(4) for nu in range(mu + 1, 4)]


def sigma(mu, nu):
    """sigma_munu = (i/2) [gamma_mu, gamma_nu] (Hermitian)."""
    return 0.5j * (GAMMA[mu] @ GAMMA[nu] - GAMMA[nu] @ GAMMA[mu])


def dag(m):
    return np.conj(np.swapaxes(m, -1, -2))


def dims_of(U):
    lt, lz, ly, lx = U.shape[:4]
    return (lx, ly, lz, lt)


# --- shifts -----------------------------------------------------------------
# A field with two trailing non-site axes (spinor (4,3) or link (3,3)) has its
# x, y, z, t axes at -3, -4, -5, -6.

def site_shift(f, mu, k):
    """f(x + k*mu_hat) with periodic wrap (no boundary phase)."""
    return np.roll(f, -k, axis=-3 - mu)


def fermion_shift(psi, mu, k, antiperiodic_t=True):
    """psi(x + k*mu_hat), k = +1 or -1, with the antiperiodic time phase."""
    out = site_shift(psi, mu, k)
    if mu == 3 and antiperiodic_t:
        idx = [slice(None)] * out.ndim
        idx[out.ndim - 6] = -1 if k > 0 else 0
        out[tuple(idx)] *= -1.0
    return out


def colour_mul(m, psi):
    """Apply per-site 3x3 colour matrices m[t,z,y,x,a,b] to psi[..., s, b]."""
    return np.matmul(m[..., None, :, :], psi[..., None])[..., 0]


def spin_mul(g, psi):
    """Apply a 4x4 spin matrix to psi[..., s, a]."""
    return np.matmul(g, psi)


# --- hopping term -------------------------------------------------------------

def hop_numpy(U, psi, antiperiodic_t=True, dagger=False):
    """H psi written with whole-field numpy operations (slow, for cross-checks)."""
    out = np.zeros_like(psi)
    sg = -1.0 if dagger else 1.0
    for mu in range(4):
        umu = U[..., mu, :, :]
        fwd = colour_mul(umu, fermion_shift(psi, mu, +1, antiperiodic_t))
        bwd = colour_mul(dag(site_shift(umu, mu, -1)), fermion_shift(psi, mu, -1, antiperiodic_t))
        out += fwd - sg * spin_mul(GAMMA[mu], fwd)
        out += bwd + sg * spin_mul(GAMMA[mu], bwd)
    return out


def hop(U, psi, antiperiodic_t=True, dagger=False):
    """H psi (dagger=True: gamma5 H gamma5) via the plain-C site loop."""
    return hop_c(U, psi, GAMMA, antiperiodic_t, dagger)


# --- clover -------------------------------------------------------------------

def plaquette_sum(U, mu, nu):
    """Q_munu(x): the four plaquettes at x in the mu-nu plane, same orientation."""
    um, un = U[..., mu, :, :], U[..., nu, :, :]
    s = site_shift
    um_m = s(um, mu, -1)             # U_mu(x - mu)
    un_n = s(un, nu, -1)             # U_nu(x - nu)
    leaf1 = um @ s(un, mu, +1) @ dag(s(um, nu, +1)) @ dag(un)
    leaf2 = un @ dag(s(um_m, nu, +1)) @ dag(s(un, mu, -1)) @ um_m
    leaf3 = dag(um_m) @ dag(s(un_n, mu, -1)) @ s(um_m, nu, -1) @ un_n
    leaf4 = dag(un_n) @ s(um, nu, -1) @ s(un_n, mu, +1) @ dag(um)
    return leaf1 + leaf2 + leaf3 + leaf4


def field_strength(U, mu, nu):
    """F_munu = (Q - Q^dagger)/8, trace removed (anti-Hermitian, traceless)."""
    q = plaquette_sum(U, mu, nu)
    f = (q - dag(q)) / 8.0
    tr = np.trace(f, axis1=-2, axis2=-1)
    return f - (tr / 3.0)[..., None, None] * np.eye(3)


def clover_term(U, csw):
    """c_sw (i/2) sum_{mu<nu} sigma_munu (x) F_munu as per-site 12x12 matrices.

    Spin-colour index is 3*s + a.  Returns shape (t, z, y, x, 12, 12)."""
    lt, lz, ly, lx = U.shape[:4]
    c = np.zeros((lt, lz, ly, lx, 4, 3, 4, 3), dtype=np.complex128)
    for mu, nu in PLANES:
        f = field_strength(U, mu, nu)
        c += np.einsum("st,...ab->...satb", sigma(mu, nu), f)
    return (0.5j * csw) * c.reshape(lt, lz, ly, lx, 12, 12)


def clover_matrix(U, m0, csw):
    """A(x) = (4 + m0) 1 + clover term, per site (12x12)."""
    return clover_term(U, csw) + (4.0 + m0) * np.eye(12)


def clover_blocks(A):
    """Chiral blocks of A: (A_plus on spins {0,1}, A_minus on spins {2,3}), 6x6 each.

    Also returns the largest modulus of the off-diagonal blocks (zero for a
    chirally block-diagonal A)."""
    off = max(np.abs(A[..., :6, 6:]).max(), np.abs(A[..., 6:, :6]).max())
    return A[..., :6, :6], A[..., 6:, 6:], off


def clover_inverse(A):
    """Per-site inverse of A through the inverses of its two 6x6 blocks."""
    ap, am, _ = clover_blocks(A)
    inv = np.zeros_like(A)
    inv[..., :6, :6] = np.linalg.inv(ap)
    inv[..., 6:, 6:] = np.linalg.inv(am)
    return inv


def apply_site_matrix(M, psi):
    """Apply per-site 12x12 matrices to psi[..., t, z, y, x, 4, 3]."""
    shp = psi.shape
    v = psi.reshape(shp[:-2] + (12,))
    out = np.matmul(M, v[..., None])[..., 0]
    return out.reshape(shp)


# --- the Dirac matrix -----------------------------------------------------------

class WilsonClover:
    """D(m0) on a fixed gauge field (links, clover term and BC captured once)."""

    def __init__(self, U, m0, csw=1.0, antiperiodic_t=True):
        self.U = np.ascontiguousarray(U)
        self.m0 = float(m0)
        self.csw = float(csw)
        self.antiperiodic_t = antiperiodic_t
        self.dims = dims_of(U)
        self.A = clover_matrix(self.U, self.m0, self.csw)
        self._Ainv = None

    @property
    def Ainv(self):
        if self._Ainv is None:
            self._Ainv = clover_inverse(self.A)
        return self._Ainv

    def hop(self, psi, dagger=False):
        return hop(self.U, psi, self.antiperiodic_t, dagger)

    def apply(self, psi):
        """D psi = A psi - 1/2 H psi."""
        return apply_site_matrix(self.A, psi) - 0.5 * self.hop(psi)

    def apply_dagger(self, psi):
        """D^dagger psi = gamma5 D gamma5 psi (A is Hermitian and commutes with gamma5)."""
        return apply_site_matrix(self.A, psi) - 0.5 * self.hop(psi, dagger=True)

    def dense(self):
        """The full (12 V) x (12 V) matrix, columns = D applied to unit vectors."""
        lx, ly, lz, lt = self.dims
        n = 12 * lx * ly * lz * lt
        eye = np.eye(n, dtype=np.complex128).reshape((n, lt, lz, ly, lx, 4, 3))
        cols = self.apply(eye).reshape(n, n)
        return cols.T.copy()


# --- even-odd (Schur complement) pieces ---------------------------------------

def parity_mask(dims):
    """1.0 on even sites ((x+y+z+t) even), 0.0 on odd, shape (t, z, y, x, 1, 1)."""
    lx, ly, lz, lt = dims
    t, z, y, x = np.meshgrid(np.arange(lt), np.arange(lz), np.arange(ly), np.arange(lx),
                             indexing="ij")
    even = ((x + y + z + t) % 2 == 0).astype(np.float64)
    return even[..., None, None]


class EvenOdd:
    """Symmetric even-odd Schur complement of D on the full-lattice arrays.

        M_hat  = 1_e - 1/4 A_ee^-1 H_eo A_oo^-1 H_oe
        b_hat  = A_ee^-1 (b_e + 1/2 H_eo A_oo^-1 b_o)
        x_o    = A_oo^-1 (b_o + 1/2 H_oe x_e)

    Fields live on the whole lattice; ``e``/``o`` are the parity masks."""

    def __init__(self, D):
        self.D = D
        self.e = parity_mask(D.dims)
        self.o = 1.0 - self.e

    def Ainv(self, psi):
        return apply_site_matrix(self.D.Ainv, psi)

    def M_hat(self, xe):
        t = self.o * self.Ainv(self.o * self.D.hop(self.e * xe))
        return self.e * xe - 0.25 * self.e * self.Ainv(self.e * self.D.hop(t))

    def prepare(self, b):
        t = self.o * self.Ainv(self.o * b)
        return self.e * self.Ainv(self.e * b + 0.5 * self.e * self.D.hop(t))

    def reconstruct(self, b, xe):
        xo = self.o * self.Ainv(self.o * b + 0.5 * self.o * self.D.hop(self.e * xe))
        return self.e * xe + xo


# --- sampled outputs ------------------------------------------------------------

def _patch(U, t, z, y, x):
    """The 3^4 block of links around site (t, z, y, x), periodic in every direction."""
    lt, lz, ly, lx = U.shape[:4]
    it = [(t + d) % lt for d in (-1, 0, 1)]
    iz = [(z + d) % lz for d in (-1, 0, 1)]
    iy = [(y + d) % ly for d in (-1, 0, 1)]
    ix = [(x + d) % lx for d in (-1, 0, 1)]
    return U[np.ix_(it, iz, iy, ix)]


def clover_matrix_at(U, site, m0, csw):
    """A(x) at one site: the clover leaves at x only touch links within distance 1,
    so the whole-field construction on the periodic 3^4 block around x gives A(x)
    at the block's centre."""
    t, z, y, x = site
    return clover_matrix(_patch(U, t, z, y, x), m0, csw)[1, 1, 1, 1]


def clover_inverse_at(U, site, m0, csw):
    """A(x)^-1 at one site (the inverse of each chiral block of clover_matrix_at)."""
    return clover_inverse(clover_matrix_at(U, site, m0, csw)[None])[0]


def hop_at_sites(U, psi, sites, antiperiodic_t=True, dagger=False):
    """(H psi)(x) (dagger: gamma5 H gamma5) at the listed sites (t, z, y, x), straight
    from the definition, one neighbour at a time; psi has a leading RHS axis.
    Returns (nrhs, nsites, 4, 3)."""
    lt, lz, ly, lx = U.shape[:4]
    ext = (lx, ly, lz, lt)
    sg = -1.0 if dagger else 1.0
    out = np.zeros((psi.shape[0], len(sites), 4, 3), dtype=np.complex128)
    for i, (t, z, y, x) in enumerate(sites):
        c = [x, y, z, t]
        hop = np.zeros((psi.shape[0], 4, 3), dtype=np.complex128)
        for mu in range(4):
            for k in (+1, -1):
                n = list(c)
                n[mu] += k
                eta = 1.0
                if n[mu] == ext[mu] or n[mu] < 0:
                    n[mu] %= ext[mu]
                    if mu == 3 and antiperiodic_t:
                        eta = -1.0
                nb = psi[:, n[3], n[2], n[1], n[0]]
                if k > 0:
                    link = U[t, z, y, x, mu]
                    spin = np.eye(4) - sg * GAMMA[mu]
                else:
                    link = dag(U[n[3], n[2], n[1], n[0], mu])
                    spin = np.eye(4) + sg * GAMMA[mu]
                w = eta * np.einsum("ab,rsb->rsa", link, nb)
                hop += np.einsum("st,rta->rsa", spin, w)
        out[:, i] = hop
    return out


def apply_at_sites(U, psi, sites, m0, csw, antiperiodic_t=True, dagger=False):
    """(D psi)(x) (or D^dagger) at the listed sites (t, z, y, x), straight from the
    definition; psi has a leading RHS axis.  Returns (nrhs, nsites, 4, 3)."""
    hop = hop_at_sites(U, psi, sites, antiperiodic_t, dagger)
    out = np.zeros_like(hop)
    for i, (t, z, y, x) in enumerate(sites):
        A = clover_matrix_at(U, (t, z, y, x), m0, csw)
        v = psi[:, t, z, y, x].reshape(-1, 12)
        out[:, i] = (v @ A.T).reshape(-1, 4, 3) - 0.5 * hop[:, i]
    return out
