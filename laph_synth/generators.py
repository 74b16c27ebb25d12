"""Seeded generators for gauge links, LapH colour vectors and test spinors.

Every generator takes an explicit integer seed and uses numpy's PCG64, so a
given (shape, seed) always yields the same array on any machine.
"""
import numpy as np


def _rng(seed):
    return np.random.Generator(np.random.PCG64(int(seed)))


def gauge_shape(dims):
    """Shape of a gauge field for lattice extents ``dims = (Lx, Ly, Lz, Lt)``."""
    lx, ly, lz, lt = dims
    return (lt, lz, ly, lx, 4, 3, 3)


def spinor_shape(dims, nrhs=None):
    """Shape of a spinor field (optionally with a leading RHS axis)."""
    lx, ly, lz, lt = dims
    s = (lt, lz, ly, lx, 4, 3)
    return s if nrhs is None else (nrhs,) + s


def _dag(m):
    return np.conj(np.swapaxes(m, -1, -2))


def _reunitarise_rows(u):
    """Gram-Schmidt on rows 0 and 1, row 2 = conj(row0 x row1): det = 1."""
    r0 = u[..., 0, :]
    r0 = r0 / np.linalg.norm(r0, axis=-1, keepdims=True)
    r1 = u[..., 1, :]
    r1 = r1 - np.sum(np.conj(r0) * r1, axis=-1, keepdims=True) * r0
    r1 = r1 / np.linalg.norm(r1, axis=-1, keepdims=True)
    r2 = np.conj(np.cross(r0, r1))
    return np.stack([r0, r1, r2], axis=-2)


def gauge_field(dims, seed, eps=0.3, chunk=1 << 20):
    """Synthetic SU(3) links ``U = exp(i*eps*H)``, reunitarised.

    ``A = Re + i Im`` with ``Re`` and then ``Im`` drawn as standard normals over
    the whole link array; ``H = (A + A^dagger)/2`` minus its trace part; the
    exponential is taken through the eigen-decomposition of ``H``; rows are then
    re-orthonormalised and the third row rebuilt so that ``det U = 1``.
    """
    shape = gauge_shape(dims)
    rng = _rng(seed)
    re = rng.standard_normal(shape)
    im = rng.standard_normal(shape)
    flat_re = re.reshape(-1, 3, 3)
    flat_im = im.reshape(-1, 3, 3)
    out = np.empty((flat_re.shape[0], 3, 3), dtype=np.complex128)
    eye = np.eye(3)
    for s in range(0, flat_re.shape[0], chunk):
        a = flat_re[s:s + chunk] + 1j * flat_im[s:s + chunk]
        h = 0.5 * (a + _dag(a))
        tr = np.trace(h, axis1=-2, axis2=-1).real
        h = h - (tr / 3.0)[:, None, None] * eye
        w, q = np.linalg.eigh(h)
        u = (q * np.exp(1j * eps * w)[:, None, :]) @ _dag(q)
        out[s:s + chunk] = _reunitarise_rows(u)
    return out.reshape(shape)


def unit_gauge(dims):
    """The free field: every link is the 3x3 identity."""
    u = np.zeros(gauge_shape(dims), dtype=np.complex128)
    u[..., 0, 0] = u[..., 1, 1] = u[..., 2, 2] = 1.0
    return u


def random_su3(n, seed):
    """``n`` Haar-random SU(3) matrices (QR of complex Gaussians, phases fixed)."""
    rng = _rng(seed)
    z = rng.standard_normal((n, 3, 3)) + 1j * rng.standard_normal((n, 3, 3))
    q, r = np.linalg.qr(z)
    d = np.diagonal(r, axis1=-2, axis2=-1)
    q = q * (d / np.abs(d))[:, None, :]
    det = np.linalg.det(q)
    q = q * (det ** (-1.0 / 3.0))[:, None, None]
    return _reunitarise_rows(q)


def orthonormal_laph_vectors(dims, nev, seed):
    """Stand-in LapH vectors: per timeslice, ``nev`` orthonormal colour fields.

    For t = 0 .. Lt-1 in order a complex Gaussian matrix ``G`` of shape
    ``(3*Lx*Ly*Lz, nev)`` is drawn (real part, then imaginary part) and
    orthonormalised by QR with the phases of ``diag(R)`` moved into ``Q`` so
    that ``diag(R) > 0``.  Returns ``V[t][l][z][y][x][a]`` (complex128).
    """
    lx, ly, lz, lt = dims
    n3 = 3 * lx * ly * lz
    rng = _rng(seed)
    v = np.empty((lt, nev, lz, ly, lx, 3), dtype=np.complex128)
    for t in range(lt):
        g = rng.standard_normal((n3, nev)) + 1j * rng.standard_normal((n3, nev))
        q, r = np.linalg.qr(g)
        d = np.diagonal(r)
        q = q * (d / np.abs(d))[None, :]
        v[t] = q.T.reshape(nev, lz, ly, lx, 3)
    return v


def random_spinor(shape, seed, dtype=np.complex128):
    """Complex Gaussian field of the given shape (real part drawn first)."""
    rng = _rng(seed)
    re = rng.standard_normal(shape)
    im = rng.standard_normal(shape)
    return (re + 1j * im).astype(dtype)
