"""GPU meson doublets and baryon triplets of the LapH vectors, against the oracle.

* small lattices (one full K chunk, a ragged chunk tail, one and several column
  tiles, nev from the minimum 3 to the maximum 64, 18 momenta for the launch
  groups): every entry against the oracle's einsum, relative to the largest entry,
  within 1e-12;
* the perambulator lattice 32^3 x 64 with nev 64: sampled entries against the
  oracle on the sampled vectors alone, the zero-momentum doublets against the
  identity (orthonormal vectors), and the antisymmetry of the full triplet tensor;
* invalid arguments raise.
"""
import numpy as np
import pytest
import torch

import laph_synth as ls
from gpu_common import dev, host, log_case, require_gpu
from oracle import laph as olaph

pytestmark = pytest.mark.gpu

MOMS = [(0, 0, 0), (1, 0, 0), (0, -1, 2), (3, 1, -1)]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _lattice(dims):
    import paper_2510_26313_amd as laph
    return laph.Lattice(dims)


def _vectors(dims, nev, seed):
    lx, ly, lz, lt = dims
    return ls.random_spinor((lt, nev, lz, ly, lx, 3), seed)


def _close(got, ref, tol=1e-12):
    scale = np.abs(ref).max()
    err = np.abs(got - ref).max()
    assert err <= tol * scale, (err, scale)


@pytest.mark.parametrize("dims,nev", [((4, 4, 4, 4), 8), ((6, 6, 6, 4), 20), ((4, 4, 4, 6), 3), ((4, 4, 4, 4), 64)])
def test_doublets_vs_oracle(dims, nev):
    V = _vectors(dims, nev, 700 + nev)
    lat = _lattice(dims)
    log_case("meson_doublets", dims=dims, nev=nev)
    got = host(lat.meson_doublets(dev(V), MOMS))
    _close(got, olaph.meson_doublets(V, MOMS))


@pytest.mark.parametrize("dims,nev", [((4, 4, 4, 4), 8), ((6, 6, 6, 4), 20), ((4, 4, 4, 6), 3), ((4, 4, 4, 4), 64)])
def test_triplets_vs_oracle(dims, nev):
    V = _vectors(dims, nev, 800 + nev)
    lat = _lattice(dims)
    moms = MOMS if nev < 64 else MOMS[:2]
    log_case("baryon_triplets", dims=dims, nev=nev)
    got = host(lat.baryon_triplets(dev(V), moms))
    _close(got, olaph.baryon_triplets(V, moms))


def test_many_momenta():
    """More momenta than one launch takes: the launch groups write their own slices."""
    dims, nev = (4, 4, 4, 4), 6
    moms = [(a, b, c) for a in (0, 1, -1) for b in (0, 2) for c in (0, 1, 3)]
    assert len(moms) == 18
    V = _vectors(dims, nev, 901)
    lat = _lattice(dims)
    log_case("contractions 18 momenta", dims=dims, nev=nev)
    _close(host(lat.meson_doublets(dev(V), moms)), olaph.meson_doublets(V, moms))
    _close(host(lat.baryon_triplets(dev(V), moms)), olaph.baryon_triplets(V, moms))


def test_full_lattice_sampled():
    cfg = ls.CONFIGS["perambulator_32x32x32x64"]
    dims, nev = cfg["dims"], cfg["nev"]
    V = ls.orthonormal_laph_vectors(dims, nev, cfg["seed_v"])
    lat = _lattice(dims)
    moms = [(0, 0, 0), (1, 1, 0)]
    Vd = dev(V)
    log_case("meson_doublets full", dims=dims, nev=nev)
    phi = host(lat.meson_doublets(Vd, moms))
    assert np.abs(phi[0] - np.eye(nev)[None]).max() <= 1e-12
    log_case("baryon_triplets full", dims=dims, nev=nev)
    B = lat.baryon_triplets(Vd, moms)
    torch.cuda.synchronize()
    # antisymmetry of the whole tensor, checked on the device
    assert torch.equal(B, -B.transpose(2, 3)) and torch.equal(B, -B.transpose(3, 4))
    rng = np.random.default_rng(5)
    for _ in range(6):
        t = int(rng.integers(dims[3]))
        l, m, n = (int(v) for v in rng.choice(nev, 3, replace=False))
        sub = V[t:t + 1, [l, m, n]]
        ref_b = olaph.baryon_triplets(sub, moms)[:, 0, 0, 1, 2]
        got_b = host(B[:, t, l, m, n])
        assert np.abs(got_b - ref_b).max() <= 1e-12 * max(np.abs(ref_b).max(), 1e-3), (t, l, m, n)
        ref_p = olaph.meson_doublets(V[t:t + 1, [l, m]], moms)[:, 0, 0, 1]
        assert np.abs(phi[:, t, l, m] - ref_p).max() <= 1e-12, (t, l, m)


def test_invalid_arguments():
    import paper_2510_26313_amd as laph
    dims = (4, 4, 4, 4)
    lat = _lattice(dims)
    with pytest.raises(laph.LaphError):
        lat.baryon_triplets(dev(_vectors(dims, 2, 1)), MOMS)
    with pytest.raises(laph.LaphError):
        lat.meson_doublets(dev(_vectors(dims, 65, 1)), MOMS)
    with pytest.raises(laph.LaphError):
        lat.meson_doublets(dev(_vectors(dims, 4, 1)), np.zeros((0, 3), dtype=np.int32))
