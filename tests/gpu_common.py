"""Shared helpers of the GPU tests: seeded inputs moved to the device, the
oracle's answers on the same inputs, and the comparison metrics."""
import numpy as np
import pytest
import torch

import laph_synth as ls


def require_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def per_rhs_rel(a, b):
    n = a.shape[0]
    a = np.asarray(a).reshape(n, -1)
    b = np.asarray(b).reshape(n, -1)
    return np.linalg.norm(a - b, axis=1) / np.maximum(np.linalg.norm(b, axis=1), 1e-300)


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def parity_mask(dims):
    lx, ly, lz, lt = dims
    t, z, y, x = np.meshgrid(np.arange(lt), np.arange(lz), np.arange(ly), np.arange(lx), indexing="ij")
    return ((x + y + z + t) % 2).astype(np.int64)


def make_lattice(dims, U, masses=(0.1,), csw=1.0, antiperiodic=True):
    import paper_2510_26313_amd as laph
    lat = laph.Lattice(dims, t_antiperiodic=antiperiodic, n_mass_max=max(8, len(masses)))
    lat.load_gauge(dev(U))
    lat.set_masses(masses, csw)
    return lat


def log_case(name, **kw):
    """Print (and flush) what the next GPU step runs, so a failing run names it."""
    print("[gpu case] %s %s" % (name, " ".join("%s=%s" % kv for kv in kw.items())), flush=True)


def gauge(dims, seed):
    return ls.gauge_field(dims, seed)
