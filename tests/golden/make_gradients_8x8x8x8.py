"""Write tests/golden/gradients_8x8x8x8.json from the FP64 oracle only.

The gradient workload (8^4, m0 = 0.05, c_sw = 1, N_ev = 16 seeded orthonormal LapH vectors,
64 spin-diluted sources at t0 = 0, L = sum |tau[t_sink = 4]|^2): the loss, the
adjoint-formula gradients with respect to m0 and to the sources, and central
differences at h = 1e-4 along seeded directions (one supported on the t0 slice,
one on the full lattice) and for 8 single source components.  The GPU
gradient test compares against these numbers.

Run:  python tests/golden/make_gradients_8x8x8x8.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import laph_synth as ls  # noqa: E402
from oracle import dirac, laph, solvers  # noqa: E402


def directions(shape, seed):
    """The two seeded unit directions: [0] on the t0 = 0 slice, [1] on the full lattice."""
    d_full = ls.random_spinor(shape, seed)
    d_slice = np.zeros_like(d_full)
    d_slice[:, 0] = ls.random_spinor(d_full[:, 0].shape, seed + 1)
    return d_slice / np.linalg.norm(d_slice), d_full / np.linalg.norm(d_full)


def single_components(shape, seed, n=8):
    rng = np.random.default_rng(seed)
    idx = []
    for _ in range(n):
        idx.append(tuple(int(rng.integers(0, s)) for s in shape))
    return idx


def main():
    cfg = ls.CONFIGS["gradients_8x8x8x8"]
    dims, m0, csw, ts, h = cfg["dims"], cfg["masses"][0], cfg["csw"], cfg["t_sink"], cfg["fd_h"]
    U = ls.gauge_field(dims, cfg["seed_u"])
    V = ls.orthonormal_laph_vectors(dims, cfg["nev"], cfg["seed_v"])
    D = dirac.WilsonClover(U, m0, csw)
    b = laph.laph_sources(V, 0)
    L, Z, gm, X = laph.adjoint_gradients(D, V, b, ts)
    print("L", L, "grad_m0", gm, flush=True)
    fd_m = laph.fd_mass(U, V, b, m0, csw, ts, h=h)
    print("fd_m0", fd_m, flush=True)
    out = dict(config="gradients_8x8x8x8", dims=list(dims), m0=m0, csw=csw, t_sink=ts, h=h, L=L, grad_m0=gm, fd_m0=fd_m,
               grad_b_norm=float(np.linalg.norm(Z)), directions=[], components=[])
    for name, d in zip(("t0_slice", "full"), directions(b.shape, cfg["seed_fd"])):
        fd = laph.fd_source(D, V, b, d, ts, h=h)
        an = float(np.real(np.vdot(Z, d)))
        print(name, an, fd, flush=True)
        out["directions"].append(dict(name=name, adjoint=an, fd=fd))
    # single components: only RHS r changes, so re-solve that RHS alone
    for idx in single_components(b.shape, cfg["seed_fd"] + 7):
        r = idx[0]
        vals = []
        for sgn in (+1, -1):
            bb = b[r:r + 1].copy()
            bb[(0,) + idx[1:]] += sgn * h
            xr, _ = solvers.bicgstab(D.apply, bb, tol=1e-13)
            Xp = X.copy()
            Xp[r] = xr[0]
            vals.append(laph.loss_from_tau(laph.project(V, Xp, b.shape[0] // 4), ts))
        fd = (vals[0] - vals[1]) / (2 * h)
        an = float(np.real(Z[idx]))
        print("component", idx, an, fd, flush=True)
        out["components"].append(dict(index=list(idx), adjoint=an, fd=fd))
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "gradients_8x8x8x8.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()
