"""Write golden perambulator columns for the two large workloads from the FP64 oracle only.

A perambulator column is everything one source produces: for RHS r = 4k + alpha
of a source time t0, tau[t][l][k][beta][alpha] over all sinks t, LapH vectors l
and sink spins beta (shape [T][nev][4]).  The oracle solves the full,
unpreconditioned system by BiCGStab to a relative residual of 1e-13 and projects
with the plain contraction.  Written here:

* ``tau_columns_32x32x32x64.npz``: the perambulator workload (32^3 x 64, m0 0.02,
  nev 64), one source per source time t0 in {0, 16, 32, 48};
* ``tau_columns_24x24x24x48.npz``: the multi-mass workload (24^3 x 48, t0 = 0,
  RHS 0/39 at m0 0.02, 40/111 at 0.05, 112/175 at 0.1, 176/255 at 0.2: the
  edges of each mass range in the 40/72/64/80 split).

Each file holds ``rhs``, ``t0``, ``mass``, ``tau`` (complex128 [n][T][nev][4]),
``true_res`` (the oracle's recomputed residual) and ``x_norm`` (the full
solution's norm per timeslice, [n][T]).  The GPU tests compare the library's
perambulator and batched-solve outputs per column against these arrays.

Run:  python tests/golden/make_tau_columns.py [perambulator_32x32x32x64|multimass_24x24x24x48]
(about 15 minutes per workload on 8 cores).
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import laph_synth as ls  # noqa: E402
from oracle import dirac, laph, solvers  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))

# (t0, rhs) pairs of each workload's golden columns
PICKS = {
    "perambulator_32x32x32x64": [(0, 0), (16, 85), (32, 170), (48, 255)],
    "multimass_24x24x24x48": [(0, r) for r in (0, 39, 40, 111, 112, 175, 176, 255)],
}


def one_source(V, t0, r):
    """The oracle's spin-diluted LapH source of RHS r = 4k + alpha at t0 (one RHS)."""
    k, alpha = divmod(r, 4)
    return laph.laph_sources(V[:, k:k + 1], t0)[alpha:alpha + 1]


def column(V, x, r):
    """tau[:, :, k, :, alpha] of one solution x (leading axis 1) through the oracle's projection."""
    k, alpha = divmod(r, 4)
    X4 = np.zeros((4,) + x.shape[1:], dtype=np.complex128)
    X4[alpha] = x[0]
    return laph.project(V, X4, 1)[:, :, 0, :, alpha]


def main(name):
    cfg = ls.CONFIGS[name]
    dims = cfg["dims"]
    t_start = time.time()
    U = ls.gauge_field(dims, cfg["seed_u"])
    V = ls.orthonormal_laph_vectors(dims, cfg["nev"], cfg["seed_v"])
    mi = ls.rhs_masses(cfg)
    print(name, "inputs", round(time.time() - t_start, 1), "s", flush=True)
    ops = {}
    out = dict(rhs=[], t0=[], mass=[], tau=[], true_res=[], x_norm=[])
    for t0, r in PICKS[name]:
        m = cfg["masses"][mi[r]]
        if m not in ops:
            ops = {m: dirac.WilsonClover(U, m, cfg["csw"])}   # one clover field in memory at a time
        b = one_source(V, t0, r)
        t1 = time.time()
        x, info = solvers.bicgstab(ops[m].apply, b, tol=1e-13)
        print(name, "t0", t0, "rhs", r, "m0", m, "iters", int(info["iters"][0]), "restarts", int(info["restarts"][0]),
              "true_res %.3e" % info["true_res"][0], round(time.time() - t1, 1), "s", flush=True)
        assert info["true_res"][0] <= 1e-13
        out["rhs"].append(r)
        out["t0"].append(t0)
        out["mass"].append(m)
        out["tau"].append(column(V, x, r))
        out["true_res"].append(float(info["true_res"][0]))
        out["x_norm"].append(np.linalg.norm(x[0].reshape(dims[3], -1), axis=1))
    path = os.path.join(HERE, "tau_columns_%s.npz" % name.split("_", 1)[1])
    np.savez(path, **{k: np.asarray(v) for k, v in out.items()})
    print("wrote", path, round(time.time() - t_start, 1), "s", flush=True)


if __name__ == "__main__":
    for nm in (sys.argv[1:] or list(PICKS)):
        main(nm)
