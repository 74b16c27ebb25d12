"""MI355X (gfx950) LapH perambulator library: C ABI (liblaph.so) + thin binding.

    import paper_2510_26313_amd as laph
    lat = laph.Lattice((32, 32, 32, 64))
    lat.load_gauge(U); lat.set_masses([0.02])
    tau = laph.perambulator(lat, V, t0=0, m0=0.02)

All arithmetic runs in the HIP library; importing this package does not load
it (``Lattice`` does, and raises if it has not been built).
"""
from ._lib import EXPORTED, LaphError, LaphNoConvergence, LIB_PATH, load  # noqa: F401
from .api import DIRAC_PAULI, Lattice, default_params, perambulator, project, solve  # noqa: F401
