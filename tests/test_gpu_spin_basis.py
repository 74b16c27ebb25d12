"""GPU spin-basis rotation of perambulators against the oracle: random blocks (also in
place), and the 4^4 perambulator in the Dirac-Pauli basis."""
import numpy as np
import pytest

import laph_synth as ls
from gpu_common import dev, host, log_case, make_lattice, rel, require_gpu
from oracle import laph

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def test_spin_rotate_random_blocks():
    dims = (4, 4, 4, 6)
    U = ls.gauge_field(dims, 91)
    lat = make_lattice(dims, U)
    rng = np.random.default_rng(92)
    tau = rng.standard_normal((6, 5, 3, 4, 4)) + 1j * rng.standard_normal((6, 5, 3, 4, 4))
    S, _ = np.linalg.qr(rng.standard_normal((4, 4)) + 1j * rng.standard_normal((4, 4)))
    ref = laph.spin_rotate(tau, S)
    log_case("spin_rotate")
    t = dev(tau)
    assert np.abs(host(lat.spin_rotate(t, S)) - ref).max() <= 1e-14 * np.abs(ref).max()
    lat.spin_rotate(t, S, out=t)
    assert np.abs(host(t) - ref).max() <= 1e-14 * np.abs(ref).max()


def test_perambulator_dirac_pauli_c0():
    import paper_2510_26313_amd as pl
    cfg = ls.CONFIGS["dense_4x4x4x4"]
    U = ls.gauge_field(cfg["dims"], cfg["seed_u"])
    V, _, _ = laph.laplacian_eigvecs(U, cfg["nev"])
    tau_ref, _ = laph.perambulator(U, V, 0, cfg["masses"][0], method="dense")
    lat = make_lattice(cfg["dims"], U, masses=cfg["masses"])
    log_case("perambulator_dirac_pauli_c0")
    tau, _ = lat.perambulator_raw(dev(V), 0, 0, 1e-12, pl.default_params(inner_prec="f64"))
    got = host(lat.spin_rotate(tau, pl.DIRAC_PAULI))
    assert rel(got, laph.spin_rotate(tau_ref, pl.DIRAC_PAULI)) < 1e-9
