"""The package's Dirac-Pauli basis matrix (CPU): unitary, gamma_t diagonal with the upper
components first, gamma_5 the block swap, starting from the oracle's DeGrand-Rossi
gamma matrices."""
import numpy as np

from oracle import dirac


def test_dirac_pauli_matrix():
    from paper_2510_26313_amd import DIRAC_PAULI as S
    assert np.abs(S @ S.conj().T - np.eye(4)).max() < 1e-15
    gt = S @ dirac.GAMMA[3] @ S.conj().T
    assert np.abs(gt - np.diag([1, 1, -1, -1])).max() < 1e-15
    g5 = S @ dirac.GAMMA5 @ S.conj().T
    swap = np.block([[np.zeros((2, 2)), np.eye(2)], [np.eye(2), np.zeros((2, 2))]])
    assert np.abs(g5 - swap).max() < 1e-15
