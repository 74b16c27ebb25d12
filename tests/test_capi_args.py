"""CPU-side checks of the C-ABI's argument validation: calls that must fail before
any device work (null context, bad extents, null noise) return LAPH_ERR_INVALID (or a
zero workspace size) and set the thread's error string.  No GPU is touched."""
import ctypes
import os

import pytest

from paper_2510_26313_amd import _lib as L


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(L.LIB_PATH):
        pytest.skip("liblaph.so not built")
    return L.load()


def _err(lib):
    return lib.laph_last_error().decode()


def test_create_rejects_bad_extents(lib):
    out = ctypes.c_void_p()
    for dims in ((3, 4, 4, 4), (4, 4, 4, 5), (4, 4, 2, 4)):
        d = (ctypes.c_int * 4)(*dims)
        assert lib.laph_create(ctypes.byref(out), d, 1, 4, None) == L.LAPH_ERR_INVALID
        assert "even" in _err(lib)
    d = (ctypes.c_int * 4)(4, 4, 4, 4)
    assert lib.laph_create(None, d, 1, 4, None) == L.LAPH_ERR_INVALID
    assert lib.laph_create(ctypes.byref(out), d, 1, 0, None) == L.LAPH_ERR_INVALID


def test_null_context_is_rejected(lib):
    p = L.SolveParams()
    lib.laph_default_params(ctypes.byref(p))
    buf = ctypes.c_void_p(1)
    mom = (ctypes.c_int * 3)(0, 0, 0)
    calls = [
        lambda: lib.laph_meson_doublets(None, buf, buf, 4, 1, mom, buf, 1 << 20),
        lambda: lib.laph_baryon_triplets(None, buf, buf, 4, 1, mom, buf, 1 << 20),
        lambda: lib.laph_make_noise_sources(None, buf, buf, 4, 0, buf, 2),
        lambda: lib.laph_stochastic_perambulator(None, buf, buf, 4, 0, 0, buf, 2, 1e-10, ctypes.byref(p), None,
                                                 buf, 1 << 20),
        lambda: lib.laph_perambulator(None, buf, buf, 4, 0, 0, 1e-10, ctypes.byref(p), None, buf, 1 << 20),
        lambda: lib.laph_laplacian_eigvecs(None, buf, buf, 4, 1e-10, 10, 0, buf, 1 << 20, None, None),
        lambda: lib.laph_make_sources(None, buf, buf, 4, 0),
        lambda: lib.laph_spin_rotate(None, buf, buf, 1, buf),
    ]
    for call in calls:
        assert call() == L.LAPH_ERR_INVALID
        assert _err(lib)


def test_stochastic_perambulator_needs_noise(lib):
    p = L.SolveParams()
    lib.laph_default_params(ctypes.byref(p))
    buf = ctypes.c_void_p(1)
    st = lib.laph_stochastic_perambulator(None, buf, buf, 4, 0, 0, None, 2, 1e-10, ctypes.byref(p), None, buf, 1)
    assert st == L.LAPH_ERR_INVALID and "noise" in _err(lib)


def test_workspace_queries_without_context(lib):
    assert lib.laph_contract_workspace_bytes(None, 1, 8, 1) == 0
    assert lib.laph_laplacian_workspace_bytes(None, 8) == 0
    p = L.SolveParams()
    lib.laph_default_params(ctypes.byref(p))
    assert lib.laph_perambulator_workspace_bytes(None, 8, ctypes.byref(p)) == 0
