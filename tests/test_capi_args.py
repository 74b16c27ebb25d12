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


_BARRIER_CHILD = r"""
import ctypes, resource, sys
sys.path.insert(0, sys.argv[1])
from paper_2510_26313_amd import _lib as L
lib = L.load()
vm = 0
for line in open("/proc/self/status"):
    if line.startswith("VmSize:"):
        vm = int(line.split()[1]) * 1024
# leave 64 MiB of address space: reading the 256 MiB cache file must fail
resource.setrlimit(resource.RLIMIT_AS, (vm + (64 << 20), resource.RLIM_INFINITY))
out = ctypes.c_void_p()
d = (ctypes.c_int * 4)(4, 4, 4, 4)
st = lib.laph_create(ctypes.byref(out), d, 1, 4, None)
print(st, lib.laph_last_error().decode(), flush=True)
"""


def test_host_allocation_failure_is_a_status_not_an_abort(lib, tmp_path):
    """The C ABI's exception barrier: a host allocation that fails inside a call
    (here reading an oversized autotune cache under a tight address-space limit)
    comes back as LAPH_ERR_HOST with a message; the process does not abort."""
    import subprocess
    import sys
    cache = tmp_path / "tune_cache.txt"
    with open(cache, "wb") as f:
        f.truncate(256 << 20)          # sparse: no disk space, 256 MiB of zeros to read
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    env = dict(os.environ, LAPH_TUNE_CACHE=str(cache))
    r = subprocess.run([sys.executable, "-c", _BARRIER_CHILD, root], env=env, capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 0, (r.returncode, r.stderr[-2000:])
    status, msg = r.stdout.strip().split(" ", 1)
    assert int(status) == L.LAPH_ERR_HOST, r.stdout
    assert "memory" in msg


def test_new_entry_points_validate_arguments(lib):
    buf = ctypes.c_void_p(1)
    g = ctypes.c_double()
    ms = ctypes.c_double()
    assert lib.laph_mass_gradient(None, ctypes.byref(g), buf, buf, 1, buf, 1 << 20) == L.LAPH_ERR_INVALID
    assert lib.laph_stream_copy(None, buf, buf, 16, 1, ctypes.byref(ms)) == L.LAPH_ERR_INVALID
    assert lib.laph_apply_stage(None, 1, buf, buf, None, None, 1, 4, 0, 0, 2, 16, 2, None, buf, 1 << 20) \
        == L.LAPH_ERR_INVALID
    f = ctypes.c_int()
    assert lib.laph_tuned_choice(None, 1, 4, ctypes.byref(f), None, None, None) == L.LAPH_ERR_INVALID
    assert lib.laph_apply_stage_workspace_bytes(None, 4) == 0
    assert lib.laph_mass_gradient_workspace_bytes(None) == 0
