"""The site windows that restrict the perambulator's source preparation to the
timeslices around t0 (a cyclic range of checkerboard indices), checked on the CPU
against a brute-force reading: a site h of either parity lies on timeslice
h // (lx ly lz / 2), the slab t0 - k .. t0 + k wraps periodically, and a block of
sites is skipped only when none of its sites is in the window."""
import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    if not (os.path.exists(HIPCC) or shutil.which("hipcc")):
        pytest.skip("hipcc not available")
    exe = str(tmp_path_factory.mktemp("win") / "window_check")
    src = os.path.join(ROOT, "tests", "host", "window_check.cpp")
    r = subprocess.run([HIPCC, "-std=c++17", "--offload-arch=gfx950", "-O1", "-x", "hip", src, "-o", exe],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-4000:]
    return exe


def run(exe, lines):
    r = subprocess.run([exe], input="\n".join(lines) + "\n", capture_output=True, text=True, timeout=60)
    assert r.returncode == 0, r.stderr
    return [tuple(int(v) for v in ln.split()) for ln in r.stdout.splitlines()]


def test_slab_window_is_the_timeslices_around_t0(checker):
    cases, want = [], []
    for dims in [(6, 4, 4, 10), (4, 4, 4, 4), (8, 4, 2, 6), (4, 2, 2, 2), (4, 2, 2, 1)]:
        lx, ly, lz, lt = dims
        vs_h = lx * ly * lz // 2
        for t0 in range(lt):
            for k in (0, 1, 2):
                cases.append("slab %d %d %d %d %d %d" % (lx, ly, lz, lt, t0, k))
                slices = {(t0 + d) % lt for d in range(-k, k + 1)}
                if 2 * k + 1 >= lt:
                    want.append((0, 0))
                else:
                    want.append((((t0 - k) % lt) * vs_h, (2 * k + 1) * vs_h))
                    # the range covers exactly those timeslices
                    lo, n = want[-1]
                    vh = vs_h * lt
                    covered = {((lo + d) % vh) // vs_h for d in range(n)}
                    assert covered == slices
    assert run(checker, cases) == want


def test_window_membership_and_block_skip(checker):
    rng = np.random.default_rng(7)
    cases, want = [], []
    for _ in range(3000):
        vh = int(rng.integers(1, 300))
        lo = int(rng.integers(0, vh))
        n = int(rng.integers(-2, vh + 1))
        h0 = int(rng.integers(0, vh))
        cnt = int(rng.integers(1, vh - h0 + 1))
        cases.append("win %d %d %d %d %d" % (vh, lo, n, h0, cnt))
        inside = [n <= 0 or ((h - lo) % vh) < n for h in range(vh)]
        want.append((int(inside[h0]), int(not any(inside[h0:h0 + cnt]))))
    assert run(checker, cases) == want
