"""Build liblaph.so (HIP, gfx950) in-tree with hipcc.

Usage: python -m paper_2510_26313_amd.build [--jobs N]
"""
import concurrent.futures
import hashlib
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "liblaph.so")
SOURCES = ["dslash_f64.hip", "dslash_f32.hip", "dslash_f16.hip", "capi.hip", "setup.hip", "dslash.hip",
           "blas.hip", "solver.hip", "project.hip", "tune.hip", "laplace.hip", "contract.hip", "reduce.hip", "mg.hip"]
# The autotuner's cache is keyed by a digest of the sources its choices depend on.
STENCIL_SOURCES = ["dslash_kernels.h", "dslash_lds.h", "laph_internal.h", "dslash_f16.hip", "dslash_f32.hip",
                   "dslash_f64.hip", "dslash.hip", "tune.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # no packed FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
]


def stencil_digest():
    """First 16 hex digits of the SHA-256 of the stencil sources (the autotune cache key)."""
    h = hashlib.sha256()
    for f in STENCIL_SOURCES:
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _compile(src):
    obj = os.path.join(OBJ, src.replace(".hip", ".o"))
    cmd = [HIPCC] + FLAGS + ['-DLAPH_STENCIL_DIGEST="%s"' % stencil_digest(), "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s\n%s" % (src, " ".join(cmd), r.stderr[-8000:]))
    return obj


def build(jobs=None, verbose=True):
    """Compile every HIP source and link liblaph.so next to this file."""
    os.makedirs(OBJ, exist_ok=True)
    jobs = jobs or min(len(SOURCES), os.cpu_count() or 4)
    with concurrent.futures.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s" % r.stderr[-8000:])
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    j = None
    if "--jobs" in sys.argv:
        j = int(sys.argv[sys.argv.index("--jobs") + 1])
    build(j)
