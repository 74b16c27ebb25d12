"""Oracle: the FP16-with-per-site-norm storage format, emulated with numpy.

Test infrastructure only (see ``oracle/__init__.py``).

The paper runs its bandwidth-bound sparse work in reduced precision (Sec.
"QUDA", mixed precision).  The half-precision storage read here: per site and
right-hand side, the 24 reals ``v`` of a spinor are held as IEEE binary16 codes
scaled by one FP32 norm

    n = max_i |fp32(v_i)|,   s = 1/n (FP32, correctly rounded),
    q_i = fp16_rne(fp32(fp32(v_i) * s)),   decode v'_i = fp32(q_i) * n (FP32)

with all-zero codes when n = 0.  Every rounding step is taken in the same
precision the kernels use, so codes can be compared bit for bit.
"""
import numpy as np


def encode(v):
    """v: real array (..., 24).  Returns (codes float16 (..., 24), norms float32 (...))."""
    v32 = np.asarray(v, dtype=np.float32)
    n = np.max(np.abs(v32), axis=-1)
    with np.errstate(divide="ignore"):
        s = np.where(n > 0, np.float32(1.0) / np.where(n > 0, n, np.float32(1.0)), np.float32(0.0))
    s = s.astype(np.float32)
    q = (v32 * s[..., None]).astype(np.float32).astype(np.float16)
    return q, n.astype(np.float32)


def decode(q, n):
    return (q.astype(np.float32) * n[..., None]).astype(np.float32)


def error_bound(n):
    """Per-real bound |v - v'| <= 2^-11 n (plus the FP32 rounding of v, s and the decode)."""
    return np.float64(2.0 ** -11) * n * (1 + 4 * 2.0 ** -23)
