"""Oracle: plain FP64 solvers for D x = b.

Test infrastructure only (see ``oracle/__init__.py``).

The paper obtains quark propagators with an iterative Dirac-matrix solver
(Sec. "QUDA"); the method's result is x = D^-1 b whatever the route, so the
oracle solves the full, unpreconditioned system:

* ``dense_solve``: LU of the explicit matrix (small lattices only);
* ``bicgstab``: van der Vorst's BiCGStab with <a, b> = sum conj(a) b, x0 = 0,
  shadow residual r_hat = r0, independent scalars per right-hand side (the
  leading axis), followed by a true-residual check that restarts from the true
  residual when the recursive one has drifted.
"""
import numpy as np


def _dot(a, b):
    """Per-RHS inner product <a, b> = sum conj(a) b over all non-RHS axes."""
    n = a.shape[0]
    return np.einsum("ij,ij->i", np.conj(a.reshape(n, -1)), b.reshape(n, -1))


def _norm(a):
    return np.sqrt(np.maximum(_dot(a, a).real, 0.0))


def _bcast(s, like):
    return s.reshape((-1,) + (1,) * (like.ndim - 1))


def dense_solve(D, b):
    """x = D^-1 b through LU of the explicit matrix (b has a leading RHS axis)."""
    m = D.dense()
    n = m.shape[0]
    rhs = b.reshape(b.shape[0], n).T
    x = np.linalg.solve(m, rhs)
    return x.T.reshape(b.shape)


def bicgstab(apply, b, tol=1e-13, maxiter=10000, max_restarts=20, x0=None):
    """Solve apply(x) = b for every RHS to ||b - apply(x)|| <= tol ||b||.

    Returns (x, info) with info = dict(iters, restarts, true_res) per RHS."""
    b = np.asarray(b, dtype=np.complex128)
    nr = b.shape[0]
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.complex128)
    bnorm = _norm(b)
    bnorm_safe = np.where(bnorm > 0, bnorm, 1.0)
    iters = np.zeros(nr, dtype=np.int64)
    restarts = np.zeros(nr, dtype=np.int64)
    done = bnorm == 0
    for _ in range(max_restarts + 1):
        r = b - apply(x)
        true_res = _norm(r) / bnorm_safe
        done = done | (true_res <= tol)
        if done.all():
            break
        active = ~done
        r_hat = r.copy()
        rho_old = np.ones(nr, dtype=np.complex128)
        alpha = np.ones(nr, dtype=np.complex128)
        omega = np.ones(nr, dtype=np.complex128)
        v = np.zeros_like(b)
        p = np.zeros_like(b)
        for _ in range(maxiter):
            rho = _dot(r_hat, r)
            breakdown = np.abs(rho) < 1e-300 * _norm(r) * _norm(r_hat) + 1e-300
            beta = np.where(active & ~breakdown,
                            (rho / np.where(rho_old == 0, 1, rho_old))
                            * (alpha / np.where(omega == 0, 1, omega)), 0)
            p = r + _bcast(beta, p) * (p - _bcast(omega, v) * v)
            v = apply(p)
            sig = _dot(r_hat, v)
            ok = active & ~breakdown & (np.abs(sig) > 0)
            alpha = np.where(ok, rho / np.where(sig == 0, 1, sig), 0)
            s = r - _bcast(alpha, v) * v
            t = apply(s)
            tt = _dot(t, t).real
            omega = np.where(ok & (tt > 0), _dot(t, s) / np.where(tt == 0, 1, tt), 0)
            x = x + _bcast(alpha, p) * p + _bcast(omega, s) * s
            r = np.where(_bcast(ok, s), s - _bcast(omega, t) * t, r)
            rho_old = rho
            iters += ok
            # stop iterating an RHS on convergence of the recursive residual or breakdown
            active = active & ok & (_norm(r) > tol * bnorm_safe) & (omega != 0)
            if not active.any():
                break
        restarts += ~done
    r = b - apply(x)
    info = dict(iters=iters, restarts=restarts, true_res=_norm(r) / bnorm_safe)
    return x, info


def solve(D, b, tol=1e-13, method="bicgstab"):
    """x = D^-1 b (leading RHS axis) by the named route."""
    if method == "dense":
        return dense_solve(D, b), None
    return bicgstab(D.apply, b, tol=tol)
