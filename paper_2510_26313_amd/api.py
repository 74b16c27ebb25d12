"""Python binding of liblaph: a context class and differentiable wrappers.

Every computation runs in the HIP library; this module only allocates device
buffers with PyTorch, passes pointers and the current HIP stream, and turns
status codes into exceptions.  Tensors are complex128 on the GPU in the
canonical layouts documented in ``include/laph.h``.
"""
import contextlib
import ctypes

import numpy as np
import torch

from . import _lib as L

# the library's two chiral signs of gamma5 = diag(1, 1, -1, -1) are not needed
# here: the adjoint solve is the library's dagger solve (D^dagger = gamma5 D gamma5)


# A Dirac-Pauli type basis, reached from the library's DeGrand-Rossi (chiral) basis by
# psi' = DIRAC_PAULI psi: gamma_t becomes diag(1, 1, -1, -1) (upper components: positive
# energy at rest) and gamma_5 becomes the off-diagonal block swap.  For laph.spin_rotate.
DIRAC_PAULI = np.array([[1, 0, 1, 0],
                        [0, 1, 0, 1],
                        [1, 0, -1, 0],
                        [0, 1, 0, -1]], dtype=np.complex128) / np.sqrt(2.0)


def default_params(**kw):
    lib = L.load()
    p = L.SolveParams()
    lib.laph_default_params(ctypes.byref(p))
    for k, v in kw.items():
        if k == "inner_prec" and isinstance(v, str):
            v = L.PREC[v]
        if not hasattr(p, k):
            raise TypeError("unknown solver parameter %r" % k)
        setattr(p, k, v)
    return p


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _check_tensor(t, shape, name):
    if not isinstance(t, torch.Tensor) or t.dtype != torch.complex128 or not t.is_cuda:
        raise TypeError("%s must be a complex128 CUDA tensor" % name)
    if tuple(t.shape) != tuple(shape):
        raise ValueError("%s has shape %s, expected %s" % (name, tuple(t.shape), tuple(shape)))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)


def _stats_list(arr, n):
    return [dict(status=L.RHS_STATUS.get(arr[i].status, arr[i].status), iters=arr[i].iters,
                 updates=arr[i].updates, restarts=arr[i].restarts, true_res=arr[i].true_res)
            for i in range(n)]


class Lattice:
    """A lattice context: gauge field, clover term for a set of masses, solver state.

    dims = (Lx, Ly, Lz, Lt); t_antiperiodic selects the fermion time boundary."""

    def __init__(self, dims, t_antiperiodic=True, n_mass_max=8, device="cuda"):
        self.lib = L.load()
        self.dims = tuple(int(d) for d in dims)
        self.device = torch.device(device)
        # a stream of its own (default priority): HIP graphs cannot be captured on
        # the legacy default stream; calls order themselves against the caller's stream
        self.stream = torch.cuda.Stream(self.device)
        self.ctx = ctypes.c_void_p()
        d = (ctypes.c_int * 4)(*self.dims)
        L.check(self.lib.laph_create(ctypes.byref(self.ctx), d, int(bool(t_antiperiodic)), int(n_mass_max),
                                     ctypes.c_void_p(self.stream.cuda_stream)))
        nbytes = self.lib.laph_state_bytes(self.ctx)
        self._state = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        off = (-self._state.data_ptr()) % 256
        L.check(self._run(self.lib.laph_attach_state, self.ctx, ctypes.c_void_p(self._state.data_ptr() + off), nbytes))
        self.masses = ()
        self.csw = None
        self._scratch_buf = None
        lx, ly, lz, lt = self.dims
        self.volume = lx * ly * lz * lt

    @contextlib.contextmanager
    def _on_stream(self):
        cur = torch.cuda.current_stream(self.device)
        self.stream.wait_stream(cur)
        try:
            yield
        finally:
            cur.wait_stream(self.stream)

    def _run(self, fn, *args):
        with self._on_stream():
            return fn(*args)

    def __del__(self):
        try:
            if self.ctx:
                self.lib.laph_destroy(self.ctx)
                self.ctx = ctypes.c_void_p()
        except Exception:
            pass

    # -- shapes -------------------------------------------------------------------
    def gauge_shape(self):
        lx, ly, lz, lt = self.dims
        return (lt, lz, ly, lx, 4, 3, 3)

    def spinor_shape(self, nrhs):
        lx, ly, lz, lt = self.dims
        return (nrhs, lt, lz, ly, lx, 4, 3)

    def laph_shape(self, nev):
        lx, ly, lz, lt = self.dims
        return (lt, nev, lz, ly, lx, 3)

    def _workspace(self, nbytes):
        return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=self.device)

    def _scratch(self, nbytes):
        """Device workspace of one library call: one buffer per lattice, kept between calls
        and grown on demand.  Calls run in order on the lattice's stream, so reuse is safe;
        keeping it avoids re-allocating (and fragmenting) buffers of up to ~180 GB."""
        n = max(int(nbytes), 256)
        if self._scratch_buf is None or self._scratch_buf.numel() < n:
            self._scratch_buf = None
            self._scratch_buf = torch.empty(n, dtype=torch.uint8, device=self.device)
        return self._scratch_buf

    def release_scratch(self):
        """Return the kept workspace to PyTorch's allocator."""
        self._scratch_buf = None

    # -- setup ----------------------------------------------------------------------
    def load_gauge(self, U):
        _check_tensor(U, self.gauge_shape(), "U")
        L.check(self._run(self.lib.laph_load_gauge, self.ctx, _ptr(U)))
        self.masses = ()

    def set_masses(self, masses, csw=1.0):
        masses = tuple(float(m) for m in masses)
        if masses == self.masses and csw == self.csw:
            return
        arr = (ctypes.c_double * len(masses))(*masses)
        L.check(self._run(self.lib.laph_set_clover, self.ctx, float(csw), len(masses), arr))
        self.masses = masses
        self.csw = csw

    def mass_index(self, m0):
        return self.masses.index(float(m0))

    # -- internal-layout operators ----------------------------------------------------
    def field_bytes(self, prec, nrhs, parity_only=True):
        return self.lib.laph_field_bytes(self.ctx, L.PREC[prec], nrhs, int(parity_only))

    def pack(self, psi, prec="f64", parity=-1, out=None, rhs_offset=0):
        """Canonical psi -> internal layout; into RHS slots rhs_offset.. of out if given."""
        n = psi.shape[0]
        _check_tensor(psi, self.spinor_shape(n), "psi")
        per = self.field_bytes(prec, 1, parity >= 0)
        if out is None:
            out = self._workspace(per * n)
            rhs_offset = 0
        elif out.numel() < per * (rhs_offset + n):
            raise ValueError("out holds fewer than rhs_offset + n fields")
        dst = ctypes.c_void_p(out.data_ptr() + per * int(rhs_offset))
        L.check(self._run(self.lib.laph_pack_spinor, self.ctx, dst, _ptr(psi), L.PREC[prec], n, parity))
        return out

    def field_slice(self, buf, prec, rhs, n=1, parity_only=True):
        """The internal fields rhs .. rhs + n - 1 of buf (a view)."""
        per = self.field_bytes(prec, 1, parity_only)
        return buf[per * rhs: per * (rhs + n)]

    def unpack(self, buf, nrhs, prec="f64", parity=-1):
        out = torch.zeros(self.spinor_shape(nrhs), dtype=torch.complex128, device=self.device)
        L.check(self._run(self.lib.laph_unpack_spinor, self.ctx, _ptr(out), _ptr(buf), L.PREC[prec], nrhs, parity))
        return out

    def apply_dslash(self, buf_in, nrhs, out_parity, prec="f64", dagger=False):
        out = self._workspace(self.field_bytes(prec, nrhs, True))
        L.check(self._run(self.lib.laph_apply_dslash, self.ctx, _ptr(out), _ptr(buf_in), out_parity, L.PREC[prec], nrhs,
                                           int(dagger)))
        return out

    def apply_clover(self, buf_in, nrhs, parity, mass_idx=0, inverse=False, prec="f64"):
        out = self._workspace(self.field_bytes(prec, nrhs, True))
        L.check(self._run(self.lib.laph_apply_clover, self.ctx, _ptr(out), _ptr(buf_in), parity, mass_idx, int(inverse),
                                           L.PREC[prec], nrhs))
        return out

    def apply_D(self, psi, mass_idx=0, dagger=False):
        n = psi.shape[0]
        _check_tensor(psi, self.spinor_shape(n), "psi")
        out = torch.empty_like(psi)
        w = self._scratch(self.field_bytes("f64", 2, False))
        L.check(self._run(self.lib.laph_apply_D, self.ctx, _ptr(out), _ptr(psi), mass_idx, n, int(dagger), _ptr(w),
                                      w.numel()))
        return out

    # -- solves ------------------------------------------------------------------------
    def solve_raw(self, B, mass_idx, tol=1e-10, params=None, X0=None, raise_on_noconv=True):
        """X = D^-1 B (or D^dagger^-1 B with params.dagger) for every RHS; returns (X, stats)."""
        n = B.shape[0]
        _check_tensor(B, self.spinor_shape(n), "B")
        p = params if params is not None else default_params()
        if isinstance(mass_idx, int):
            mass_idx = [mass_idx] * n
        mi = (ctypes.c_int * n)(*mass_idx)
        if X0 is not None:
            _check_tensor(X0, self.spinor_shape(n), "X0")
            X = X0.clone()
            p.use_x0 = 1
        else:
            X = torch.empty_like(B)
            p.use_x0 = 0
        w = self._scratch(self.lib.laph_solve_workspace_bytes(self.ctx, n, ctypes.byref(p)))
        stats = (L.RhsStats * n)()
        st = self._run(self.lib.laph_solve, self.ctx, _ptr(X), _ptr(B), n, mi, float(tol), ctypes.byref(p), stats,
                                 _ptr(w), w.numel())
        sl = _stats_list(stats, n)
        if st != L.LAPH_OK and (raise_on_noconv or st != L.LAPH_ERR_NOCONV):
            L.check(st, sl)
        return X, sl

    def perambulator_raw(self, V, t0, mass_idx=0, tol=1e-10, params=None):
        """tau[t][l][k][beta][alpha] for sources at t0 (fused solve + projection)."""
        nev = V.shape[1]
        _check_tensor(V, self.laph_shape(nev), "V")
        p = params if params is not None else default_params()
        lt = self.dims[3]
        tau = torch.zeros((lt, nev, nev, 4, 4), dtype=torch.complex128, device=self.device)
        w = self._scratch(self.lib.laph_perambulator_workspace_bytes(self.ctx, nev, ctypes.byref(p)))
        stats = (L.RhsStats * (4 * nev))()
        st = self._run(self.lib.laph_perambulator, self.ctx, _ptr(tau), _ptr(V), nev, int(t0), int(mass_idx), float(tol),
                                        ctypes.byref(p), stats, _ptr(w), w.numel())
        sl = _stats_list(stats, 4 * nev)
        L.check(st, sl)
        return tau, sl

    def perambulator_workspace_bytes(self, nev, params):
        return self.lib.laph_perambulator_workspace_bytes(self.ctx, nev, ctypes.byref(params))

    def timings(self):
        ms = (ctypes.c_double * 3)()
        L.check(self.lib.laph_last_timings(self.ctx, ms))
        return dict(total_ms=ms[0], solve_ms=ms[1], project_ms=ms[2])

    def time_stages(self, prec, nrhs, rhs_tile=4, mass_idx=0, reps=20, stencil=2, traversal=2):
        """Average ms per launch of the solver's two fused stencil stages (HIP events)."""
        w = self._scratch(self.lib.laph_time_stages_workspace_bytes(self.ctx, L.PREC[prec], nrhs, rhs_tile))
        ms = (ctypes.c_double * 2)()
        L.check(self._run(self.lib.laph_time_stages, self.ctx, L.PREC[prec], nrhs, stencil, rhs_tile, traversal,
                          mass_idx, reps, _ptr(w), w.numel(), ms))
        return ms[0], ms[1]

    def autotune(self, prec, nrhs, mass_idx=0):
        """Measure and keep the fastest stencil form / RHS per link load for this batch size."""
        w = self._scratch(self.lib.laph_time_stages_workspace_bytes(self.ctx, L.PREC[prec], nrhs, 16))
        st, tile, trav, ms = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_double()
        L.check(self._run(self.lib.laph_autotune, self.ctx, L.PREC[prec], nrhs, mass_idx, _ptr(w), w.numel(),
                          ctypes.byref(st), ctypes.byref(tile), ctypes.byref(trav), ctypes.byref(ms)))
        return dict(stencil=st.value, rhs_tile=tile.value, traversal=trav.value, ms=ms.value)

    def tuned_choice(self, prec, nrhs):
        """The stored autotuner choice for (prec, nrhs), or None (nothing is timed)."""
        f, st, tile, trav = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        L.check(self.lib.laph_tuned_choice(self.ctx, L.PREC[prec], int(nrhs), ctypes.byref(f), ctypes.byref(st),
                                           ctypes.byref(tile), ctypes.byref(trav)))
        return dict(stencil=st.value, rhs_tile=tile.value, traversal=trav.value) if f.value else None

    def apply_stage(self, which, buf_in, nrhs, prec="f32", y=None, w=None, mass_idx=0, dagger=False, stencil=2,
                    rhs_tile=16, traversal=2, noalloc=False, out=None):
        """One fused stage of the solver's M_hat on internal parity-only fields (see
        laph_apply_stage): which 1 -> out_o = A_oo^-1 H_oe in; 2 -> out_e = y - 1/4
        A_ee^-1 H_eo in with <w, out>; 3 -> the same with <out, y>, |out|^2.
        noalloc: call laph_apply_stage_noalloc (the library's fixed device scratch, no
        workspace).  out: an output buffer to write (allocated when None).
        Returns (out buffer, dots numpy [nrhs][3] or None)."""
        if out is None:
            out = self._workspace(self.field_bytes(prec, nrhs, True))
        dots = np.zeros((nrhs, 3)) if which >= 2 else None
        nullp = ctypes.c_void_p(0)
        args = [self.ctx, int(which), _ptr(out), _ptr(buf_in), _ptr(y) if y is not None else nullp,
                _ptr(w) if w is not None else nullp, L.PREC[prec], int(nrhs), int(mass_idx), int(bool(dagger)),
                int(stencil), int(rhs_tile), int(traversal),
                dots.ctypes.data_as(ctypes.c_void_p) if dots is not None else nullp]
        if noalloc:
            L.check(self._run(self.lib.laph_apply_stage_noalloc, *args))
        else:
            ws = self._scratch(self.lib.laph_apply_stage_workspace_bytes(self.ctx, nrhs))
            L.check(self._run(self.lib.laph_apply_stage, *args, _ptr(ws), ws.numel()))
        return out, dots

    def mass_gradient(self, Z, X):
        """-sum_r Re<Z_r, X_r> over canonical spinor fields (the library's FP64 reduction)."""
        n = X.shape[0]
        _check_tensor(X, self.spinor_shape(n), "X")
        _check_tensor(Z, self.spinor_shape(n), "Z")
        w = self._workspace(self.lib.laph_mass_gradient_workspace_bytes(self.ctx))
        g = ctypes.c_double()
        L.check(self._run(self.lib.laph_mass_gradient, self.ctx, ctypes.byref(g), _ptr(Z), _ptr(X), n, _ptr(w),
                          w.numel()))
        return g.value

    # -- two-level aggregation multigrid ---------------------------------------------------
    def mg_params(self, **kw):
        p = L.MgParams()
        self.lib.laph_mg_default_params(ctypes.byref(p))
        for k, v in kw.items():
            if k == "block":
                for i in range(4):
                    p.block[i] = int(v[i])
                continue
            if not hasattr(p, k):
                raise TypeError("unknown multigrid parameter %r" % k)
            setattr(p, k, v)
        return p

    def mg_setup(self, V0, block, mass_idx=0, **kw):
        """Build the multigrid of mass mass_idx from the start vectors V0 (complex128
        [nvec][Lt][Lz][Ly][Lx][4][3] on the device); kw: the laph_mg_params fields."""
        nvec = V0.shape[0]
        _check_tensor(V0, (nvec,) + self.spinor_shape(1)[1:], "V0")
        p = self.mg_params(nvec=nvec, block=block, **kw)
        self._mg_state = None
        nbytes = self.lib.laph_mg_state_bytes(self.ctx, ctypes.byref(p))
        if nbytes == 0:
            # invalid shape: let the library report why (and detach any multigrid)
            L.check(self._run(self.lib.laph_mg_setup, self.ctx, int(mass_idx), ctypes.byref(p), _ptr(V0),
                              ctypes.c_void_p(0), 0, ctypes.c_void_p(0), 0))
        state = self._workspace(nbytes)
        ws = self._scratch(self.lib.laph_mg_setup_workspace_bytes(self.ctx, ctypes.byref(p)))
        L.check(self._run(self.lib.laph_mg_setup, self.ctx, int(mass_idx), ctypes.byref(p), _ptr(V0), _ptr(state),
                          state.numel(), _ptr(ws), ws.numel()))
        self._mg_state = state   # the library uses it until the next setup
        self._mg_params = p
        self._mg_block = tuple(int(b) for b in block)
        return p

    def mg_coarse_shape(self, n):
        xc, yc, zc, tc = (d // b for d, b in zip(self.dims, self._mg_block))
        return (n, tc, zc, yc, xc, 2, self._mg_params.nvec)

    def mg_basis(self):
        if getattr(self, "_mg_state", None) is None:
            L.check(self.lib.laph_mg_basis(self.ctx, ctypes.c_void_p(0)))
        out = torch.empty((self._mg_params.nvec,) + self.spinor_shape(1)[1:], dtype=torch.complex128,
                          device=self.device)
        L.check(self._run(self.lib.laph_mg_basis, self.ctx, _ptr(out)))
        return out

    def mg_coarse_matrix(self):
        xc, yc, zc, tc = (d // b for d, b in zip(self.dims, self._mg_block))
        m = 2 * self._mg_params.nvec
        out = torch.empty((xc * yc * zc * tc, 9, m, m), dtype=torch.complex128, device=self.device)
        L.check(self._run(self.lib.laph_mg_coarse_matrix, self.ctx, _ptr(out)))
        return out

    def mg_restrict(self, F):
        n = F.shape[0]
        _check_tensor(F, self.spinor_shape(n), "F")
        out = torch.empty(self.mg_coarse_shape(n), dtype=torch.complex128, device=self.device)
        ws = self._scratch(self.lib.laph_mg_field_workspace_bytes(self.ctx, n))
        L.check(self._run(self.lib.laph_mg_restrict, self.ctx, _ptr(out), _ptr(F), n, _ptr(ws), ws.numel()))
        return out

    def mg_prolong(self, c):
        n = c.shape[0]
        _check_tensor(c, self.mg_coarse_shape(n), "c")
        out = torch.empty(self.spinor_shape(n), dtype=torch.complex128, device=self.device)
        ws = self._scratch(self.lib.laph_mg_field_workspace_bytes(self.ctx, n))
        L.check(self._run(self.lib.laph_mg_prolong, self.ctx, _ptr(out), _ptr(c), n, _ptr(ws), ws.numel()))
        return out

    def mg_coarse_apply(self, c):
        n = c.shape[0]
        _check_tensor(c, self.mg_coarse_shape(n), "c")
        out = torch.empty_like(c)
        L.check(self._run(self.lib.laph_mg_coarse_apply, self.ctx, _ptr(out), _ptr(c), n))
        return out

    def _mg_run_params(self, kw):
        if not kw:
            return None
        p = L.MgParams()
        ctypes.memmove(ctypes.byref(p), ctypes.byref(self._mg_params), ctypes.sizeof(p))
        for k, v in kw.items():
            if k not in ("smooth_iters", "coarse_iters", "coarse_tol", "restart", "maxiter"):
                raise TypeError("not a cycle parameter: %r" % k)
            setattr(p, k, v)
        return p

    def mg_component(self, what, F, **kw):
        """One building block of the multigrid cycle (laph_mg_component): what 0 D in FP32,
        1 the smoother, 2 the cycle, 4 D in FP64 (spinor fields); 3 the coarse solve (coarse
        vectors); 5, 6 the GCR directions z, w after kw['maxiter'] iterations."""
        n = F.shape[0]
        _check_tensor(F, self.mg_coarse_shape(n) if what == 3 else self.spinor_shape(n), "F")
        p = self._mg_run_params(kw)
        pp = ctypes.byref(p) if p is not None else None
        if what in (5, 6):
            m = (p or self._mg_params).restart
            out = torch.empty((m,) + tuple(F.shape), dtype=torch.complex128, device=self.device)
        else:
            out = torch.empty_like(F)
        ws = self._scratch(self.lib.laph_mg_solve_workspace_bytes(self.ctx, n, pp))
        L.check(self._run(self.lib.laph_mg_component, self.ctx, int(what), _ptr(out), _ptr(F), n, pp, _ptr(ws),
                          ws.numel()))
        return out

    def mg_solve(self, B, tol=1e-10, allow_noconv=False, **kw):
        """X = D^-1 B by multigrid-preconditioned GCR (all RHS in one batch); kw: cycle
        parameters of this call (smooth_iters, coarse_iters, coarse_tol, restart, maxiter).
        Returns (X, per-RHS stats); raises LaphNoConvergence with the stats attached
        unless allow_noconv."""
        n = B.shape[0]
        _check_tensor(B, self.spinor_shape(n), "B")
        p = self._mg_run_params(kw)
        pp = ctypes.byref(p) if p is not None else None
        X = torch.empty_like(B)
        stats = (L.RhsStats * n)()
        ws = self._scratch(self.lib.laph_mg_solve_workspace_bytes(self.ctx, n, pp))
        st = self._run(self.lib.laph_mg_solve, self.ctx, _ptr(X), _ptr(B), n, float(tol), pp, stats, _ptr(ws),
                       ws.numel())
        lst = _stats_list(stats, n)
        if not (allow_noconv and st == L.LAPH_ERR_NOCONV):
            L.check(st, lst)
        return X, lst

    def stream_copy(self, dst, src, reps=5):
        """Average ms of the library's streaming copy of src into dst (device tensors)."""
        nbytes = src.numel() * src.element_size()
        if dst.numel() * dst.element_size() < nbytes:
            raise ValueError("dst smaller than src")
        ms = ctypes.c_double()
        L.check(self._run(self.lib.laph_stream_copy, self.ctx, _ptr(dst), _ptr(src), nbytes, int(reps),
                          ctypes.byref(ms)))
        return ms.value

    def apply_laplacian(self, X):
        """(-Delta) X on every timeslice; X: complex128 [Lt][nvec][Lz][Ly][Lx][3] on the device."""
        nvec = X.shape[1]
        _check_tensor(X, self.laph_shape(nvec), "X")
        out = torch.empty_like(X)
        L.check(self._run(self.lib.laph_apply_laplacian, self.ctx, _ptr(out), _ptr(X), nvec))
        return out

    def laplacian_eigvecs(self, nev, tol=1e-10, max_iter=200, degree=0):
        """Lowest nev eigenpairs of -Delta on every timeslice: (V [Lt][nev][Lz][Ly][Lx][3]
        on the device, eigenvalues [Lt][nev] (numpy), dict(iters, residual)).  degree: the
        Chebyshev filter degree per iteration (0: the library's default)."""
        lt = self.dims[3]
        V = torch.empty(self.laph_shape(nev), dtype=torch.complex128, device=self.device)
        lam = np.zeros((lt, nev))
        w = self._scratch(self.lib.laph_laplacian_workspace_bytes(self.ctx, nev))
        its, res = ctypes.c_int(0), ctypes.c_double(0)
        st = self._run(self.lib.laph_laplacian_eigvecs, self.ctx, _ptr(V),
                       lam.ctypes.data_as(ctypes.c_void_p), int(nev), float(tol), int(max_iter), int(degree),
                       _ptr(w), w.numel(), ctypes.byref(its), ctypes.byref(res))
        L.check(st)
        return V, lam, dict(iters=its.value, residual=res.value)

    def _contract(self, kind, fn, V, moms):
        nev = V.shape[1]
        _check_tensor(V, self.laph_shape(nev), "V")
        mom = np.ascontiguousarray(np.asarray(moms, dtype=np.int32).reshape(-1, 3))
        nm = mom.shape[0]
        shape = (nm, self.dims[3]) + (nev,) * (2 + kind)
        out = torch.empty(shape, dtype=torch.complex128, device=self.device)
        w = self._scratch(self.lib.laph_contract_workspace_bytes(self.ctx, kind, nev, nm))
        L.check(self._run(fn, self.ctx, _ptr(out), _ptr(V), nev, nm, mom.ctypes.data_as(ctypes.c_void_p),
                          _ptr(w), w.numel()))
        return out

    def meson_doublets(self, V, moms):
        """Phi[q][t][l][m] = sum_x exp(-i p_q.x) conj(V_l(x,t)) . V_m(x,t) for integer
        momenta moms[q] = (nx, ny, nz), p = 2 pi (nx/Lx, ny/Ly, nz/Lz); V [Lt][nev][Lz][Ly][Lx][3]."""
        return self._contract(0, self.lib.laph_meson_doublets, V, moms)

    def baryon_triplets(self, V, moms):
        """B[q][t][l][m][n] = sum_x exp(-i p_q.x) eps_abc V_l(x,t)_a V_m(x,t)_b V_n(x,t)_c."""
        return self._contract(1, self.lib.laph_baryon_triplets, V, moms)

    def stochastic_perambulator_raw(self, V, t0, rho, n_dil, mass_idx=0, tol=1e-10, params=None):
        """phi[t][l][j][beta][alpha] for the noise-diluted sources of rho [4][nev] (complex,
        on the device) at t0 with n_dil interlaced LapH groups (fused solve + projection)."""
        nev = V.shape[1]
        _check_tensor(V, self.laph_shape(nev), "V")
        _check_tensor(rho, (4, nev), "rho")
        p = params if params is not None else default_params()
        lt = self.dims[3]
        phi = torch.zeros((lt, nev, int(n_dil), 4, 4), dtype=torch.complex128, device=self.device)
        w = self._scratch(self.lib.laph_perambulator_workspace_bytes(self.ctx, nev, ctypes.byref(p)))
        stats = (L.RhsStats * (4 * int(n_dil)))()
        st = self._run(self.lib.laph_stochastic_perambulator, self.ctx, _ptr(phi), _ptr(V), nev, int(t0),
                       int(mass_idx), _ptr(rho), int(n_dil), float(tol), ctypes.byref(p), stats, _ptr(w), w.numel())
        sl = _stats_list(stats, 4 * int(n_dil))
        L.check(st, sl)
        return phi, sl

    def make_noise_sources(self, V, t0, rho, n_dil):
        nev = V.shape[1]
        _check_tensor(V, self.laph_shape(nev), "V")
        _check_tensor(rho, (4, nev), "rho")
        B = torch.empty(self.spinor_shape(4 * int(n_dil)), dtype=torch.complex128, device=self.device)
        L.check(self._run(self.lib.laph_make_noise_sources, self.ctx, _ptr(B), _ptr(V), nev, int(t0), _ptr(rho),
                          int(n_dil)))
        return B

    def spin_rotate(self, tau, S, out=None):
        """tau' = S tau S^dagger on the trailing (sink spin, source spin) 4 x 4 blocks of a
        perambulator-shaped tensor, for a change of Dirac basis psi' = S psi (S: 4 x 4
        unitary, numpy).  out=tau rotates in place."""
        if not isinstance(tau, torch.Tensor) or tau.dtype != torch.complex128 or not tau.is_cuda:
            raise TypeError("tau must be a complex128 CUDA tensor")
        if tuple(tau.shape[-2:]) != (4, 4) or not tau.is_contiguous():
            raise ValueError("tau must be contiguous with trailing 4 x 4 spin blocks")
        S = np.ascontiguousarray(np.asarray(S, dtype=np.complex128))
        if S.shape != (4, 4):
            raise ValueError("S must be 4 x 4")
        out = torch.empty_like(tau) if out is None else out
        if out.shape != tau.shape or out.dtype != tau.dtype or not out.is_contiguous():
            raise ValueError("out must match tau")
        L.check(self._run(self.lib.laph_spin_rotate, self.ctx, _ptr(out), _ptr(tau), tau.numel() // 16,
                          S.ctypes.data_as(ctypes.c_void_p)))
        return out

    def make_sources(self, V, t0):
        nev = V.shape[1]
        _check_tensor(V, self.laph_shape(nev), "V")
        B = torch.empty(self.spinor_shape(4 * nev), dtype=torch.complex128, device=self.device)
        L.check(self._run(self.lib.laph_make_sources, self.ctx, _ptr(B), _ptr(V), nev, int(t0)))
        return B

    def project_raw(self, X, V):
        nev = V.shape[1]
        _check_tensor(V, self.laph_shape(nev), "V")
        n = X.shape[0]
        if n % 4:
            raise ValueError("X must hold 4 * nev_src right-hand sides")
        _check_tensor(X, self.spinor_shape(n), "X")
        lt = self.dims[3]
        tau = torch.zeros((lt, nev, n // 4, 4, 4), dtype=torch.complex128, device=self.device)
        w = self._scratch(self.lib.laph_project_workspace_bytes(self.ctx, nev, n // 4))
        L.check(self._run(self.lib.laph_project, self.ctx, _ptr(tau), _ptr(X), _ptr(V), nev, n // 4, _ptr(w), w.numel()))
        return tau

    def project_adjoint_raw(self, G_tau, V):
        nev = V.shape[1]
        nsrc = G_tau.shape[2]
        G_tau = G_tau.contiguous()
        _check_tensor(G_tau, (self.dims[3], nev, nsrc, 4, 4), "G_tau")
        GX = torch.empty(self.spinor_shape(4 * nsrc), dtype=torch.complex128, device=self.device)
        L.check(self._run(self.lib.laph_project_adjoint, self.ctx, _ptr(GX), _ptr(G_tau), _ptr(V), nev, nsrc))
        return GX


# ---------------------------------------------------------------------------
# differentiable wrappers
# ---------------------------------------------------------------------------

class _SolveFn(torch.autograd.Function):
    """X = D(m0)^-1 B.  Backward: Z = D(m0)^-dagger G_X (the library's dagger solve,
    D^dagger = gamma5 D gamma5), grad_B = Z, grad_m0 = -sum Re<Z, X>."""

    @staticmethod
    def forward(ctx, lat, B, m0, tol, params_kw):
        m = float(m0.detach().cpu())
        lat.set_masses((m,), lat.csw if lat.csw is not None else 1.0)
        p = default_params(**params_kw)
        X, stats = lat.solve_raw(B.detach().contiguous(), 0, tol, p)
        ctx.lat, ctx.tol, ctx.kw, ctx.m = lat, tol, params_kw, m
        ctx.save_for_backward(X)
        ctx.stats = stats
        return X

    @staticmethod
    def backward(ctx, gX):
        (X,) = ctx.saved_tensors
        lat = ctx.lat
        lat.set_masses((ctx.m,), lat.csw if lat.csw is not None else 1.0)
        kw = dict(ctx.kw)
        kw["dagger"] = 1
        Z, _ = lat.solve_raw(gX.contiguous(), 0, ctx.tol, default_params(**kw))
        g_m0 = torch.tensor(lat.mass_gradient(Z, X), dtype=torch.float64)
        return None, Z, g_m0, None, None


class _ProjectFn(torch.autograd.Function):
    """tau = V^dagger X on every sink timeslice; backward G_X = V G_tau (V is a constant)."""

    @staticmethod
    def forward(ctx, lat, X, V):
        ctx.lat = lat
        ctx.save_for_backward(V)
        return lat.project_raw(X.detach().contiguous(), V)

    @staticmethod
    def backward(ctx, g_tau):
        (V,) = ctx.saved_tensors
        return None, ctx.lat.project_adjoint_raw(g_tau, V), None


def solve(lat, B, m0, tol=1e-10, csw=None, **params):
    """Differentiable X = D(m0)^-1 B (gradients for B and the scalar tensor m0)."""
    if csw is not None:
        lat.csw = csw
    if not isinstance(m0, torch.Tensor):
        m0 = torch.tensor(float(m0), dtype=torch.float64)
    return _SolveFn.apply(lat, B, m0, tol, params)


def project(lat, X, V):
    """Differentiable tau = V^dagger X (gradient for X)."""
    return _ProjectFn.apply(lat, X, V)


def perambulator(lat, V, t0, m0, tol=1e-10, csw=1.0, **params):
    """tau = V^dagger D(m0)^-1 V from spin-diluted sources at t0.

    Without autograd this is the library's fused call (solutions streamed in
    batches, never stored whole); when gradients are needed it is composed as
    sources -> solve -> projection, with the sources as a differentiable input."""
    lat.csw = csw
    need_grad = torch.is_grad_enabled() and isinstance(m0, torch.Tensor) and m0.requires_grad
    if not need_grad:
        lat.set_masses((float(m0),), csw)
        tau, stats = lat.perambulator_raw(V, t0, 0, tol, default_params(**params))
        return tau
    B = lat.make_sources(V, t0)
    X = solve(lat, B, m0, tol, **params)
    return project(lat, X, V)
