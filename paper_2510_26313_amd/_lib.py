"""ctypes declarations of liblaph.so (argument marshalling only).

The library is built in-tree by ``python -m paper_2510_26313_amd.build``.  If
it is missing this module raises: there is no fallback implementation.
"""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblaph.so")

c_int = ctypes.c_int
c_double = ctypes.c_double
c_size_t = ctypes.c_size_t
c_void_p = ctypes.c_void_p
P = ctypes.POINTER

LAPH_OK, LAPH_ERR_INVALID, LAPH_ERR_HIP, LAPH_ERR_WORKSPACE, LAPH_ERR_NOCONV, LAPH_ERR_BREAKDOWN, \
    LAPH_ERR_NONFINITE, LAPH_ERR_HOST = range(8)
LAPH_F64, LAPH_F32, LAPH_F16N = range(3)
PREC = {"f64": LAPH_F64, "f32": LAPH_F32, "f16n": LAPH_F16N}
RHS_STATUS = {0: "active", 1: "converged", 2: "noconv", 3: "breakdown", 4: "nonfinite"}
STATUS_NAMES = {0: "OK", 1: "INVALID", 2: "HIP", 3: "WORKSPACE", 4: "NOCONV", 5: "BREAKDOWN", 6: "NONFINITE",
                7: "HOST"}


class SolveParams(ctypes.Structure):
    _fields_ = [("inner_prec", c_int), ("batched", c_int), ("delta", c_double), ("maxiter", c_int),
                ("graph_iters", c_int), ("use_graph", c_int), ("dagger", c_int), ("use_x0", c_int),
                ("rhs_tile", c_int), ("chunk", c_int), ("stencil", c_int),
                ("traversal", c_int), ("stencil64", c_int), ("rhs_tile64", c_int)]


class RhsStats(ctypes.Structure):
    _fields_ = [("status", c_int), ("iters", c_int), ("updates", c_int), ("restarts", c_int),
                ("true_res", c_double)]


class MgParams(ctypes.Structure):
    _fields_ = [("nvec", c_int), ("block", c_int * 4), ("null_passes", c_int), ("null_tol", c_double),
                ("smooth_iters", c_int), ("coarse_iters", c_int), ("coarse_tol", c_double), ("restart", c_int),
                ("maxiter", c_int)]


# (name, restype, argtypes)
_SIGS = [
    ("laph_default_params", None, [P(SolveParams)]),
    ("laph_create", c_int, [P(c_void_p), P(c_int), c_int, c_int, c_void_p]),
    ("laph_destroy", c_int, [c_void_p]),
    ("laph_last_error", ctypes.c_char_p, []),
    ("laph_state_bytes", c_size_t, [c_void_p]),
    ("laph_attach_state", c_int, [c_void_p, c_void_p, c_size_t]),
    ("laph_load_gauge", c_int, [c_void_p, c_void_p]),
    ("laph_set_clover", c_int, [c_void_p, c_double, c_int, P(c_double)]),
    ("laph_field_bytes", c_size_t, [c_void_p, c_int, c_int, c_int]),
    ("laph_pack_spinor", c_int, [c_void_p, c_void_p, c_void_p, c_int, c_int, c_int]),
    ("laph_unpack_spinor", c_int, [c_void_p, c_void_p, c_void_p, c_int, c_int, c_int]),
    ("laph_apply_dslash", c_int, [c_void_p, c_void_p, c_void_p, c_int, c_int, c_int, c_int]),
    ("laph_apply_clover", c_int, [c_void_p, c_void_p, c_void_p, c_int, c_int, c_int, c_int, c_int]),
    ("laph_apply_D", c_int, [c_void_p, c_void_p, c_void_p, c_int, c_int, c_int, c_void_p, c_size_t]),
    ("laph_solve_workspace_bytes", c_size_t, [c_void_p, c_int, P(SolveParams)]),
    ("laph_solve", c_int, [c_void_p, c_void_p, c_void_p, c_int, P(c_int), c_double, P(SolveParams),
                           P(RhsStats), c_void_p, c_size_t]),
    ("laph_perambulator_workspace_bytes", c_size_t, [c_void_p, c_int, P(SolveParams)]),
    ("laph_perambulator", c_int, [c_void_p, c_void_p, c_void_p, c_int, c_int, c_int, c_double,
                                  P(SolveParams), P(RhsStats), c_void_p, c_size_t]),
    ("laph_make_sources", c_int, [c_void_p, c_void_p, c_void_p, c_int, c_int]),
    ("laph_stochastic_perambulator", c_int, [c_void_p, c_void_p, c_void_p, c_int, c_int, c_int, c_void_p, c_int,
                                             c_double, P(SolveParams), P(RhsStats), c_void_p, c_size_t]),
    ("laph_make_noise_sources", c_int, [c_void_p, c_void_p, c_void_p, c_int, c_int, c_void_p, c_int]),
    ("laph_laplacian_workspace_bytes", c_size_t, [c_void_p, c_int]),
    ("laph_apply_laplacian", c_int, [c_void_p, c_void_p, c_void_p, c_int]),
    ("laph_laplacian_eigvecs", c_int, [c_void_p, c_void_p, c_void_p, c_int, c_double, c_int, c_int, c_void_p,
                                       c_size_t, P(c_int), P(c_double)]),
    ("laph_contract_workspace_bytes", c_size_t, [c_void_p, c_int, c_int, c_int]),
    ("laph_meson_doublets", c_int, [c_void_p, c_void_p, c_void_p, c_int, c_int, c_void_p, c_void_p, c_size_t]),
    ("laph_baryon_triplets", c_int, [c_void_p, c_void_p, c_void_p, c_int, c_int, c_void_p, c_void_p, c_size_t]),
    ("laph_project_workspace_bytes", c_size_t, [c_void_p, c_int, c_int]),
    ("laph_project", c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_int, c_int, c_void_p, c_size_t]),
    ("laph_project_adjoint", c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_int, c_int]),
    ("laph_spin_rotate", c_int, [c_void_p, c_void_p, c_void_p, ctypes.c_long, c_void_p]),
    ("laph_last_timings", c_int, [c_void_p, P(c_double)]),
    ("laph_time_stages_workspace_bytes", c_size_t, [c_void_p, c_int, c_int, c_int]),
    ("laph_time_stages", c_int, [c_void_p, c_int, c_int, c_int, c_int, c_int, c_int, c_int, c_void_p, c_size_t,
                                 P(c_double)]),
    ("laph_autotune", c_int, [c_void_p, c_int, c_int, c_int, c_void_p, c_size_t, P(c_int), P(c_int), P(c_int),
                              P(c_double)]),
    ("laph_tuned_choice", c_int, [c_void_p, c_int, c_int, P(c_int), P(c_int), P(c_int), P(c_int)]),
    ("laph_apply_stage_workspace_bytes", c_size_t, [c_void_p, c_int]),
    ("laph_apply_stage", c_int, [c_void_p, c_int, c_void_p, c_void_p, c_void_p, c_void_p, c_int, c_int, c_int, c_int,
                                 c_int, c_int, c_int, c_void_p, c_void_p, c_size_t]),
    ("laph_apply_stage_noalloc", c_int, [c_void_p, c_int, c_void_p, c_void_p, c_void_p, c_void_p, c_int, c_int,
                                         c_int, c_int, c_int, c_int, c_int, c_void_p]),
    ("laph_mass_gradient_workspace_bytes", c_size_t, [c_void_p]),
    ("laph_mass_gradient", c_int, [c_void_p, P(c_double), c_void_p, c_void_p, c_int, c_void_p, c_size_t]),
    ("laph_stream_copy", c_int, [c_void_p, c_void_p, c_void_p, c_size_t, c_int, P(c_double)]),
    ("laph_mg_default_params", None, [P(MgParams)]),
    ("laph_mg_state_bytes", c_size_t, [c_void_p, P(MgParams)]),
    ("laph_mg_setup_workspace_bytes", c_size_t, [c_void_p, P(MgParams)]),
    ("laph_mg_setup", c_int, [c_void_p, c_int, P(MgParams), c_void_p, c_void_p, c_size_t, c_void_p, c_size_t]),
    ("laph_mg_basis", c_int, [c_void_p, c_void_p]),
    ("laph_mg_coarse_matrix", c_int, [c_void_p, c_void_p]),
    ("laph_mg_field_workspace_bytes", c_size_t, [c_void_p, c_int]),
    ("laph_mg_restrict", c_int, [c_void_p, c_void_p, c_void_p, c_int, c_void_p, c_size_t]),
    ("laph_mg_prolong", c_int, [c_void_p, c_void_p, c_void_p, c_int, c_void_p, c_size_t]),
    ("laph_mg_coarse_apply", c_int, [c_void_p, c_void_p, c_void_p, c_int]),
    ("laph_mg_component", c_int, [c_void_p, c_int, c_void_p, c_void_p, c_int, c_void_p, c_void_p, c_size_t]),
    ("laph_mg_solve_workspace_bytes", c_size_t, [c_void_p, c_int, c_void_p]),
    ("laph_mg_solve", c_int, [c_void_p, c_void_p, c_void_p, c_int, c_double, c_void_p, P(RhsStats), c_void_p,
                              c_size_t]),
]
EXPORTED = [s[0] for s in _SIGS]

_lib = None


def load(path=None):
    """Load liblaph.so and declare every entry point (raises if it is missing)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError("liblaph.so not built (%s); run `python -m paper_2510_26313_amd.build`" % p)
    lib = ctypes.CDLL(p)
    for name, res, args in _SIGS:
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    if path is None:
        _lib = lib
    return lib


class LaphError(RuntimeError):
    def __init__(self, status, message, stats=None):
        super().__init__("laph status %s: %s" % (STATUS_NAMES.get(status, status), message))
        self.status = status
        self.stats = stats


class LaphNoConvergence(LaphError):
    pass


def check(status, stats=None):
    if status == LAPH_OK:
        return
    msg = _lib.laph_last_error().decode() if _lib is not None else ""
    if status == LAPH_ERR_NOCONV:
        raise LaphNoConvergence(status, msg, stats)
    raise LaphError(status, msg, stats)
