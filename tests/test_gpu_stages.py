"""Single-application parity of the solver's fused stencil stages.

laph_apply_stage runs exactly the kernels (and launch shapes) the batched solver
uses inside its iterations: stage 1 A_oo^-1 H_oe p, stage 2 p - 1/4 A_ee^-1 H_eo t
with the fused <r^, v>, and the t-variant with <t, s> and |t|^2.  Inside a solve
the FP64 reliable updates would correct an error of these kernels, so they are
pinned here one application at a time against the oracle's hop and clover
inverse, per RHS, for every stencil form, RHS tile, traversal and dagger, on a
ragged lattice (site blocks cut mid-row, no 4-D block tiles) and on one whose
64-site blocks are whole rows taken in 4-D tiles; nrhs = 19 leaves a partly
filled last tile.
"""
import numpy as np
import pytest

import laph_synth as ls
from gpu_common import dev, host, log_case, make_lattice, parity_mask, per_rhs_rel, require_gpu
from oracle import dirac

pytestmark = pytest.mark.gpu

DIMS_RAGGED = (6, 4, 4, 10)
DIMS_TILED = (16, 8, 4, 4)
NRHS = 19
M0 = 0.05
SHAPES = [(2, 4, 1), (2, 8, 2), (2, 16, 1), (2, 16, 2), (1, 1, 2), (1, 2, 1), (1, 4, 2)]
TOL = {"f64": 1e-13, "f32": 1e-6, "f16n": 3e-3}


@pytest.fixture(scope="module", params=[DIMS_RAGGED, DIMS_TILED], ids=["ragged", "tiled"])
def case(request):
    require_gpu()
    dims = request.param
    U = ls.gauge_field(dims, 61)
    lat = make_lattice(dims, U, masses=(0.1, M0))
    par = parity_mask(dims)[..., None, None]
    Ai = dirac.clover_inverse(dirac.clover_matrix(U, M0, 1.0))
    sh = ls.spinor_shape(dims, NRHS)
    inp = ls.random_spinor(sh, 7100)
    y = 0.3 * ls.random_spinor(sh, 7101) * (par == 0)
    noise = ls.random_spinor(sh, 7102) * (par == 0)
    out = {}
    for dag in (False, True):
        # stage 1: odd output from the even part of inp
        e_in = inp * (par == 0)
        s1 = dirac.apply_site_matrix(Ai, dirac.hop(U, e_in, True, dag)) * (par == 1)
        # stage 2: even output from the odd part of inp
        o_in = inp * (par == 1)
        s2 = (y - 0.25 * dirac.apply_site_matrix(Ai, dirac.hop(U, o_in, True, dag))) * (par == 0)
        # w correlated with the output, so <w, out> is of the size of |w| |out|
        w = s2 + 0.3 * noise
        out[dag] = dict(e_in=e_in, o_in=o_in, s1=s1, s2=s2, w=w)
    return dict(dims=dims, lat=lat, y=y, par=par, ref=out)


def _dot(a, b):
    n = a.shape[0]
    return np.einsum("ij,ij->i", np.conj(a.reshape(n, -1)), b.reshape(n, -1))


@pytest.mark.parametrize("dagger", [False, True])
@pytest.mark.parametrize("prec", ["f64", "f32", "f16n"])
def test_fused_stages_vs_oracle(case, prec, dagger):
    lat, dims, ref = case["lat"], case["dims"], case["ref"][dagger]
    tol = TOL[prec]
    b_e = lat.pack(dev(ref["e_in"]), prec, parity=0)
    b_o = lat.pack(dev(ref["o_in"]), prec, parity=1)
    b_y = lat.pack(dev(case["y"]), prec, parity=0)
    b_w = lat.pack(dev(ref["w"]), prec, parity=0)
    s2 = ref["s2"]
    nw, no, ny = (np.linalg.norm(a.reshape(NRHS, -1), axis=1) for a in (ref["w"], s2, case["y"]))
    for stencil, tile, trav in SHAPES:
        kw = dict(prec=prec, mass_idx=1, dagger=dagger, stencil=stencil, rhs_tile=tile, traversal=trav)
        log_case("apply_stage 1", dims=dims, **kw)
        o1, _ = lat.apply_stage(1, b_e, NRHS, **kw)
        e1 = per_rhs_rel(host(lat.unpack(o1, NRHS, prec, parity=1)), ref["s1"])
        assert e1.max() < tol, (stencil, tile, trav, e1.max())
        log_case("apply_stage 2", dims=dims, **kw)
        o2, d2 = lat.apply_stage(2, b_o, NRHS, y=b_y, w=b_w, **kw)
        got2 = host(lat.unpack(o2, NRHS, prec, parity=0))
        e2 = per_rhs_rel(got2, s2)
        assert e2.max() < tol, (stencil, tile, trav, e2.max())
        exp_d = _dot(ref["w"], s2)
        err = np.abs(d2[:, 0] + 1j * d2[:, 1] - exp_d)
        assert np.all(err <= tol * nw * no), (stencil, tile, trav, (err / (nw * no)).max())
        assert np.all(d2[:, 2] == 0)
        log_case("apply_stage 3", dims=dims, **kw)
        o3, d3 = lat.apply_stage(3, b_o, NRHS, y=b_y, **kw)
        got3 = host(lat.unpack(o3, NRHS, prec, parity=0))
        assert per_rhs_rel(got3, s2).max() < tol
        exp_ty = _dot(s2, case["y"])
        err = np.abs(d3[:, 0] + 1j * d3[:, 1] - exp_ty)
        assert np.all(err <= tol * no * ny), (stencil, tile, trav, (err / (no * ny)).max())
        exp_tt = np.linalg.norm(s2.reshape(NRHS, -1), axis=1) ** 2
        assert np.all(np.abs(d3[:, 2] - exp_tt) <= 2 * tol * exp_tt), (stencil, tile, trav)
        if prec != "f16n":
            # the reduction sums exactly what the kernel stored (up to FP32 / FP64 rounding)
            own = _dot(host(lat.unpack(b_w, NRHS, prec, parity=0)), got2)
            assert np.all(np.abs(d2[:, 0] + 1j * d2[:, 1] - own) <= tol * nw * no)


def test_stage_argument_checks(case):
    import paper_2510_26313_amd as pl
    lat = case["lat"]
    b = lat.pack(dev(case["ref"][False]["e_in"]), "f32", parity=0)
    log_case("apply_stage arguments")
    with pytest.raises(pl.LaphError):
        lat.apply_stage(1, b, NRHS, prec="f32", stencil=2, rhs_tile=2)      # LDS tiles are 4, 8, 16
    with pytest.raises(pl.LaphError):
        lat.apply_stage(2, b, NRHS, prec="f32", y=b, w=None)                # stage 2 needs w
    with pytest.raises(pl.LaphError):
        lat.apply_stage(1, b, NRHS, prec="f32", mass_idx=5)
