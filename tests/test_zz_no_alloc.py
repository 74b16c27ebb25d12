"""laph_apply_stage_noalloc against laph_apply_stage.

The no-allocation entry point runs the same fused stages with the library's fixed
device scratch instead of a caller workspace.  Its outputs and inner products must
equal those of laph_apply_stage on the same inputs (same kernels, same launch
shape, fixed-order sums: bit for bit), on two calls in a row, the second with
fewer RHS than the first, so stale scratch contents from the first call cannot
leak into the second.  A request whose scratch need exceeds the fixed size fails
with LAPH_ERR_WORKSPACE before anything runs.
"""
import pytest
import torch

import laph_synth as ls
from gpu_common import dev, log_case, make_lattice, parity_mask, require_gpu

pytestmark = pytest.mark.gpu

DIMS = (6, 4, 4, 10)
BIG_DIMS = (16, 8, 8, 8)
SHAPES = [(2, 16, 2), (1, 2, 1)]


@pytest.fixture(scope="module")
def fields():
    require_gpu()
    U = ls.gauge_field(DIMS, 71)
    lat = make_lattice(DIMS, U, masses=(0.1, 0.05))
    par = parity_mask(DIMS)[..., None, None]
    sh = ls.spinor_shape(DIMS, 19)
    e_in = ls.random_spinor(sh, 7200) * (par == 0)
    o_in = ls.random_spinor(sh, 7201) * (par == 1)
    y = ls.random_spinor(sh, 7202) * (par == 0)
    w = ls.random_spinor(sh, 7203) * (par == 0)
    return lat, dict(e_in=e_in, o_in=o_in, y=y, w=w)


def _run(lat, which, prec, n, bufs, shape, noalloc):
    stencil, tile, trav = shape
    b_in = bufs["e"] if which == 1 else bufs["o"]
    # zero-filled, so the alignment padding the kernels never write compares equal too
    out = torch.zeros(lat.field_bytes(prec, n, True), dtype=torch.uint8, device="cuda")
    return lat.apply_stage(which, b_in, n, prec=prec, y=bufs["y"] if which >= 2 else None,
                           w=bufs["w"] if which == 2 else None, mass_idx=1, stencil=stencil, rhs_tile=tile,
                           traversal=trav, noalloc=noalloc, out=out)


@pytest.mark.parametrize("prec", ["f64", "f32", "f16n"])
def test_noalloc_matches_workspace_entry(fields, prec):
    lat, f = fields
    bufs = {"e": lat.pack(dev(f["e_in"]), prec, parity=0), "o": lat.pack(dev(f["o_in"]), prec, parity=1),
            "y": lat.pack(dev(f["y"]), prec, parity=0), "w": lat.pack(dev(f["w"]), prec, parity=0)}
    per_rhs = lat.field_bytes(prec, 1, True)
    for shape in SHAPES:
        for which in (1, 2, 3):
            for n in (19, 7):   # two calls in a row, the second smaller
                log_case("apply_stage_noalloc", prec=prec, which=which, nrhs=n, shape=shape)
                o_ref, d_ref = _run(lat, which, prec, n, bufs, shape, noalloc=False)
                o_new, d_new = _run(lat, which, prec, n, bufs, shape, noalloc=True)
                torch.cuda.synchronize()
                nb = n * per_rhs
                assert torch.equal(o_new[:nb], o_ref[:nb]), (prec, which, n, shape)
                if which >= 2:
                    assert (d_new == d_ref).all(), (prec, which, n, shape, abs(d_new - d_ref).max())


def test_noalloc_rejects_oversized_request():
    import paper_2510_26313_amd as pl
    require_gpu()
    U = ls.gauge_field(BIG_DIMS, 72)
    lat = make_lattice(BIG_DIMS, U, masses=(0.1,))
    b = lat.pack(dev(ls.random_spinor(ls.spinor_shape(BIG_DIMS, 1), 7204)), "f32", parity=0)
    out = torch.empty_like(b)
    # 30000 RHS at 16x8x8x8 need ~46 MB of partial sums: refused before any launch
    log_case("apply_stage_noalloc oversized", dims=BIG_DIMS, nrhs=30000)
    with pytest.raises(pl.LaphError) as ei:
        lat.apply_stage(1, b, 30000, prec="f32", stencil=2, rhs_tile=16, traversal=2, noalloc=True, out=out)
    assert ei.value.status == pl._lib.LAPH_ERR_WORKSPACE
    assert "device scratch" in str(ei.value)
