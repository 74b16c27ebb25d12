"""The library's streaming copy (the measured HBM ceiling the bench reports its
bandwidth fractions against) copies exactly: sizes of one 16-byte word, a partly
filled last workgroup, and several MiB; bytes past the copied range stay untouched."""
import numpy as np
import pytest
import torch

import laph_synth as ls
from gpu_common import log_case, make_lattice, require_gpu

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("nbytes", [16, 4096 + 16, 3 * 2**20 + 48])
def test_stream_copy_is_exact(nbytes):
    require_gpu()
    dims = (4, 4, 4, 4)
    lat = make_lattice(dims, ls.unit_gauge(dims))
    rng = np.random.default_rng(nbytes)
    src = torch.from_numpy(rng.integers(0, 256, nbytes, dtype=np.uint8)).cuda()
    dst = torch.full((nbytes + 64,), 0xA5, dtype=torch.uint8, device="cuda")
    log_case("stream_copy", nbytes=nbytes)
    ms = lat.stream_copy(dst, src, reps=2)
    assert ms > 0
    torch.cuda.synchronize()
    assert torch.equal(dst[:nbytes], src)
    assert bool((dst[nbytes:] == 0xA5).all())
