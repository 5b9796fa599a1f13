"""Device twin of the seeded input generator against the host generator,
including one launch over more than 2^32 elements (a dispatch's grid size
counts work-items in 32 bits, so the generator strides over a capped grid)."""
import numpy as np
import pytest
import torch

import synth
from gpu_util import say

pytestmark = pytest.mark.gpu


@pytest.mark.timeout(300)
def test_device_generator_beyond_32bit_grid():
    nocc, nvir, naux = 16, 4096, 65600          # 4.30e9 elements > 2^32
    assert nocc * nvir * naux > 2 ** 32
    k = synth.key(5, 0, 1)
    scale = synth.decay_scale(naux, 1200.0)
    say("device generator %d x %d x %d" % (nocc, nvir, naux))
    out = torch.full((nocc, nvir, naux), float("nan"), dtype=torch.float64, device="cuda:0")
    synth.three_index_device(k, nocc, nvir, naux, scale, out)
    torch.cuda.synchronize()
    assert not bool(torch.isnan(out).any())
    for i in (0, nocc - 1):
        host = synth.three_index(k, nocc, nvir, naux, scale, i, i + 1)[0]
        got = out[i].cpu().numpy()
        np.testing.assert_allclose(got, host, rtol=1e-13, atol=1e-14)
    del out
    torch.cuda.empty_cache()
