"""The allocation-free Adam entry point (inrct_adam_noalloc, partials in a
static device array) against inrct_adam on the same inputs, through the C
ABI: two calls in a row, the second with fewer parameters, bitwise equal."""
import ctypes

import numpy as np
import pytest
import torch

from tests.gpu_util import dev, host, say

pytestmark = pytest.mark.gpu


def _p(t):
    return ctypes.c_void_p(t.data_ptr())


def test_adam_noalloc_matches_adam_on_two_calls():
    from paper_2604_09884_amd import configs
    from paper_2604_09884_amd import lib as L
    from paper_2604_09884_amd import ops
    lib = L.load()
    # parameter counts: the 501^3 FFN (193 partials) and then a smaller one
    for p_count, seed in ((394753, 1), (49665, 2)):
        arch = configs.C4.arch if p_count == 394753 else configs.C1.arch
        m = ops.Model(arch, arch.in_dim, 16, "fp32", max_k=1)
        assert m.n_params == p_count
        rng = np.random.default_rng(seed)
        th0, g0 = rng.standard_normal(p_count), rng.standard_normal(p_count)
        m0, v0 = rng.standard_normal(p_count) * 0.1, rng.random(p_count) * 0.01
        ref = [dev(x) for x in (th0, m0, v0)]
        new = [dev(x) for x in (th0, m0, v0)]
        g = dev(g0)
        gn_ref = torch.zeros(1, dtype=torch.float64, device="cuda")
        gn_new = torch.full((1,), -1.0, dtype=torch.float64, device="cuda")
        L.check(lib.inrct_adam(m.handle, *[_p(x) for x in ref], _p(g), 3, 1e-3, 0.9, 0.999,
                               1e-8, _p(gn_ref), None))
        L.check(lib.inrct_adam_noalloc(*[_p(x) for x in new], _p(g), p_count, 3, 1e-3, 0.9,
                                       0.999, 1e-8, _p(gn_new), None))
        torch.cuda.synchronize()
        for a, b in zip(ref, new):
            assert np.array_equal(host(a), host(b))
        assert host(gn_ref)[0] == host(gn_new)[0]
        say("adam noalloc p %d: theta, m, v and ||g||^2 bitwise equal (%.6g)"
            % (p_count, host(gn_new)[0]))
        m.close()
    # sizes outside the documented range are refused on the host
    x = dev(np.zeros(4))
    assert lib.inrct_adam_noalloc(_p(x), _p(x), _p(x), _p(x), 0, 1, 1e-3, 0.9, 0.999, 1e-8,
                                  None, None) == L.INRCT_EINVAL
    assert b"outside" in lib.inrct_last_error()
