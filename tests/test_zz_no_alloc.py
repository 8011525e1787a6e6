"""pump_mlp_sample_noalloc (draws with no allocation on the call, host arrays
staged through the library's static per-GPU array) against pump_mlp_sample,
through the C ABI: equal draws on two calls in a row (the second smaller, so
stale staging contents from the first would show), in host and device
memory, and the capacity error past the staging limit."""

import numpy as np
import pytest

from oracle import proposal as pp
from paper_1607_06886_amd import _lib
from tests._gpu import print_case

pytestmark = pytest.mark.gpu


def _flat(params):
    return np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in params]).astype(np.float32)


def _draw_inputs(rng, q, n):
    cond = np.zeros((q, pp.D_IN), np.float32)
    cond[:, :12] = rng.uniform(0, 1, (q, 12))
    cond[:, 12:60] = rng.uniform(0, 1, (q, 48))
    u = rng.uniform(0, 1, (q, n)).astype(np.float32)
    eps = rng.standard_normal((q, n, 6)).astype(np.float32)
    return cond, u, eps


def test_noalloc_sampling_equals_sampling():
    import torch
    print_case("mlp_sample_noalloc")
    rng = np.random.default_rng(91)
    m = _lib.MLP(16)
    m.set_params(_flat(pp.init_params(5)))
    for q, n in ((16, 9000), (3, 700)):          # the second call is smaller
        cond, u, eps = _draw_inputs(rng, q, n)
        want = m.sample(cond, u, eps)
        got = m.sample_noalloc(cond, u, eps)
        assert got.shape == (q, n, 6)
        np.testing.assert_array_equal(got, want)
        assert np.isfinite(got).all() and np.abs(got).max() > 0
        t = lambda a: torch.from_numpy(a).cuda()
        got_d = m.sample_noalloc(t(cond), t(u), t(eps)).cpu().numpy()
        np.testing.assert_array_equal(got_d, want)
    # past the staging limit (2^21 floats, 13 per draw): a clear error
    cond, u, eps = _draw_inputs(rng, 16, 10_100)
    with pytest.raises(_lib.PumpError) as ei:
        m.sample_noalloc(cond, u, eps)
    assert ei.value.code == -2 and "no-alloc staging" in str(ei.value)
    m.close()
