"""Pins for the learned proposal's oracle: mixture density, gradients, Adam,
sampling."""

import numpy as np
import pytest
import scipy.special
import scipy.stats

from oracle import proposal as pp


def _small_batch(seed, B=5):
    rng = np.random.default_rng(seed)
    X = rng.uniform(0, 1, (B, pp.D_IN))
    Z = np.concatenate([rng.uniform(0, 1, (B, 3)), rng.uniform(-0.5, 0.5, (B, 3))], 1)
    return X, Z


def test_mixture_density_matches_scipy():
    rng = np.random.default_rng(1)
    y = rng.normal(0, 0.5, (3, pp.D_OUT))
    Z = rng.uniform(0, 1, (3, 6))
    logits, mu, ls = pp.split_heads(y)
    for b in range(3):
        logpi = logits[b] - scipy.special.logsumexp(logits[b])
        comp = [logpi[k] + scipy.stats.multivariate_normal.logpdf(
            Z[b], mu[b, k], np.diag(np.exp(2 * np.clip(ls[b, k], -4, 2)))) for k in range(16)]
        ref = -scipy.special.logsumexp(comp)
        assert abs(pp.nll(y[b:b + 1], Z[b:b + 1]) - ref) <= 1e-10 * max(1.0, abs(ref))


def test_single_isotropic_component_is_the_textbook_gaussian_nll():
    """All mass on one component with equal log-std s: NLL = 0.5 |z-mu|^2 e^{-2s}
    + 6 s + 3 log(2 pi)."""
    y = np.zeros((1, pp.D_OUT))
    y[0, :16] = -1e3
    y[0, 0] = 0.0
    mu = np.array([0.2, 0.4, 0.6, 0.1, -0.1, 0.0])
    y[0, 16:22] = mu
    s = -1.3
    y[0, 16 * 7:16 * 7 + 6] = s
    z = np.array([[0.25, 0.35, 0.5, 0.0, 0.0, 0.2]])
    ref = 0.5 * np.sum((z[0] - mu) ** 2) * np.exp(-2 * s) + 6 * s + 3 * np.log(2 * np.pi)
    assert abs(pp.nll(y, z) - ref) < 1e-12


def test_gradient_matches_central_differences():
    """Analytic backward vs FP64 central differences on every parameter kind
    (sampled entries), relative error < 1e-6."""
    params = pp.init_params(3)
    params = [(W.astype(np.float64) * 0.5, b.astype(np.float64) + 0.01) for W, b in params]
    X, Z = _small_batch(4)

    def loss(ps):
        y, _ = pp.forward(ps, X)
        return pp.nll(y, Z)

    y, cache = pp.forward(params, X)
    grads = pp.backward(params, cache, pp.nll_grad(y, Z))
    rng = np.random.default_rng(5)
    h = 1e-6
    checked = 0
    for l, (W, b) in enumerate(params):
        for arr_i, arr in enumerate((W, b)):
            g = grads[l][arr_i]
            for _ in range(6):
                idx = tuple(rng.integers(0, s) for s in arr.shape)
                orig = arr[idx]
                arr[idx] = orig + h
                lp = loss(params)
                arr[idx] = orig - h
                lm = loss(params)
                arr[idx] = orig
                fd = (lp - lm) / (2 * h)
                assert abs(fd - g[idx]) <= 1e-6 * max(1e-3, abs(fd)) + 1e-9, (l, arr_i, idx)
                checked += 1
    assert checked == 60


def test_output_gradient_matches_central_differences_including_clamp():
    rng = np.random.default_rng(6)
    y = rng.normal(0, 1.0, (4, pp.D_OUT))
    y[:, 16 * 7:] = rng.uniform(-9, 4, (4, 96))   # some log-std outside the clamp
    Z = rng.uniform(0, 1, (4, 6))
    g = pp.nll_grad(y, Z)
    h = 1e-6
    for _ in range(40):
        b, j = rng.integers(0, 4), rng.integers(0, pp.D_OUT)
        yp, ym = y.copy(), y.copy()
        yp[b, j] += h
        ym[b, j] -= h
        fd = (pp.nll(yp, Z) - pp.nll(ym, Z)) / (2 * h)
        assert abs(fd - g[b, j]) <= 1e-6 * max(1e-3, abs(fd)) + 1e-9


def test_adam_matches_the_published_update():
    """Kingma & Ba, Alg. 1, written out for a scalar over three steps."""
    p = [(np.array([[0.5]], np.float32), np.array([0.0], np.float32))]
    st = pp.adam_state(p)
    gs = [0.3, -0.1, 0.2]
    m = v = 0.0
    x = 0.5
    for t, g in enumerate(gs, start=1):
        p, st = pp.adam(p, [(np.array([[g]]), np.array([0.0]))], st, 0.01, t)
        m = 0.9 * m + 0.1 * g
        v = 0.999 * v + 0.001 * g * g
        x = x - 0.01 * (m / (1 - 0.9 ** t)) / (np.sqrt(v / (1 - 0.999 ** t)) + 1e-8)
        assert abs(float(p[0][0][0, 0]) - x) < 1e-7


def test_bf16_rounding_is_nearest_even():
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 1.0 + 2 ** -9, -2.5, 0.0, 1e-40],
                    np.float32)
    out = pp.bf16(vals)
    assert out[0] == 1.0
    assert out[1] == 1.0                     # tie -> even (mantissa ...0)
    assert out[2] == 1.0 + 4 * 2 ** -8       # tie -> even (rounds up)
    assert out[3] == 1.0
    assert out[4] == -2.5 and out[5] == 0.0


def test_sampling_moments():
    """Two-component mixture: sample frequencies and per-component means match."""
    y = np.zeros(pp.D_OUT)
    y[:16] = -50.0
    y[0], y[1] = np.log(0.3), np.log(0.7)
    y[16:22] = [0.2, 0.2, 0.2, 0.0, 0.0, 0.0]
    y[22:28] = [0.7, 0.6, 0.5, 0.1, 0.1, 0.1]
    y[16 * 7:] = np.log(0.02)
    rng = np.random.default_rng(7)
    n = 200_000
    z, k = pp.sample(y, rng.uniform(0, 1, n), rng.standard_normal((n, 6)))
    frac = (k == 0).mean()
    assert abs(frac - 0.3) < 4 * np.sqrt(0.21 / n)
    np.testing.assert_allclose(z[k == 1].mean(0), [0.7, 0.6, 0.5, 0.1, 0.1, 0.1], atol=1e-3)
    np.testing.assert_allclose(z[k == 1].std(0), 0.02, rtol=0.02)
    assert np.all(z >= pp.STATE_LO) and np.all(z <= pp.STATE_HI)


def test_condition_vector_layout():
    boxes = np.arange(70 * 6, dtype=np.float64).reshape(70, 6)
    v = pp.condition([1, 2, 3, 4, 5, 6], [0.8, 0.8, 0.8, 0.9, 1.0, 0.9], boxes)
    assert v.shape == (396,)
    np.testing.assert_allclose(v[:12], [1, 2, 3, 4, 5, 6, 0.85, 0.9, 0.85, 0.05, 0.1, 0.05])
    np.testing.assert_array_equal(v[12:], boxes[:64].reshape(-1))
