"""Learned sampling proposal (oracle, FP64): a small MLP emitting a Gaussian
mixture over the 6-D state, its negative log-likelihood, gradients, Adam and
mixture sampling.

The paper samples SampleFree(n) uniformly (Alg. 3; Halton in Sec. V-A).  The
learned proposal only changes that sample set: half of the samples come from
the mixture, half stay uniform, and every plan is still certified by MC(p)
(Alg. 5), so the CP guarantee is untouched.

Network: condition vector (start 6, goal centre 3, goal half-size 3, 64
zero-padded boxes x (lo, hi) = 396) -> 4 hidden layers of 256 with ReLU ->
16 x (1 logit + 6 means + 6 log-std) = 208; log-std clamped to [-4, 2].
Reading: weights are stored in BF16 and every matrix product takes BF16
operands with FP32 accumulation; `bf16=True` rounds weights and layer inputs
to BF16 (round to nearest even) exactly where the device does.
"""

from __future__ import annotations

import numpy as np

K_COMP = 16
D_STATE = 6
MAX_BOXES = 64
D_IN = 12 + 6 * MAX_BOXES          # 396
HIDDEN = 256
N_HIDDEN = 4
D_OUT = K_COMP * (1 + 2 * D_STATE)  # 208
LOGSTD_MIN, LOGSTD_MAX = -4.0, 2.0
LAYERS = [(D_IN, HIDDEN)] + [(HIDDEN, HIDDEN)] * (N_HIDDEN - 1) + [(HIDDEN, D_OUT)]
# state box the samples live in (positions in the unit cube, velocities)
STATE_LO = np.array([0.0, 0.0, 0.0, -0.5, -0.5, -0.5])
STATE_HI = np.array([1.0, 1.0, 1.0, 0.5, 0.5, 0.5])


def condition(x_init, goal, boxes):
    """Condition vector of one query (396 values)."""
    v = np.zeros(D_IN)
    v[:6] = np.asarray(x_init, np.float64)[:6]
    g = np.asarray(goal, np.float64)
    v[6:9] = 0.5 * (g[:3] + g[3:])
    v[9:12] = 0.5 * (g[3:] - g[:3])
    b = np.asarray(boxes, np.float64).reshape(-1, 6)[:MAX_BOXES]
    v[12:12 + 6 * b.shape[0]] = b.reshape(-1)
    return v


def bf16(x):
    """Round to the nearest BF16 value (ties to even), returned as float64."""
    a = np.asarray(x, np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    return np.where(np.isnan(a), np.nan, out)


def init_params(seed):
    """He-uniform weights, zero biases (FP32 master values)."""
    rng = np.random.default_rng(seed)
    params = []
    for fi, fo in LAYERS:
        lim = np.sqrt(6.0 / fi)
        params.append((rng.uniform(-lim, lim, (fo, fi)).astype(np.float32),
                       np.zeros(fo, np.float32)))
    return params


def forward(params, X, bf16_ops=False):
    """Outputs [B, 208] and the per-layer cache (inputs, pre-activations)."""
    h = np.asarray(X, np.float64)
    cache = []
    for l, (W, b) in enumerate(params):
        Wd = bf16(W) if bf16_ops else np.asarray(W, np.float64)
        hin = bf16(h) if bf16_ops else h
        z = hin @ Wd.T + np.asarray(b, np.float64)
        cache.append((hin, Wd, z))
        h = np.maximum(z, 0.0) if l < len(params) - 1 else z
    return h, cache


def split_heads(y):
    """logits [B,16], means [B,16,6], raw log-std [B,16,6]."""
    B = y.shape[0]
    logits = y[:, :K_COMP]
    mu = y[:, K_COMP:K_COMP * 7].reshape(B, K_COMP, D_STATE)
    ls = y[:, K_COMP * 7:].reshape(B, K_COMP, D_STATE)
    return logits, mu, ls


def _logsumexp(a, axis):
    m = np.max(a, axis=axis, keepdims=True)
    return (m + np.log(np.sum(np.exp(a - m), axis=axis, keepdims=True))).squeeze(axis)


def component_logpdf(y, Z):
    """log pi_k + log N(z; mu_k, diag(sigma_k^2)) for each sample and k."""
    logits, mu, ls = split_heads(y)
    s = np.clip(ls, LOGSTD_MIN, LOGSTD_MAX)
    logpi = logits - _logsumexp(logits, 1)[:, None]
    r = (np.asarray(Z, np.float64)[:, None, :] - mu) * np.exp(-s)
    lp = -0.5 * np.sum(r * r, -1) - np.sum(s, -1) - 0.5 * D_STATE * np.log(2 * np.pi)
    return logpi + lp


def nll(y, Z):
    """Mean negative log-likelihood of targets Z [B, 6] under the mixtures."""
    return float(-np.mean(_logsumexp(component_logpdf(y, Z), 1)))


def nll_grad(y, Z):
    """d(mean NLL)/dy [B, 208] (the clamp passes no gradient outside its range)."""
    B = y.shape[0]
    logits, mu, ls = split_heads(y)
    s = np.clip(ls, LOGSTD_MIN, LOGSTD_MAX)
    a = component_logpdf(y, Z)
    w = np.exp(a - _logsumexp(a, 1)[:, None])              # responsibilities
    pi = np.exp(logits - _logsumexp(logits, 1)[:, None])
    inv = np.exp(-s)
    r = (np.asarray(Z, np.float64)[:, None, :] - mu) * inv
    g_logit = pi - w
    g_mu = -w[..., None] * r * inv
    g_s = w[..., None] * (1.0 - r * r)
    inside = (ls > LOGSTD_MIN) & (ls < LOGSTD_MAX)
    g_s = np.where(inside, g_s, 0.0)
    g = np.concatenate([g_logit, g_mu.reshape(B, -1), g_s.reshape(B, -1)], axis=1)
    return g / B


def backward(params, cache, gy, bf16_ops=False):
    """Parameter gradients [(dW, db)] for output gradient gy.  With bf16_ops
    the back-propagated gradient is rounded to BF16 where it enters a matrix
    product (bias gradients use the unrounded values)."""
    grads = [None] * len(params)
    g = np.asarray(gy, np.float64)
    for l in range(len(params) - 1, -1, -1):
        hin, Wd, z = cache[l]
        if l < len(params) - 1:
            g = g * (z > 0)
        gm = bf16(g) if bf16_ops else g
        grads[l] = (gm.T @ hin, g.sum(0))
        g = gm @ Wd
    return grads


def adam(params, grads, state, lr, t, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (Kingma & Ba) on FP32 master weights; returns the new
    params and state.  t counts from 1."""
    out, new_state = [], []
    for (W, b), (dW, db), st in zip(params, grads, state):
        upd = []
        nst = []
        for p, g, (m, v) in zip((W, b), (dW, db), st):
            m = b1 * m + (1 - b1) * g
            v = b2 * v + (1 - b2) * g * g
            mh = m / (1 - b1 ** t)
            vh = v / (1 - b2 ** t)
            upd.append((np.asarray(p, np.float64) - lr * mh / (np.sqrt(vh) + eps)).astype(np.float32))
            nst.append((m, v))
        out.append(tuple(upd))
        new_state.append(tuple(nst))
    return out, new_state


def adam_state(params):
    return [tuple((np.zeros(p.shape), np.zeros(p.shape)) for p in layer) for layer in params]


def sample(y, u, eps):
    """Draws from the mixture of one query: y [208] (outputs), u [n] uniforms
    choose components by inverse CDF of softmax(logits); eps [n, 6] standard
    normals give mu + sigma * eps; results are clamped to the state box."""
    logits, mu, ls = split_heads(np.asarray(y, np.float64)[None])
    logits, mu, ls = logits[0], mu[0], np.clip(ls[0], LOGSTD_MIN, LOGSTD_MAX)
    p = np.exp(logits - _logsumexp(logits, 0))
    cdf = np.cumsum(p)
    k = np.minimum(np.searchsorted(cdf, np.asarray(u, np.float64) * cdf[-1], side="right"),
                   K_COMP - 1)
    z = mu[k] + np.exp(ls[k]) * np.asarray(eps, np.float64)
    return np.clip(z, STATE_LO, STATE_HI), k
