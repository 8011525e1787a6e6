"""GPU parity of the learned proposal's kernels (BF16 MFMA forward/backward,
mixture NLL, Adam, sampling, condition vectors) with the FP64 oracle, which
rounds weights, layer inputs and back-propagated gradients to BF16 where the
device does.  Tolerances follow from the BF16 unit roundoff (2^-8) and the
fan-in: outputs within 2% of their range (mean error 0.4%); gradients element
by element within 2^-8 of each layer's largest gradient (one BF16 rounding
step of a back-propagated value taken differently where the FP32 and FP64
sums straddle a rounding boundary; measured at most 0.07%), their mean
error within 2^-10 of the layer's mean magnitude."""

import numpy as np
import pytest

from oracle import proposal as pp
from paper_1607_06886_amd import _lib
from tests._gpu import print_case

pytestmark = pytest.mark.gpu


def flat(params):
    return np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in params]).astype(np.float32)


def unflat(f):
    out, o = [], 0
    for fi, fo in pp.LAYERS:
        W = f[o:o + fi * fo].reshape(fo, fi)
        o += fi * fo
        b = f[o:o + fo]
        o += fo
        out.append((W.astype(np.float64), b.astype(np.float64)))
    return out


def _inputs(seed, B):
    rng = np.random.default_rng(seed)
    X = np.zeros((B, pp.D_IN), np.float32)
    X[:, :12] = rng.uniform(0, 1, (B, 12))
    nb = rng.integers(5, 64, B)
    for i in range(B):
        X[i, 12:12 + 6 * nb[i]] = rng.uniform(0, 1, 6 * nb[i])
    Z = np.concatenate([rng.uniform(0, 1, (B, 3)), rng.uniform(-0.5, 0.5, (B, 3))], 1).astype(np.float32)
    return X, Z


def test_param_count():
    assert _lib.load().pump_mlp_num_params() == sum(fi * fo + fo for fi, fo in pp.LAYERS) == 352464


@pytest.mark.parametrize("B", [1, 37, 256])
def test_forward_matches_oracle(B):
    print_case("mlp_forward", B=B)
    params = pp.init_params(11)
    params = [(W, (np.random.default_rng(12).normal(0, 0.1, b.shape)).astype(np.float32)) for W, b in params]
    X, _ = _inputs(13, B)
    m = _lib.MLP(512)
    m.set_params(flat(params))
    y = m.forward(X).astype(np.float64)
    ref, _ = pp.forward(params, X, bf16_ops=True)
    scale = np.abs(ref).max()
    err = np.abs(y - ref)
    assert err.max() <= 0.02 * scale, (err.max(), scale)
    assert err.mean() <= 0.004 * np.abs(ref).mean()
    m.close()


def test_gradients_match_oracle():
    print_case("mlp_grad")
    params = pp.init_params(21)
    X, Z = _inputs(22, 96)
    m = _lib.MLP(128)
    m.set_params(flat(params))
    loss, g = m.loss_grad(X, Z)
    y, cache = pp.forward(params, X, bf16_ops=True)
    lref = pp.nll(y, Z)
    gref = flat([(dW, db) for dW, db in pp.backward(params, cache, pp.nll_grad(y, Z), bf16_ops=True)])
    assert abs(loss - lref) <= 1e-2 * abs(lref) + 1e-3
    g64, r64 = g.astype(np.float64), gref.astype(np.float64)
    cos = g64 @ r64 / (np.linalg.norm(g64) * np.linalg.norm(r64))
    assert cos > 0.999, cos
    assert abs(np.linalg.norm(g64) / np.linalg.norm(r64) - 1) < 0.02
    # per layer, element by element
    o = 0
    for li, (fi, fo) in enumerate(pp.LAYERS):
        n = fi * fo + fo
        a, b = g64[o:o + n], r64[o:o + n]
        assert a @ b / (np.linalg.norm(a) * np.linalg.norm(b) + 1e-30) > 0.995
        err = np.abs(a - b)
        print(f"  layer {li}: max error / max |grad| {err.max() / np.abs(b).max():.2e}, "
              f"mean error / mean |grad| {err.mean() / np.abs(b).mean():.2e}", flush=True)
        assert err.max() <= 2.0 ** -8 * np.abs(b).max(), li
        assert err.mean() <= 2.0 ** -10 * np.abs(b).mean(), li
        o += n
    m.close()


def test_adam_step_matches_oracle():
    print_case("mlp_adam")
    params = pp.init_params(31)
    X, Z = _inputs(32, 64)
    m = _lib.MLP(64)
    m.set_params(flat(params))
    lr = 1e-3
    m.train_step(X, Z, lr)
    got = m.get_params().astype(np.float64)
    y, cache = pp.forward(params, X, bf16_ops=True)
    grads = pp.backward(params, cache, pp.nll_grad(y, Z), bf16_ops=True)
    new, _ = pp.adam(params, grads, pp.adam_state(params), lr, 1)
    want = flat(new).astype(np.float64)
    p0 = flat(params).astype(np.float64)
    step_gpu, step_ref = got - p0, want - p0
    # first Adam step moves each weight by about lr * sign(g)
    assert np.abs(step_gpu).max() <= 1.01 * lr
    agree = np.mean(np.sign(step_gpu) == np.sign(step_ref))
    assert agree > 0.98, agree
    m.close()


def test_sampling_matches_oracle():
    """All weights zero: the outputs equal the last bias exactly, so both sides
    sample the same mixture from the same uniforms and normals."""
    print_case("mlp_sample")
    rng = np.random.default_rng(41)
    params = [(np.zeros((fo, fi), np.float32), np.zeros(fo, np.float32)) for fi, fo in pp.LAYERS]
    yb = np.zeros(pp.D_OUT, np.float32)
    yb[:16] = rng.normal(0, 1.0, 16)
    yb[16:112] = np.concatenate([rng.uniform(0, 1, (16, 3)), rng.uniform(-0.5, 0.5, (16, 3))], 1).ravel()
    yb[112:] = rng.uniform(-4, -1, 96)
    params[-1] = (params[-1][0], yb)
    m = _lib.MLP(8)
    m.set_params(flat(params))
    q, n = 3, 2000
    cond = rng.uniform(0, 1, (q, pp.D_IN)).astype(np.float32)
    u = rng.uniform(0, 1, (q, n)).astype(np.float32)
    eps = rng.standard_normal((q, n, 6)).astype(np.float32)
    out = m.sample(cond, u, eps)
    for i in range(q):
        z, k = pp.sample(yb.astype(np.float64), u[i].astype(np.float64), eps[i].astype(np.float64))
        np.testing.assert_allclose(out[i], z, rtol=0, atol=2e-6)
    m.close()


def test_condition_vectors():
    import torch
    print_case("mlp_condition")
    rng = np.random.default_rng(51)
    q, maxb = 4, 70
    x0 = rng.uniform(0, 1, (q, 6)).astype(np.float32)
    goal = np.sort(rng.uniform(0, 1, (q, 2, 3)), axis=1).reshape(q, 6).astype(np.float32)
    boxes = rng.uniform(0, 1, (q, maxb, 6)).astype(np.float32)
    nobs = np.array([3, 64, 70, 0], np.int32)
    m = _lib.MLP(8)
    t = lambda a: torch.from_numpy(a).cuda()
    got = m.condition(t(x0), t(goal), t(boxes), t(nobs)).cpu().numpy()
    for i in range(q):
        ref = pp.condition(x0[i], goal[i], boxes[i, :nobs[i]])
        np.testing.assert_allclose(got[i], ref, rtol=1e-6, atol=1e-7)
    m.close()


def test_training_reduces_the_loss():
    """Targets depend on the condition (a shifted copy of the start state):
    200 Adam steps on the device lower the mean NLL well below its start."""
    print_case("mlp_train")
    rng = np.random.default_rng(61)
    B = 256
    m = _lib.MLP(B)
    m.set_params(flat(pp.init_params(62)))
    first = last = None
    for step in range(200):
        X, _ = _inputs(1000 + step, B)
        Z = np.clip(X[:, :6] + 0.05 + 0.01 * rng.standard_normal((B, 6)), -0.5, 1.0).astype(np.float32)
        loss = m.train_step(X, Z, 1e-3)
        first = loss if first is None else first
        last = loss
    assert np.isfinite(last) and last < first - 5.0, (first, last)
    m.close()


def test_adam_matches_oracle_elementwise():
    """Two Adam steps on given gradient vectors (the same FP32 values on both
    sides): parameters and both moment estimates equal the FP64 oracle's
    element by element, to FP32 rounding."""
    print_case("mlp_adam_elementwise")
    rng = np.random.default_rng(57)
    params = pp.init_params(33)
    m = _lib.MLP(8)
    m.set_params(flat(params))
    n = m.n_params
    grads = [rng.standard_normal(n).astype(np.float32) * np.float32(s) for s in (1e-2, 3e-3)]
    lr = 1e-3
    ref_p = [(W.astype(np.float64), b.astype(np.float64)) for W, b in params]
    state = pp.adam_state(params)
    for t, g in enumerate(grads, start=1):
        m.adam_step(g, lr)
        ref_p, state = pp.adam(ref_p, unflat(g), state, lr, t)
        ref_p = [(W.astype(np.float64), b.astype(np.float64)) for W, b in ref_p]
    st = m.get_state()
    assert st["t"] == 2
    want_p = flat(ref_p).astype(np.float64)
    want_m1 = np.concatenate([np.concatenate([a[0].ravel(), b[0].ravel()]) for a, b in state])
    want_m2 = np.concatenate([np.concatenate([a[1].ravel(), b[1].ravel()]) for a, b in state])
    p0 = flat(params).astype(np.float64)
    step = np.abs(want_p - p0)
    ulp = np.spacing(np.abs(want_p).astype(np.float32)).astype(np.float64)
    err = np.abs(st["params"].astype(np.float64) - want_p)
    assert (err <= 2 * ulp + 1e-5 * step).all(), float((err / (2 * ulp + 1e-5 * step)).max())
    # m1 = 0.9 m1' + 0.1 g can cancel: its FP32 error is relative to the two
    # terms' magnitudes, not to the result
    g1, g2 = grads[0].astype(np.float64), grads[1].astype(np.float64)
    scale1 = 0.9 * np.abs(0.1 * g1) + 0.1 * np.abs(g2)
    assert (np.abs(st["m1"] - want_m1) <= 2e-6 * scale1 + 1e-30).all()
    np.testing.assert_allclose(st["m2"], want_m2, rtol=2e-6, atol=1e-16)
    m.close()


def test_checkpoint_resume_continues_training(tmp_path):
    """Training state saved after some steps and loaded into a fresh network
    continues as the uninterrupted run: the same parameters, moments and step
    count after the same further steps."""
    print_case("mlp_checkpoint")
    X, Z = _inputs(61, 128)
    a = _lib.MLP(128)
    a.set_params(flat(pp.init_params(35)))
    for _ in range(4):
        a.train_step(X[:64], Z[:64], 1e-3)
    path = str(tmp_path / "mlp_state.npz")
    a.save(path)
    b = _lib.MLP(128)
    b.set_params(flat(pp.init_params(99)))      # overwritten by load
    b.load(path)
    sa, sb = a.get_state(), b.get_state()
    for k in ("params", "m1", "m2"):
        np.testing.assert_array_equal(sa[k], sb[k])
    assert sa["t"] == sb["t"] == 4 and np.abs(sa["m2"]).max() > 0
    for _ in range(3):
        la = a.train_step(X[64:], Z[64:], 1e-3)
        lb = b.train_step(X[64:], Z[64:], 1e-3)
        assert abs(la - lb) <= 1e-5 * max(1.0, abs(la))
    sa, sb = a.get_state(), b.get_state()
    assert sa["t"] == sb["t"] == 7
    for k in ("params", "m1", "m2"):
        np.testing.assert_allclose(sa[k], sb[k], rtol=1e-5, atol=1e-8)
    # set_params starts over: moments and step count back to zero
    b.set_params(sa["params"])
    sb = b.get_state()
    assert sb["t"] == 0 and not sb["m1"].any() and not sb["m2"].any()
    a.close()
    b.close()
