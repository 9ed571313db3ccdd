"""GPU parity of the scorer network's kernels (mpdp_scorer.h) against
oracle/mlp.py.

Both sides hold the same bfloat16 values (inputs, weights) and round the
activations and back-propagated pre-activation gradients to bfloat16 at the
same points; the device sums in float32 (matrix cores for the wide layers)
where the oracle sums in float64.  Every logit and every gradient element is
compared with its own bound from oracle.mlp.error_bounds: float32
summation error gamma(K) * sum|terms| (zero where the terms sit on a common
binary grid narrow enough for every partial sum to be a float32), carried
through the bfloat16 roundings by interval rounding (a stored value may
differ only where its interval crosses a rounding boundary).  Batches of
few-bit inputs and weights keep most sums exact, so most bounds are zero or
a few 1e-4 of the value; batches of He-initialised weights get the same
rigorous, looser bounds.  The loss is a float32 sum: within 1e-5 relative.
"""
import numpy as np
import pytest

from oracle import mlp
from paper_2202_13511_amd import mpdp

pytestmark = pytest.mark.gpu


def batch(seed, B):
    rng = np.random.Generator(np.random.PCG64(seed))
    x = mlp.bf16_bits(rng.normal(0.0, 1.0, (B, mlp.IN)))
    y = (rng.random(B) < 0.3).astype(np.float32)
    return x, y


def grid_params(seed):
    """Weights on coarse binary grids (w1: multiples of 1/32 up to 1/4; w2:
    of 1/16 up to 1/8; w3: of 1/64 up to 1/16; biases of 1/8)."""
    rng = np.random.Generator(np.random.PCG64(seed))

    def g(q, lim, shape):
        return (rng.integers(-lim, lim + 1, size=shape) / q).astype(np.float32)

    return dict(w1=g(32, 8, (mlp.IN, mlp.HID)), b1=g(8, 2, mlp.HID), w2=g(16, 2, (mlp.HID, mlp.HID)),
                b2=g(8, 2, mlp.HID), w3=g(64, 4, mlp.HID), b3=np.array([-0.75], np.float32))


def grid_batch(seed, B):
    """Inputs on multiples of 1/4 in [-1, 1]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    x = mlp.bf16_bits(rng.integers(-4, 5, size=(B, mlp.IN)) / 4.0)
    y = (rng.random(B) < 0.3).astype(np.float32)
    return x, y


def within(got, want, bound, name):
    d = np.abs(np.asarray(got, np.float64) - want)
    bad = d > bound
    assert not np.any(bad), (name, int(bad.sum()), float(d[bad].max()), np.argwhere(bad)[:4].tolist())


def test_forward_matches_oracle():
    for seed, B in ((1, 1), (2, 63), (3, 257), (4, 1024)):
        print("forward", seed, B, flush=True)
        w = mlp.init_params(seed)
        block = mpdp.scorer_params()
        mpdp.scorer_load(block, w)
        x, _ = batch(seed, B)
        got = mpdp.scorer_forward(block, x)
        want, _ = mlp.forward(w, x)
        assert got.shape == (B,)
        assert np.all(np.abs(got - want) <= 2e-3 * (1.0 + np.abs(want))), (seed, B, np.max(np.abs(got - want)))
        within(got, want, mlp.error_bounds(w, x, np.zeros(B, np.float32))["logit"], ("logit", seed, B))
        back = mpdp.scorer_weights(block)
        for k in w:
            assert np.array_equal(back[k], w[k]), k
    # few-bit weights and inputs: every logit sum is exact, so the logits are equal
    for seed, B in ((7, 100), (8, 1024)):
        w = grid_params(seed)
        block = mpdp.scorer_params()
        mpdp.scorer_load(block, w)
        x, _ = grid_batch(seed, B)
        got = mpdp.scorer_forward(block, x)
        want, _ = mlp.forward(w, x)
        within(got, want, mlp.error_bounds(w, x, np.zeros(B, np.float32))["logit"], ("grid logit", seed, B))


@pytest.mark.parametrize("kind,seed,B", [("grid", 5, 64), ("grid", 6, 257), ("he", 5, 64), ("he", 6, 257)])
def test_gradients_match_oracle(kind, seed, B):
    """Every element of every gradient within its own bound."""
    print("grad", kind, seed, B, flush=True)
    if kind == "grid":
        w = grid_params(seed)
        x, y = grid_batch(100 + seed, B)
    else:
        w = mlp.init_params(seed)
        w["b3"] = np.array([-0.7], np.float32)
        x, y = batch(100 + seed, B)
    block = mpdp.scorer_params()
    mpdp.scorer_load(block, w)
    loss = mpdp.scorer_grad(block, x, y)
    want_loss, want = mlp.loss_and_grads(w, x, y)
    assert abs(loss - want_loss) <= 1e-5 * abs(want_loss) + 1e-6, (loss, want_loss)
    got = mpdp.scorer_grads(block)
    bounds = mlp.error_bounds(w, x, y)
    for k in want:
        within(got[k], want[k], bounds[k], (kind, k))


def test_adam_step_and_training_reduce_loss():
    w = mlp.init_params(9)
    block = mpdp.scorer_params()
    mpdp.scorer_load(block, w)
    x, y = batch(11, 512)
    _, g = mlp.loss_and_grads(w, x, y)
    lr = 1e-3
    l0 = mpdp.scorer_train_step(block, x, y, lr, 1)
    w1 = mpdp.scorer_weights(block)
    # first Adam step: w -= lr * g / (|g| + eps), i.e. lr * sign(g) where |g| >> eps
    for k in w:
        big = np.abs(g[k]) > 1e-5
        step = (w[k].astype(np.float64) - w1[k].astype(np.float64))[big]
        assert np.mean(np.sign(step) == np.sign(g[k][big])) >= 0.99, k
        assert np.allclose(np.abs(step), lr, rtol=1e-2, atol=1e-6), k
    losses = [l0]
    for t in range(2, 41):
        losses.append(mpdp.scorer_train_step(block, x, y, lr, t))
    assert losses[-1] < 0.5 * losses[0], losses[::8]
