"""GPU parity of the scorer network's kernels (mpdp_scorer.h) against
oracle/mlp.py.

Both sides hold the same bfloat16 values (inputs, weights) and round the
activations and back-propagated pre-activation gradients to bfloat16 at the
same points; the device sums in float32 (matrix cores for the wide layers)
where the oracle sums in float64.  A float32 sum of K terms is off by at most
about K * 2^-24 relative (K <= batch = 257 here: ~1.5e-5), which can move a
value across a bfloat16 rounding boundary now and then (one bfloat16 ulp,
2^-8 relative, on a small fraction of the elements).  Hence: logits within
2e-3 * (1 + |logit|) each, weight gradients within 1e-2 relative Frobenius
norm per tensor, loss within 1e-5 relative.
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
        back = mpdp.scorer_weights(block)
        for k in w:
            assert np.array_equal(back[k], w[k]), k


def test_gradients_match_oracle():
    for seed, B in ((5, 64), (6, 257)):
        print("grad", seed, B, flush=True)
        w = mlp.init_params(seed)
        w["b3"] = np.array([-0.7], np.float32)
        block = mpdp.scorer_params()
        mpdp.scorer_load(block, w)
        x, y = batch(100 + seed, B)
        loss = mpdp.scorer_grad(block, x, y)
        want_loss, want = mlp.loss_and_grads(w, x, y)
        assert abs(loss - want_loss) <= 1e-5 * abs(want_loss) + 1e-6, (loss, want_loss)
        got = mpdp.scorer_grads(block)
        for k in want:
            num = np.linalg.norm(got[k].astype(np.float64) - want[k])
            den = np.linalg.norm(want[k])
            assert num <= 1e-2 * den + 1e-7, (k, num / max(den, 1e-30))


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
