"""Pins of the scorer network's oracle (oracle/mlp.py).

  * bfloat16 rounding: exact values, ties to even, NaN;
  * the gradient formulas against central finite differences of the loss in
    float64 with rounding switched off, on parameters of every layer (a
    transposed operand, a missing ReLU mask or a wrong loss derivative fails);
  * the loss at zero weights is log 2 and its bias gradient is mean(0.5 - y).
"""
import numpy as np

from oracle import mlp


def test_bf16_rounding():
    assert mlp.bf16_bits(1.0)[()] == 0x3F80
    assert mlp.bf16_bits(-2.0)[()] == 0xC000
    assert mlp.bf16_bits(1.0 + 2.0 ** -8)[()] == 0x3F80          # tie, even stays
    assert mlp.bf16_bits(1.0 + 3 * 2.0 ** -8)[()] == 0x3F82      # tie, rounds up to even
    assert mlp.bf16_bits(1.0 + 2.0 ** -8 + 2.0 ** -12)[()] == 0x3F81
    assert (mlp.bf16_bits(np.nan)[()] & 0x7F80) == 0x7F80 and (mlp.bf16_bits(np.nan)[()] & 0x7F) != 0
    assert mlp.bf16_value(np.uint16(0x4049))[()] == 3.140625


def test_gradients_against_finite_differences():
    rng = np.random.Generator(np.random.PCG64(3))
    p = {k: v.astype(np.float64) for k, v in mlp.init_params(7).items()}
    p["b1"] = rng.normal(0, 0.1, mlp.HID)
    p["b2"] = rng.normal(0, 0.1, mlp.HID)
    p["b3"] = np.array([0.3])
    x = rng.normal(0, 1, (12, mlp.IN))
    y = (rng.random(12) < 0.4).astype(np.float64)
    loss, g = mlp.loss_and_grads(p, x, y, rounding=False)
    h = 1e-6
    for name, shape in (("w1", (mlp.IN, mlp.HID)), ("b1", (mlp.HID,)), ("w2", (mlp.HID, mlp.HID)),
                        ("b2", (mlp.HID,)), ("w3", (mlp.HID,)), ("b3", (1,))):
        flat = [tuple(int(i) for i in np.unravel_index(j, shape)) for j in rng.choice(int(np.prod(shape)), 6)]
        for idx in flat:
            q = {k: v.copy() for k, v in p.items()}
            q[name][idx] += h
            lp, _ = mlp.loss_and_grads(q, x, y, rounding=False)
            q[name][idx] -= 2 * h
            lm, _ = mlp.loss_and_grads(q, x, y, rounding=False)
            fd = (lp - lm) / (2 * h)
            assert abs(fd - g[name][idx]) <= 1e-6 + 1e-4 * abs(fd), (name, idx, fd, g[name][idx])


def test_zero_network():
    z = {k: np.zeros_like(v) for k, v in mlp.init_params(0).items()}
    x = mlp.bf16_bits(np.ones((4, mlp.IN)))
    y = np.array([0.0, 1.0, 1.0, 1.0])
    loss, g = mlp.loss_and_grads(z, x, y)
    assert abs(loss - np.log(2.0)) < 1e-15
    assert abs(g["b3"][0] - np.mean(0.5 - y)) < 1e-15
    assert not np.any(g["w1"]) and not np.any(g["w2"]) and not np.any(g["w3"])
