"""Pins of the scorer network's oracle (oracle/mlp.py).

  * bfloat16 rounding: exact values, ties to even, NaN;
  * the gradient formulas against central finite differences of the loss in
    float64 with rounding switched off, on parameters of every layer (a
    transposed operand, a missing ReLU mask or a wrong loss derivative fails);
  * the loss at zero weights is log 2 and its bias gradient is mean(0.5 - y).
"""
import numpy as np
import pytest

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


def _f32_device_like(w, xbits, y, order):
    """The network in float32 with bfloat16 storage at the device's points;
    `order` picks the summation order of the wide products (BLAS, or a
    sequential float32 sum in reverse)."""
    def mm(A, B):
        A = np.asarray(A, np.float32)
        B = np.asarray(B, np.float32)
        if order == "blas":
            return A @ B
        out = np.zeros((A.shape[0], B.shape[1]), np.float32)
        for k in reversed(range(A.shape[1])):
            out = (out + A[:, k:k + 1] * B[k:k + 1, :]).astype(np.float32)
        return out

    bf = lambda a: mlp.bf16(a).astype(np.float32)  # noqa: E731
    x = mlp.bf16_value(xbits).astype(np.float32)
    w1, w2, w3 = bf(w["w1"]), bf(w["w2"]), bf(w["w3"])
    b1, b2, b3 = (np.asarray(w[k], np.float32) for k in ("b1", "b2", "b3"))
    h1 = bf(np.maximum(mm(x, w1) + b1, 0))
    h2 = bf(np.maximum(mm(h1, w2) + b2, 0))
    logit = (mm(h2, w3[:, None])[:, 0] + b3[0]).astype(np.float32)
    B = x.shape[0]
    p = (np.float32(1) / (np.float32(1) + np.exp(-logit))).astype(np.float32)
    g = ((p - np.asarray(y, np.float32)) / np.float32(B)).astype(np.float32)
    dw3 = mm(h2.T, g[:, None])[:, 0]
    db3 = np.array([g.sum(dtype=np.float32)])
    dz2 = np.where(h2 > 0, bf(g[:, None] * w3[None, :]), 0).astype(np.float32)
    dw2 = mm(h1.T, dz2)
    db2 = dz2.sum(axis=0, dtype=np.float32)
    dz1 = np.where(h1 > 0, bf(mm(dz2, w2.T)), 0).astype(np.float32)
    dw1 = mm(x.T, dz1)
    db1 = dz1.sum(axis=0, dtype=np.float32)
    return dict(logit=logit, w1=dw1, b1=db1, w2=dw2, b2=db2, w3=dw3, b3=db3)


@pytest.mark.parametrize("kind", ["grid", "he"])
def test_error_bounds_cover_float32_runs(kind):
    """oracle.mlp.error_bounds holds for float32 runs of the same network in
    two summation orders; on few-bit weights most bounds are zero and the
    float32 runs hit them exactly."""
    rng = np.random.Generator(np.random.PCG64(3))
    B = 96
    if kind == "grid":
        g = lambda q, lim, shape: (rng.integers(-lim, lim + 1, size=shape) / q).astype(np.float32)  # noqa: E731
        w = dict(w1=g(32, 8, (mlp.IN, mlp.HID)), b1=g(8, 2, mlp.HID), w2=g(16, 2, (mlp.HID, mlp.HID)),
                 b2=g(8, 2, mlp.HID), w3=g(64, 4, mlp.HID), b3=np.array([-0.75], np.float32))
        x = mlp.bf16_bits(rng.integers(-4, 5, size=(B, mlp.IN)) / 4.0)
    else:
        w = mlp.init_params(4)
        x = mlp.bf16_bits(rng.normal(0.0, 1.0, (B, mlp.IN)))
    y = (rng.random(B) < 0.3).astype(np.float32)
    logit, _ = mlp.forward(w, x)
    _, want = mlp.loss_and_grads(w, x, y)
    want["logit"] = logit
    E = mlp.error_bounds(w, x, y)
    for order in ("blas", "reverse"):
        got = _f32_device_like(w, x, y, order)
        for k in want:
            d = np.abs(got[k].astype(np.float64) - want[k])
            assert np.all(d <= E[k]), (kind, order, k, float((d - E[k]).max()))
    if kind == "grid":
        assert np.all(E["logit"] == 0) and np.mean(E["w2"] == 0) > 0.5


def test_exact_sums_grid_rule():
    """exact_sums: terms on a 2^g grid with sum|terms| < 2^(g+24) are exact
    in float32; one term off the grid, or a total too large, is not."""
    A = np.array([[1.0, 2.0 ** -10, 3.0]])
    B = np.array([[1.0], [1.0], [1.0]])
    assert mlp.exact_sums(A, B)[0, 0]
    A2 = np.array([[2.0 ** 14, 2.0 ** -10, 3.0]])  # needs 25 bits
    assert not mlp.exact_sums(A2, B)[0, 0]
    assert mlp.lsb_exp(np.array([0.75, 8.0, 0.0])).tolist() == [-2.0, 3.0, float("inf")]
