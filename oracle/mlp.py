"""CPU oracle of the learned subgraph scorer's network (mpdp_scorer.h).
TEST INFRASTRUCTURE ONLY: tests, the smoke check and the benchmark's
CPU-baseline leg may use it; the library never does.

The network: h1 = relu(x w1 + b1), h2 = relu(h1 w2 + b2), logit = h2 . w3 + b3,
trained on the mean binary cross-entropy with logits.  Arithmetic here is
float64; values are rounded to bfloat16 (round to nearest even) exactly where
the device keeps bfloat16: the inputs x, the weights w1, w2, w3 (copies of
float32 master values), the activations h1 and h2, and the back-propagated
pre-activation gradients dz2 and dz1.  ReLU's derivative is taken where the
stored activation is positive.  Everything else (sums, biases, the loss, the
gradients of the weights) stays float64, so the device's float32
accumulation is the only difference left, which the tests bound.
"""
from __future__ import annotations

import numpy as np

IN, HID = 32, 256


def f32(x):
    return np.asarray(x, dtype=np.float64).astype(np.float32)


def bf16_bits(x) -> np.ndarray:
    """Round to bfloat16 (nearest even) via float32; returns uint16 bit patterns."""
    u = np.asarray(f32(x)).view(np.uint32).astype(np.uint64)
    nan = (u & 0x7FFFFFFF) > 0x7F800000
    rounded = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return np.where(nan, (u >> 16) | 0x40, rounded).astype(np.uint16)


def bf16_value(bits) -> np.ndarray:
    return (np.asarray(bits, dtype=np.uint32) << 16).view(np.float32).astype(np.float64)


def bf16(x) -> np.ndarray:
    return bf16_value(bf16_bits(x))


def forward(params: dict, xbits: np.ndarray, rounding: bool = True):
    """params: float32 master arrays w1 (IN, HID), b1, w2 (HID, HID), b2, w3 (HID,), b3 (1,).
    xbits: (B, IN) uint16 bfloat16 inputs.  Returns (logits, cache).
    rounding=False keeps every value in float64 (for finite-difference
    checks of the formulas; params are then used as given)."""
    r = bf16 if rounding else (lambda a: np.asarray(a, np.float64))
    x = bf16_value(xbits) if xbits.dtype == np.uint16 else np.asarray(xbits, np.float64)
    w1, w2, w3 = r(params["w1"]), r(params["w2"]), r(params["w3"])
    cast = (lambda k: np.asarray(params[k], np.float32).astype(np.float64)) if rounding else \
        (lambda k: np.asarray(params[k], np.float64))
    b1, b2, b3 = cast("b1"), cast("b2"), cast("b3")
    z1 = x @ w1 + b1
    h1 = r(np.maximum(z1, 0.0))
    z2 = h1 @ w2 + b2
    h2 = r(np.maximum(z2, 0.0))
    logit = h2 @ w3 + b3[0]
    return logit, dict(x=x, h1=h1, h2=h2, w2=w2, w3=w3)


def loss_and_grads(params: dict, xbits: np.ndarray, y: np.ndarray, rounding: bool = True):
    """Mean BCE with logits and the gradients of every parameter (float64)."""
    r = bf16 if rounding else (lambda a: np.asarray(a, np.float64))
    logit, c = forward(params, xbits, rounding)
    B = logit.shape[0]
    y = np.asarray(y, np.float64)
    loss = np.mean(np.maximum(logit, 0.0) - logit * y + np.log1p(np.exp(-np.abs(logit))))
    g = (1.0 / (1.0 + np.exp(-logit)) - y) / B
    dw3 = c["h2"].T @ g
    db3 = np.array([g.sum()])
    dz2 = r(np.where(c["h2"] > 0, g[:, None] * c["w3"][None, :], 0.0))
    dw2 = c["h1"].T @ dz2
    db2 = dz2.sum(axis=0)
    dz1 = r(np.where(c["h1"] > 0, dz2 @ c["w2"].T, 0.0))
    dw1 = c["x"].T @ dz1
    db1 = dz1.sum(axis=0)
    return loss, dict(w1=dw1, b1=db1, w2=dw2, b2=db2, w3=dw3, b3=db3)


def init_params(seed: int) -> dict:
    """He-uniform weights, zero biases, from PCG64(seed) (the caller's draw)."""
    rng = np.random.Generator(np.random.PCG64(seed))

    def he(fan_in, shape):
        lim = np.sqrt(6.0 / fan_in)
        return rng.uniform(-lim, lim, size=shape).astype(np.float32)

    return dict(w1=he(IN, (IN, HID)), b1=np.zeros(HID, np.float32), w2=he(HID, (HID, HID)),
                b2=np.zeros(HID, np.float32), w3=he(HID, (HID,)), b3=np.zeros(1, np.float32))
