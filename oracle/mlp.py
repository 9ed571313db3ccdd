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


# ------------------------------------------------------------------ device error bounds
#
# How far the device's float32 results may lie from this float64 oracle,
# element by element.  Both sides start from the same bfloat16 inputs and
# weights and float32 biases; the device sums in float32 (any order, any
# grouping: a sum of K terms is within gamma(K) * sum|terms| of the exact
# sum, gamma(K) = K u / (1 - K u), with u = 2^-23 so that directed rounding
# inside the matrix cores is covered too).  Each bfloat16-rounded value
# (h1, h2, dz2, dz1) is then bounded by interval rounding: the device's value
# before rounding lies in [P - E, P + E] around the oracle's P, rounding to
# nearest is monotone, so the device's stored value is between
# bf16(P - E) and bf16(P + E); where both ends round to the oracle's value
# the stored values are equal and carry no error forward.  A ReLU mask is
# uncertain where that interval reaches both zero and positive values.

U32 = 2.0 ** -23


def gamma(k: int) -> float:
    return k * U32 / (1.0 - k * U32)


def lsb_exp(a) -> np.ndarray:
    """Exponent of the lowest set bit of each (binary64) value; +inf for 0."""
    a = np.asarray(a, np.float64)
    m, e = np.frexp(np.abs(a))
    M = (m * 2.0 ** 53).astype(np.int64)
    tz = np.zeros(M.shape, np.int64)
    nz = M != 0
    low = M & -M
    tz[nz] = np.log2(low[nz].astype(np.float64)).astype(np.int64)
    out = (e - 53 + tz).astype(np.float64)
    out[~nz] = np.inf
    return out


def exact_sums(A, B, bias=None) -> np.ndarray:
    """True where (A @ B + bias) is computed exactly by float32 additions in
    any order: every product A[i,k] B[k,j] (exact: bfloat16 x bfloat16, or
    the caller guarantees it) and the bias lie on the grid 2^g of the
    coarsest common lowest bit g, and sum|terms| < 2^(g + 24), so every
    partial sum is a float32."""
    la, lb = lsb_exp(A), lsb_exp(B)
    g = np.min(la[:, :, None] + lb[None, :, :], axis=1)
    tot = np.abs(A) @ np.abs(B)
    if bias is not None:
        g = np.minimum(g, lsb_exp(bias)[None, :])
        tot = tot + np.abs(bias)[None, :]
    return (tot < np.exp2(np.minimum(g, 900.0) + 24.0)) | (tot == 0)


def _bf16_interval(p, e):
    """Device value range of bf16(x) for x in [p - e, p + e]."""
    return bf16(p - e), bf16(p + e)


def error_bounds(params: dict, xbits: np.ndarray, y: np.ndarray) -> dict:
    """Per-element bounds on |device - oracle| for the logits and every
    gradient of loss_and_grads (same keys, plus "logit")."""
    logit, c = forward(params, xbits)
    x, h1, h2, w2, w3 = c["x"], c["h1"], c["h2"], c["w2"], c["w3"]
    w1 = bf16(params["w1"])
    b1 = np.asarray(params["b1"], np.float32).astype(np.float64)
    b2 = np.asarray(params["b2"], np.float32).astype(np.float64)
    b3 = np.asarray(params["b3"], np.float32).astype(np.float64)
    B = x.shape[0]
    ax, aw1, aw2, aw3 = np.abs(x), np.abs(w1), np.abs(w2), np.abs(w3)

    def stored(pre, e, mask_pre=None):
        """Bound on the stored bf16 value of relu(pre) (mask_pre None) or of
        pre where the mask is on: returns (oracle value, bound)."""
        lo, hi = _bf16_interval(pre, e)
        val = bf16(pre)
        if mask_pre is None:  # relu then round: monotone, clamp at 0
            lo, hi, val = np.maximum(lo, 0.0), np.maximum(hi, 0.0), np.maximum(val, 0.0)
            return val, np.maximum(hi - val, val - lo)
        on, maybe = mask_pre
        val = np.where(on, val, 0.0)
        lo_all = np.where(maybe, np.minimum(lo, 0.0), np.where(on, lo, 0.0))
        hi_all = np.where(maybe, np.maximum(hi, 0.0), np.where(on, hi, 0.0))
        return val, np.maximum(hi_all - val, val - lo_all)

    def relu_mask(pre, e):
        """(oracle's mask, mask uncertain) for a stored relu(pre)."""
        lo, hi = _bf16_interval(np.maximum(pre, 0.0), 0.0 * pre)
        on = np.maximum(bf16(pre), 0.0) > 0
        dev_lo, dev_hi = np.maximum(bf16(pre - e), 0.0), np.maximum(bf16(pre + e), 0.0)
        return on, (dev_lo > 0) != (dev_hi > 0)

    def sum_err(A, Bm, e_in, bias=None):
        """Float32 summation error of A @ Bm (+ bias) whose inputs A carry
        the errors e_in: zero where the inputs are exact and the sum is."""
        k = A.shape[1] + 2
        tot = (np.abs(A) + e_in) @ np.abs(Bm) + (0.0 if bias is None else np.abs(bias))
        e = e_in @ np.abs(Bm) + gamma(k) * tot
        exact = exact_sums(A, Bm, bias) & ~np.any(e_in > 0, axis=1)[:, None]
        return np.where(exact, 0.0, e)

    # forward
    z1 = x @ w1 + b1
    e_z1 = sum_err(x, w1, np.zeros_like(x), b1)
    h1v, e_h1 = stored(z1, e_z1)
    m1 = relu_mask(z1, e_z1)
    z2 = h1 @ w2 + b2
    e_z2 = sum_err(h1, w2, e_h1, b2)
    h2v, e_h2 = stored(z2, e_z2)
    m2 = relu_mask(z2, e_z2)
    e_logit = sum_err(h2, w3[:, None], e_h2, b3)[:, 0]
    # dlogit = (sigmoid(logit) - y) / B: sigmoid is 1/4-Lipschitz; the
    # float32 exp, add, divide, subtract and scale add a few roundings
    g = (1.0 / (1.0 + np.exp(-logit)) - np.asarray(y, np.float64)) / B
    e_g = (e_logit / 4.0 + 16.0 * U32) / B
    ag = np.abs(g)
    # head gradients (float32 sums over the batch)
    dw3 = e_h2.T @ ag + (np.abs(h2) + e_h2).T @ e_g + gamma(B + 1) * ((np.abs(h2) + e_h2).T @ (ag + e_g))
    db3 = np.array([e_g.sum() + gamma(B + 1) * (ag + e_g).sum()])
    # dz2 = bf16(g * w3) where h2 > 0 (float32 product: one more rounding)
    p2 = g[:, None] * w3[None, :]
    e_p2 = e_g[:, None] * aw3[None, :] + U32 * (ag + e_g)[:, None] * aw3[None, :]
    dz2v, e_dz2 = stored(p2, e_p2, m2)
    adz2 = np.abs(dz2v)
    dw2 = np.abs(h1).T @ e_dz2 + e_h1.T @ (adz2 + e_dz2) + gamma(B + 1) * ((np.abs(h1) + e_h1).T @ (adz2 + e_dz2))
    dw2 = np.where(exact_sums(h1.T, dz2v) & ~np.any(e_h1 > 0, axis=0)[:, None] & ~np.any(e_dz2 > 0, axis=0)[None, :],
                   0.0, dw2)
    db2 = e_dz2.sum(axis=0) + gamma(B + 1) * (adz2 + e_dz2).sum(axis=0)
    # dz1 = bf16(dz2 w2^T) where h1 > 0
    p1 = dz2v @ w2.T
    e_p1 = sum_err(dz2v, w2.T, e_dz2)
    dz1v, e_dz1 = stored(p1, e_p1, m1)
    adz1 = np.abs(dz1v)
    dw1 = ax.T @ e_dz1 + gamma(B + 1) * (ax.T @ (adz1 + e_dz1))
    dw1 = np.where(exact_sums(x.T, dz1v) & ~np.any(e_dz1 > 0, axis=0)[None, :], 0.0, dw1)
    db1 = e_dz1.sum(axis=0) + gamma(B + 1) * (adz1 + e_dz1).sum(axis=0)
    return dict(logit=e_logit, w1=dw1, b1=db1, w2=dw2, b2=db2, w3=dw3, b3=db3)
