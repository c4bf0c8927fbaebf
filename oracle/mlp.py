"""FP64 reference of the candidate-proposal MLP -- test infrastructure only.

The learned proposal form is not in the paper; the network, its
initialisation, loss and optimizer are readings fixed for this library (they
decide only which centroids are proposed; a proposal is accepted only under a
triangle-inequality certificate, so labels never depend on them):

  architecture   d -> h -> h -> k, ReLU after the two hidden layers
                 (d=32, h=256, k=4096 for the learned workload)
  parameters     one flat vector, in this order: W1 (d x h, row-major, W1[i][j]
                 joins input i to unit j), b1 (h), W2 (h x h), b2 (h),
                 W3 (h x k), b3 (k)
  init           He-uniform: W[i][j] = (2u - 1) sqrt(6 / fan_in), with u the
                 next SplitMix64 (Steele, Lea, Flood 2014) output of `seed`
                 taken as (z >> 11) * 2^-53, drawn in parameter order; b = 0
  inputs         standardized: (x - mean) / std per dimension (population std;
                 std = 0 -> 1)
  loss           mean softmax cross-entropy of the labels
  optimizer      Adam, lr 1e-3, beta (0.9, 0.999), eps 1e-8, bias-corrected
  precision      every matrix-product operand is rounded to BF16 (round to
                 nearest even) and products are summed in FP32 on the GPU; this
                 reference rounds the same operands and sums in FP64.  Bias
                 sums, softmax and Adam are FP32 on the GPU, FP64 here.

With bf16=False every operand is kept exact: the plain FP64 network, which the
finite-difference pin checks.
"""
from __future__ import annotations

import numpy as np

ADAM_LR, ADAM_B1, ADAM_B2, ADAM_EPS = 1e-3, 0.9, 0.999, 1e-8

_M64 = (1 << 64) - 1


def splitmix64(state: int, count: int) -> tuple[int, np.ndarray]:
    """count outputs of SplitMix64 from `state`; returns (new state, outputs)."""
    out = np.empty(count, dtype=np.uint64)
    for i in range(count):
        state = (state + 0x9E3779B97F4A7C15) & _M64
        z = state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
        out[i] = z ^ (z >> 31)
    return state, out


def layer_shapes(d: int, h: int, k: int):
    return [("W1", (d, h)), ("b1", (h,)), ("W2", (h, h)), ("b2", (h,)),
            ("W3", (h, k)), ("b3", (k,))]


def param_count(d: int, h: int, k: int) -> int:
    return int(sum(np.prod(s) for _, s in layer_shapes(d, h, k)))


def unflatten(theta: np.ndarray, d: int, h: int, k: int) -> dict:
    out, o = {}, 0
    for name, shape in layer_shapes(d, h, k):
        m = int(np.prod(shape))
        out[name] = theta[o:o + m].reshape(shape)
        o += m
    return out


def init_params(d: int, h: int, k: int, seed: int) -> np.ndarray:
    """He-uniform weights from one SplitMix64 stream, zero biases (FP64)."""
    theta = np.zeros(param_count(d, h, k), np.float64)
    p = unflatten(theta, d, h, k)
    state = seed
    for name, fan_in in (("W1", d), ("W2", h), ("W3", h)):
        W = p[name]
        state, z = splitmix64(state, W.size)
        u = (z >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
        W[...] = ((2.0 * u - 1.0) * np.sqrt(6.0 / fan_in)).reshape(W.shape)
    return theta


def bf16(a: np.ndarray) -> np.ndarray:
    """Round FP64 values to the nearest BF16 value (ties to even), as FP64.
    The value is first rounded to FP32, as the GPU keeps it in FP32."""
    f = np.asarray(a, dtype=np.float32)
    b = f.view(np.uint32).astype(np.uint64)
    lsb = (b >> np.uint64(16)) & np.uint64(1)
    r = (b + np.uint64(0x7FFF) + lsb) & np.uint64(0xFFFF0000)
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def standardize(X: np.ndarray):
    """(mean, std) per dimension in FP64; std = 0 is replaced by 1."""
    X = np.asarray(X, np.float64)
    mean = X.mean(axis=0)
    std = np.sqrt(((X - mean) ** 2).mean(axis=0))
    std[std == 0] = 1.0
    return mean, std


def _op(a, use_bf16):
    return bf16(a) if use_bf16 else np.asarray(a, np.float64)


def forward(theta, Xs, d, h, k, use_bf16=True):
    """Returns (h1, h2, z): hidden activations and logits."""
    p = unflatten(theta, d, h, k)
    h1 = np.maximum(_op(Xs, use_bf16) @ _op(p["W1"], use_bf16) + p["b1"], 0.0)
    h2 = np.maximum(_op(h1, use_bf16) @ _op(p["W2"], use_bf16) + p["b2"], 0.0)
    z = _op(h2, use_bf16) @ _op(p["W3"], use_bf16) + p["b3"]
    return h1, h2, z


def loss_and_grad(theta, Xs, y, d, h, k, use_bf16=True):
    """Mean softmax cross-entropy of labels y and its gradient (flat)."""
    B = Xs.shape[0]
    p = unflatten(theta, d, h, k)
    h1, h2, z = forward(theta, Xs, d, h, k, use_bf16)
    zmax = z.max(axis=1, keepdims=True)
    e = np.exp(z - zmax)
    s = e.sum(axis=1, keepdims=True)
    loss = float(np.mean(np.log(s[:, 0]) + zmax[:, 0] - z[np.arange(B), y]))
    dz = e / s
    dz[np.arange(B), y] -= 1.0
    dz /= B
    g = np.zeros_like(theta)
    G = unflatten(g, d, h, k)
    G["W3"][...] = _op(h2, use_bf16).T @ _op(dz, use_bf16)
    G["b3"][...] = dz.sum(axis=0)
    dh2 = (_op(dz, use_bf16) @ _op(p["W3"], use_bf16).T) * (h2 > 0)
    G["W2"][...] = _op(h1, use_bf16).T @ _op(dh2, use_bf16)
    G["b2"][...] = dh2.sum(axis=0)
    dh1 = (_op(dh2, use_bf16) @ _op(p["W2"], use_bf16).T) * (h1 > 0)
    G["W1"][...] = _op(Xs, use_bf16).T @ _op(dh1, use_bf16)
    G["b1"][...] = dh1.sum(axis=0)
    return loss, g


def adam_step(theta, m, v, g, t, lr=ADAM_LR):
    """One Adam step (t = the step number after this update, from 1)."""
    m = ADAM_B1 * m + (1.0 - ADAM_B1) * g
    v = ADAM_B2 * v + (1.0 - ADAM_B2) * g * g
    mh = m / (1.0 - ADAM_B1 ** t)
    vh = v / (1.0 - ADAM_B2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + ADAM_EPS), m, v
