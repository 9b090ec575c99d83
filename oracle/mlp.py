"""FP64 reference of the learned order predictor — TEST INFRASTRUCTURE ONLY.

The predictor (a project addition, not in the paper) maps one active bin to a
class a in 0..L (its number of aliased frequencies), replacing the rank test
of the order estimate (the analogue of Pruning Step 1, Sec. III-C).

Features of a bin (L = 4, from its 2L de-rotated syndromes mt_l, energy
E = sum |mt_l|^2, mean bin energy E_ref):
    u_l = mt_l * conj(mt_0) / |mt_0| / rms,   rms = sqrt(E / 2L)
    f[2l], f[2l+1] = Re u_l, Im u_l            (l < 8)
    f[16 + l]      = |mt_l| / rms              (l < 8)
    f[24]          = log(E / E_ref)
    f[25..31]      = 0
(when mt_0 = 0 the phase factor is 1).

Network: h1 = gelu(W1 f + b1), h2 = gelu(W2 h1 + b2), z = W3 h2 + b3, with
W1 [128, 32], W2 [128, 128], W3 [5, 128] and gelu(x) = x Phi(x) (exact, erf).
Loss: mean cross-entropy.  Parameters are one flat FP32 vector in the order
W1, b1, W2, b2, W3, b3 (row-major), as in the C ABI.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

NF, NH, NC = 32, 128, 5
SIZES = [("W1", (NH, NF)), ("b1", (NH,)), ("W2", (NH, NH)), ("b2", (NH,)), ("W3", (NC, NH)), ("b3", (NC,))]
NPARAMS = sum(int(np.prod(s)) for _, s in SIZES)


def unpack(theta):
    theta = np.asarray(theta, np.float64)
    out, off = {}, 0
    for name, shape in SIZES:
        n = int(np.prod(shape))
        out[name] = theta[off:off + n].reshape(shape)
        off += n
    return out


def pack(p):
    return np.concatenate([np.asarray(p[name], np.float64).reshape(-1) for name, _ in SIZES])


def features(mt, e_ref):
    """Features of one bin from its 8 de-rotated syndromes (see module doc)."""
    mt = np.asarray(mt, np.complex128)
    e = float(np.sum(np.abs(mt) ** 2))
    rms = math.sqrt(e / 8.0)
    ph = np.conj(mt[0]) / abs(mt[0]) if abs(mt[0]) > 0 else 1.0
    u = mt * ph / rms
    f = np.zeros(NF)
    f[0:16:2] = u.real
    f[1:16:2] = u.imag
    f[16:24] = np.abs(mt) / rms
    f[24] = math.log(e / e_ref)
    return f


def gelu(x):
    return 0.5 * x * (1.0 + erf(x / math.sqrt(2.0)))


def gelu_grad(x):
    return 0.5 * (1.0 + erf(x / math.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)


def forward(theta, x, bf16=False):
    """Logits [n, 5] and the cache for backward.

    bf16=True rounds the weights W1..W3, the inputs and the hidden activations
    to bfloat16 where the device's MFMA path does (products then sum in FP64
    here, FP32 there)."""
    p = unpack(theta)
    x = np.asarray(x, np.float64)
    r = bf16_round if bf16 else (lambda v: v)
    w1, w2, w3 = r(p["W1"]), r(p["W2"]), r(p["W3"])
    x = r(x)
    z1 = x @ w1.T + p["b1"]
    h1 = r(gelu(z1))
    z2 = h1 @ w2.T + p["b2"]
    h2 = r(gelu(z2))
    z3 = h2 @ w3.T + p["b3"]
    return z3, (x, z1, h1, z2, h2)


def loss_and_grad(theta, x, labels, bf16=False, bf16_backward=False):
    """Mean cross-entropy and its gradient with respect to the flat parameters
    (bf16 as in forward: the gradient of the rounded network).

    bf16_backward=True also rounds the backward deltas where the device's
    MFMA products take them in bfloat16: dZ3 for dH2 = dZ3 W3 and
    dW3 = dZ3^T H2 (b3 keeps the unrounded dZ3), and dZ2 = dH2 * gelu'(Z2),
    dZ1 = dH1 * gelu'(Z1) for every later use (the weight gradients, the
    bias sums and the next backward product)."""
    p = unpack(theta)
    if bf16:
        p = dict(p, W1=bf16_round(p["W1"]), W2=bf16_round(p["W2"]), W3=bf16_round(p["W3"]))
    rb = bf16_round if bf16_backward else (lambda v: v)
    z3, (x, z1, h1, z2, h2) = forward(theta, x, bf16)
    n = len(labels)
    zmax = z3.max(axis=1, keepdims=True)
    ez = np.exp(z3 - zmax)
    prob = ez / ez.sum(axis=1, keepdims=True)
    labels = np.asarray(labels, np.int64)
    loss = float(-np.mean(np.log(prob[np.arange(n), labels])))
    dz3 = prob.copy()
    dz3[np.arange(n), labels] -= 1.0
    dz3 /= n
    dz3r = rb(dz3)
    g = {"W3": dz3r.T @ h2, "b3": dz3.sum(0)}
    dh2 = dz3r @ p["W3"]
    dz2 = rb(dh2 * gelu_grad(z2))
    g["W2"] = dz2.T @ h1
    g["b2"] = dz2.sum(0)
    dh1 = dz2 @ p["W2"]
    dz1 = rb(dh1 * gelu_grad(z1))
    g["W1"] = dz1.T @ x
    g["b1"] = dz1.sum(0)
    return loss, pack(g)


def predict(theta, x):
    z3, _ = forward(theta, x)
    return np.argmax(z3, axis=1)


def bf16_round(v):
    """Round FP32 values to bfloat16 (nearest, ties to even), back as float64."""
    a = np.asarray(v, np.float32).view(np.uint32).astype(np.uint64)
    a = (a + 0x7FFF + ((a >> 16) & 1)) & 0xFFFF0000
    return a.astype(np.uint32).view(np.float32).astype(np.float64)
