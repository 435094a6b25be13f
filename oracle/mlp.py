"""CPU oracle of the learned speculation proposal (TEST INFRASTRUCTURE ONLY).

Not part of the paper: the benchmark plan adds a small MLP that ranks DFA
states at a chunk boundary from the 32 bytes before it. This module is its
plain float64 definition, forward and backward, written out with numpy:

    x      = concat(emb[w_0], ..., emb[w_31])              (32 x 16 = 512)
    h1     = gelu(W1 x + b1)                                (256)
    h2     = gelu(W2 h1 + b2)                               (256)
    z      = W3 h2 + b3                                     (one logit per state)
    loss   = -log softmax(z masked to the allowed states)[label]

gelu(u) = u * Phi(u) with Phi the standard normal CDF (the erf form).
Parameter layout (one flat float vector, in this order): emb [256, 16],
W1 [256, 512], b1 [256], W2 [256, 256], b2 [256], W3 [S, 256], b3 [S], where
S is the number of head rows (the DFA's state count). The optimizer is
AdamW (decoupled weight decay).

Operand precision. The network is specified with bf16 operands and wide
accumulation. ``forward`` and ``loss_and_grad`` take an optional rounding
function ``rnd`` applied where a value becomes an operand of a product: the
hidden activations h1 and h2, and the back-propagated products' left
operands dz, da2 and da1 (the bias gradients sum the unrounded values). With
``rnd=None`` every value stays float64: the exact definition, which the
finite-difference pins check. With ``rnd=bf16_round`` the sums still run in
float64, so the only difference from the exact definition is where operands
are rounded, as the specified arithmetic rounds them (the weight matrices and
the embedding are rounded by the caller, biases stay fp32).
"""
from __future__ import annotations

import math

import numpy as np

WINDOW = 32
EMB = 16
HID = 256
IN = WINDOW * EMB

_SQRT2 = math.sqrt(2.0)
_INV_SQRT_2PI = 1.0 / math.sqrt(2.0 * math.pi)
_erf = np.vectorize(math.erf, otypes=[np.float64])


def param_shapes(states: int):
    return [("emb", (256, EMB)), ("W1", (HID, IN)), ("b1", (HID,)), ("W2", (HID, HID)), ("b2", (HID,)),
            ("W3", (states, HID)), ("b3", (states,))]


def param_count(states: int) -> int:
    return sum(int(np.prod(s)) for _, s in param_shapes(states))


def unpack(flat: np.ndarray, states: int) -> dict:
    out, k = {}, 0
    for name, shape in param_shapes(states):
        n = int(np.prod(shape))
        out[name] = flat[k:k + n].reshape(shape)
        k += n
    assert k == flat.size
    return out


def pack(p: dict) -> np.ndarray:
    return np.concatenate([np.asarray(p[name], dtype=np.float64).reshape(-1) for name, _ in param_shapes(
        p["W3"].shape[0])])


def gelu(u):
    return 0.5 * u * (1.0 + _erf(u / _SQRT2))


def gelu_grad(u):
    return 0.5 * (1.0 + _erf(u / _SQRT2)) + u * _INV_SQRT_2PI * np.exp(-0.5 * u * u)


PAD = 256  # window index of a byte before the text start: embeds as zeros


def _identity(a):
    return a


def _rounder(rnd):
    if rnd is None:
        return _identity
    return lambda a: rnd(np.asarray(a, dtype=np.float32)).astype(np.float64)


def forward(flat, states, windows, mask, rnd=None):
    """windows: [B, 32] byte values or PAD; mask: [B, S] bool (allowed
    states). Returns logits [B, S] (masked entries -inf) and the cache for
    backward. ``rnd`` rounds the hidden activations (see the module notes)."""
    r = _rounder(rnd)
    p = unpack(np.asarray(flat, dtype=np.float64), states)
    emb = np.vstack([p["emb"], np.zeros((1, EMB))])
    x = emb[np.asarray(windows, dtype=np.int64)].reshape(len(windows), IN)
    a1 = x @ p["W1"].T + p["b1"]
    h1 = r(gelu(a1))
    a2 = h1 @ p["W2"].T + p["b2"]
    h2 = r(gelu(a2))
    z = h2 @ p["W3"].T + p["b3"]
    z = np.where(mask, z, -np.inf)
    return z, (p, x, a1, h1, a2, h2)


def loss_and_grad(flat, states, windows, mask, labels, rnd=None, denom=None):
    """Mean masked softmax cross-entropy and its gradient (flat, float64).
    ``rnd`` rounds the products' operands (see the module notes). ``denom``
    replaces the row count as the mean's divisor (a batch some of whose rows
    were left out still divides by its full size)."""
    r = _rounder(rnd)
    z, (p, x, a1, h1, a2, h2) = forward(flat, states, windows, mask, rnd)
    b = len(labels)
    nb = b if denom is None else denom
    zmax = np.max(z, axis=1, keepdims=True)
    e = np.where(mask, np.exp(z - zmax), 0.0)
    s = e.sum(axis=1, keepdims=True)
    prob = e / s
    lab = np.asarray(labels, dtype=np.int64)
    loss = float(np.sum(np.log(s[:, 0]) + zmax[:, 0] - z[np.arange(b), lab]) / nb)
    dz = prob.copy()
    dz[np.arange(b), lab] -= 1.0
    dz /= nb
    g = {}
    dzr = r(dz)
    g["W3"] = dzr.T @ h2
    g["b3"] = dz.sum(axis=0)
    dh2 = dzr @ p["W3"]
    da2 = dh2 * gelu_grad(a2)
    da2r = r(da2)
    g["W2"] = da2r.T @ h1
    g["b2"] = da2.sum(axis=0)
    dh1 = da2r @ p["W2"]
    da1 = dh1 * gelu_grad(a1)
    da1r = r(da1)
    g["W1"] = da1r.T @ x
    g["b1"] = da1.sum(axis=0)
    dx = (da1r @ p["W1"]).reshape(b, WINDOW, EMB)
    demb = np.zeros((257, EMB))
    np.add.at(demb, np.asarray(windows, dtype=np.int64), dx)
    g["emb"] = demb[:256]  # the pad row is constant
    return loss, pack(g)


def magnitudes(flat, states, windows, mask, labels, rnd=None, denom=None):
    """Error-bound scale of every logit and gradient entry: the entry's own
    last sum taken over absolute values of its terms (sum_k |a_k| |b_k|, plus
    |bias|), with the operands that sum has under ``rnd``. A floating-point
    error bound of a sum is proportional to this quantity. Returns (logit
    scale [B, S], gradient scale, flat like the parameters). For tolerances
    only."""
    r = _rounder(rnd)
    z, (p, x, a1, h1, a2, h2) = forward(flat, states, windows, mask, rnd)
    b = len(labels)
    ab = {k: np.abs(v) for k, v in p.items()}
    zs = np.abs(h2) @ ab["W3"].T + ab["b3"]
    zmax = np.max(z, axis=1, keepdims=True)
    e = np.where(mask, np.exp(z - zmax), 0.0)
    prob = e / e.sum(axis=1, keepdims=True)
    lab = np.asarray(labels, dtype=np.int64)
    dz = prob.copy()
    dz[np.arange(b), lab] -= 1.0
    dz /= b if denom is None else denom
    dzr = r(dz)
    da2 = (dzr @ p["W3"]) * gelu_grad(a2)
    da2r = r(da2)
    da1 = (da2r @ p["W2"]) * gelu_grad(a1)
    da1r = r(da1)
    g = {}
    g["W3"] = np.abs(dzr).T @ np.abs(h2)
    g["b3"] = np.abs(dz).sum(axis=0)
    g["W2"] = np.abs(da2r).T @ np.abs(h1)
    g["b2"] = np.abs(da2).sum(axis=0)
    g["W1"] = np.abs(da1r).T @ np.abs(x)
    g["b1"] = np.abs(da1).sum(axis=0)
    dx = (np.abs(da1r) @ ab["W1"]).reshape(b, WINDOW, EMB)
    demb = np.zeros((257, EMB))
    np.add.at(demb, np.asarray(windows, dtype=np.int64), dx)
    g["emb"] = demb[:256]
    return zs, pack(g)


def adamw(flat, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8, wd=0.01):
    """One AdamW step (bias-corrected moments, decoupled weight decay)."""
    m = beta1 * m + (1 - beta1) * grad
    v = beta2 * v + (1 - beta2) * grad * grad
    mhat = m / (1 - beta1 ** step)
    vhat = v / (1 - beta2 ** step)
    flat = flat - lr * (mhat / (np.sqrt(vhat) + eps) + wd * flat)
    return flat, m, v


def bf16_round(a: np.ndarray) -> np.ndarray:
    """Round float32 values to the nearest bfloat16 (ties to even), returned
    as float32 — the rounding the GPU applies to bf16 operands."""
    f = np.ascontiguousarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u >> 16) & 1) + 0x7FFF
    out = ((u + r) >> 16 << 16).astype(np.uint32)
    return out.view(np.float32)


def topm(logits: np.ndarray, allowed: np.ndarray, m: int) -> list:
    """Indices of the m largest logits among the allowed states, ties broken
    by the lower state id; fewer if fewer are allowed."""
    out = []
    for row, ok in zip(logits, allowed):
        ids = np.flatnonzero(ok)
        order = sorted(ids.tolist(), key=lambda s: (-float(row[s]), s))
        out.append(order[:m])
    return out
