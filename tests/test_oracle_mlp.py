"""Pins of the CPU oracle of the learned proposal (float64 MLP).

The MLP is not in the paper; its definition is fixed by the benchmark plan
(32-byte window, 16-d embeddings, two GELU layers of 256, one logit per
state, masked softmax cross-entropy, AdamW). These tests pin the oracle to
closed forms and to finite differences, never to itself.
"""
import math

import numpy as np
import pytest

from oracle import mlp
import workloads as W


def test_gelu_closed_forms():
    assert mlp.gelu(np.array([0.0]))[0] == 0.0
    # gelu(1) = Phi(1)
    assert abs(mlp.gelu(np.array([1.0]))[0] - 0.5 * (1 + math.erf(1 / math.sqrt(2)))) < 1e-15
    assert abs(mlp.gelu(np.array([1.0]))[0] - 0.8413447460685429) < 1e-12
    x = np.linspace(-5, 5, 41)
    # gelu(-x) = gelu(x) - x
    assert np.allclose(mlp.gelu(-x), mlp.gelu(x) - x, atol=1e-14)
    # large arguments: identity and zero
    assert abs(mlp.gelu(np.array([30.0]))[0] - 30.0) < 1e-12
    assert abs(mlp.gelu(np.array([-30.0]))[0]) < 1e-12


def test_gelu_grad_finite_difference():
    x = np.linspace(-4, 4, 33)
    h = 1e-6
    fd = (mlp.gelu(x + h) - mlp.gelu(x - h)) / (2 * h)
    assert np.allclose(mlp.gelu_grad(x), fd, atol=1e-8)


def tiny_case(rng, states=7, batch=5):
    flat = W.mlp_init_params(states, seed=int(rng.integers(0, 1000))).astype(np.float64)
    flat += 0.01 * rng.standard_normal(flat.size)  # non-zero biases too
    windows = rng.integers(0, 256, size=(batch, 32), dtype=np.uint8)
    mask = rng.random((batch, states)) < 0.7
    labels = np.array([rng.choice(np.flatnonzero(m)) if m.any() else 0 for m in mask])
    for i, m in enumerate(mask):
        if not m.any():
            mask[i, 0] = True
    return flat, windows, mask, labels


def test_uniform_logits_loss_is_log_k():
    states = 6
    flat = np.zeros(mlp.param_count(states))
    windows = np.zeros((3, 32), dtype=np.uint8)
    mask = np.array([[1, 1, 1, 0, 0, 0], [1, 1, 1, 1, 1, 1], [0, 1, 0, 1, 0, 0]], dtype=bool)
    labels = np.array([2, 5, 3])
    loss, grad = mlp.loss_and_grad(flat, states, windows, mask, labels)
    assert abs(loss - np.mean([math.log(3), math.log(6), math.log(2)])) < 1e-12


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(0)
    flat, windows, mask, labels = tiny_case(rng)
    states = 7
    _, g = mlp.loss_and_grad(flat, states, windows, mask, labels)
    # probe coordinates in every tensor (the embedding rows actually used included)
    shapes = mlp.param_shapes(states)
    offsets = np.cumsum([0] + [int(np.prod(s)) for _, s in shapes])
    picks = []
    for t in range(len(shapes)):
        picks += list(rng.integers(offsets[t], offsets[t + 1], size=6))
    used = int(windows[0, 0])
    picks += [used * 16 + d for d in range(4)]
    h = 1e-6
    for k in picks:
        e = np.zeros_like(flat)
        e[k] = h
        lp, _ = mlp.loss_and_grad(flat + e, states, windows, mask, labels)
        lm, _ = mlp.loss_and_grad(flat - e, states, windows, mask, labels)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[k]) <= 1e-7 + 1e-5 * abs(fd), (k, fd, g[k])


def test_softmax_gradient_rows_sum_to_zero():
    rng = np.random.default_rng(1)
    flat, windows, mask, labels = tiny_case(rng, batch=9)
    _, g = mlp.loss_and_grad(flat, 7, windows, mask, labels)
    # d loss / d b3 = sum over rows of (prob - onehot) / B, and each row sums to 0
    b3 = mlp.unpack(g, 7)["b3"]
    assert abs(b3.sum()) < 1e-12


def test_topm_ties_prefer_lower_ids():
    logits = np.array([[1.0, 3.0, 3.0, 2.0, 3.0]])
    allowed = np.array([[True, True, False, True, True]])
    assert mlp.topm(logits, allowed, 2) == [[1, 4]]
    assert mlp.topm(logits, allowed, 9) == [[1, 4, 3, 0]]


def test_adamw_first_step_closed_form():
    flat = np.array([1.0, -2.0, 0.5])
    grad = np.array([0.3, -0.1, 0.0])
    m = np.zeros(3)
    v = np.zeros(3)
    new, m, v = mlp.adamw(flat, grad, m, v, step=1, lr=0.01, eps=1e-12, wd=0.1)
    # step 1: mhat = g, vhat = g^2 -> update = lr * (sign(g) + wd * w)
    want = flat - 0.01 * (np.sign(grad) + 0.1 * flat)
    assert np.allclose(new, want, atol=1e-9)


def test_bf16_round_ties_to_even():
    x = np.array([1.0, 1.00390625, 1.01171875, 3.140625, -2.0000002], dtype=np.float32)
    r = mlp.bf16_round(x)
    # 1 + 2^-8 is halfway between 1 and 1 + 2^-7: ties to even -> 1
    assert r[0] == 1.0 and r[1] == 1.0
    # 1 + 3*2^-8 halfway between 1+2^-7 and 1+2^-6: even mantissa -> 1 + 2^-6
    assert r[2] == np.float32(1.015625)
    assert r[3] == np.float32(3.140625)
    assert r[4] == np.float32(-2.0)


def test_param_count_of_the_planned_network():
    # 4096 head rows: 4096 + 131328 + 65792 + 1052672
    assert mlp.param_count(4096) == 1253888
    assert W.mlp_init_params(35).size == mlp.param_count(35)


def test_pad_bytes_embed_as_zero_and_get_no_gradient():
    rng = np.random.default_rng(6)
    flat, windows, mask, labels = tiny_case(rng)
    w = windows.astype(np.int64)
    w[:, :5] = mlp.PAD
    z_pad, _ = mlp.forward(flat, 7, w, mask)
    # same as zeroing those embedding inputs: replace the pad by a byte whose
    # embedding row is set to zero
    p = mlp.unpack(flat.copy(), 7)
    p["emb"][0] = 0.0
    w0 = w.copy()
    w0[w0 == mlp.PAD] = 0
    z0, _ = mlp.forward(mlp.pack(p), 7, w0, mask)
    assert np.allclose(z_pad, z0)
    loss, g = mlp.loss_and_grad(flat, 7, w, mask, labels)
    assert np.all(np.isfinite(g))


def test_rounded_operands_stay_near_the_exact_definition():
    """The bf16-operand variant differs from the exact definition only by
    operand rounding (each rounding moves a value by at most 2^-8 of itself);
    its gradient stays within a few percent of the exact one in norm, and
    every entry's scale bounds the entry (triangle inequality)."""
    rng = np.random.default_rng(12)
    flat, windows, mask, labels = tiny_case(rng, states=9, batch=40)
    zs, gs = mlp.magnitudes(flat, 9, windows, mask, labels, rnd=mlp.bf16_round)
    l0, g0 = mlp.loss_and_grad(flat, 9, windows, mask, labels)
    l1, g1 = mlp.loss_and_grad(flat, 9, windows, mask, labels, rnd=mlp.bf16_round)
    assert np.all(np.abs(g1) <= gs * (1 + 1e-12) + 1e-300)
    for k in ("emb", "W1", "b1", "W2", "b2", "W3", "b3"):
        a, b = mlp.unpack(g1, 9)[k], mlp.unpack(g0, 9)[k]
        assert np.linalg.norm(a - b) <= 0.05 * np.linalg.norm(b), k
    z0, _ = mlp.forward(flat, 9, windows, mask)
    z1, _ = mlp.forward(flat, 9, windows, mask, rnd=mlp.bf16_round)
    ok = np.isfinite(z0)
    assert np.all(np.abs(z1)[ok] <= zs[ok] * (1 + 1e-12))
    # the head's operand h2 carries the rounding of two layers
    assert np.all(np.abs(z1 - z0)[ok] <= 4 * 2.0 ** -8 * zs[ok])
    assert abs(l1 - l0) <= 0.05 * abs(l0)
    # without a rounding function the variant is the exact definition
    l2, g2 = mlp.loss_and_grad(flat, 9, windows, mask, labels, rnd=None)
    assert l2 == l0 and np.array_equal(g2, g0)


def test_scale_exposes_a_dropped_column():
    """A planted mistake (the last embedding column's gradient dropped, or
    the bias of one hidden unit) is far outside the comparison bound the GPU
    gradient is held to (2^-10 of the entry's scale) for nearly every entry:
    the scale does not hide a wrong element."""
    rng = np.random.default_rng(13)
    flat, windows, mask, labels = tiny_case(rng, states=9, batch=40)
    _, gs = mlp.magnitudes(flat, 9, windows, mask, labels, rnd=mlp.bf16_round)
    _, g = mlp.loss_and_grad(flat, 9, windows, mask, labels, rnd=mlp.bf16_round)
    G, GS = mlp.unpack(g, 9), mlp.unpack(gs, 9)
    used = np.unique(windows)
    for k, sl in (("emb", (used, -1)), ("W1", (slice(None), 7)), ("W2", (3, slice(None))),
                  ("b1", (slice(None),)), ("W3", (2, slice(None)))):
        assert np.mean(np.abs(G[k][sl]) > 2.0 ** -10 * GS[k][sl]) > 0.9, k
