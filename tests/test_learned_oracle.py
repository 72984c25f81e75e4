"""Pins of the learned-threshold oracle (oracle/learned.py) against facts that
do not come from the oracle itself: printed values of the normal distribution,
brute force in pure Python, central finite differences, Adam's closed form
under a constant gradient, and brute-force threshold labels.
"""

from __future__ import annotations

import math

import numpy as np
import pytest

import oracle
from oracle import learned
from paper_2103_13042_amd import inputs


def test_gelu_is_the_erf_form():
    # GELU(x) = x * Phi(x); Phi(1) = 0.8413447460685429 and Phi(2) =
    # 0.9772498680518208 are the standard normal table values.  The tanh
    # approximation gives 0.841192 at 1 and fails this.
    assert learned.gelu(np.array(1.0)) == pytest.approx(0.8413447460685429, abs=1e-15)
    assert learned.gelu(np.array(2.0)) == pytest.approx(2 * 0.9772498680518208, abs=1e-15)
    assert learned.gelu(np.array(0.0)) == 0.0
    x = np.linspace(-6, 6, 97)
    # Phi(x) + Phi(-x) = 1  =>  GELU(x) - GELU(-x) = x
    assert np.allclose(learned.gelu(x) - learned.gelu(-x), x, rtol=0, atol=1e-14)
    h = 1e-6
    fd = (learned.gelu(x + h) - learned.gelu(x - h)) / (2 * h)
    assert np.allclose(learned.gelu_grad(x), fd, rtol=0, atol=1e-9)
    assert learned.gelu_grad(np.array(0.0)) == pytest.approx(0.5, abs=1e-15)


def test_parameter_count_and_layout():
    assert learned.N_PARAMS == 33281  # 129*128 + 128 + 128*128 + 128 + 128 + 1
    flat = np.arange(learned.N_PARAMS, dtype=np.float64)
    p = learned.unpack(flat)
    assert p["W1"][1, 0] == 129 and p["b1"][0] == 128 * 129 and p["b3"][0] == learned.N_PARAMS - 1
    assert np.array_equal(learned.pack(p), flat)


def _hist_brute(norms, rows):
    counts = [0] * 64
    for v in np.asarray(norms, dtype=np.float64).ravel().tolist():
        if v <= 0.0:
            continue  # zero norms are not counted
        t = (math.log10(v) + 46.0) * 64.0 / 49.0
        counts[min(63, max(0, math.floor(t)))] += 1
    return [min(c / rows, 4.0) for c in counts]


def test_histogram_brute_force():
    rng = np.random.default_rng(3)
    vals = np.concatenate([10.0 ** rng.uniform(-50, 6, size=500), [0.0, 0.0, 1e-300, 5e3, 1.0]])
    h = learned.histogram(vals, 100)
    assert np.allclose(h, _hist_brute(vals, 100), rtol=0, atol=1e-15)
    assert h.sum() == pytest.approx(503 / 100, abs=1e-12)  # the positive values, per row, none capped
    assert np.allclose(learned.histogram(vals, 2), _hist_brute(vals, 2), rtol=0, atol=1e-15)
    assert learned.histogram(vals, 2).max() == 4.0  # capped
    # leaf norms of an actual decay matrix
    a = inputs.exp_decay(256, 0.3, 5)
    na = oracle.leaf_norms(a, 16)
    assert np.allclose(learned.histogram(na, 16), _hist_brute(na, 16), rtol=0, atol=1e-15)


def test_histogram_is_size_invariant_for_a_band():
    # a matrix that is a pure band (|i-j| < 2.5 tiles, equal values): the
    # histogram per tile row only moves by the band's truncated rows at the
    # edges, which shrink like 1/bdim
    def band(n):
        i = np.arange(n)
        return (np.abs(i[:, None] - i[None, :]) < 2 * 32 + 16).astype(np.float32)

    h1 = learned.histogram(oracle.leaf_norms(band(1024), 32), 32)
    h2 = learned.histogram(oracle.leaf_norms(band(4096), 32), 128)
    assert np.count_nonzero(h1) == np.count_nonzero(h2) >= 1
    assert np.allclose(h1, h2, rtol=0, atol=5.0 / 32)


def _forward_brute(flat, x):
    p = learned.unpack(flat)

    def g(v):
        return 0.5 * v * (1.0 + math.erf(v / math.sqrt(2.0)))

    out = []
    for row in np.asarray(x, dtype=np.float64).tolist():
        h1 = [g(sum(p["W1"][o, i] * row[i] for i in range(129)) + p["b1"][o]) for o in range(128)]
        h2 = [g(sum(p["W2"][o, i] * h1[i] for i in range(128)) + p["b2"][o]) for o in range(128)]
        out.append(sum(p["w3"][i] * h2[i] for i in range(128)) + p["b3"][0])
    return np.array(out)


def _batch(nb, seed):
    rng = np.random.default_rng(seed)
    x = np.concatenate([rng.dirichlet(np.ones(64), size=nb), rng.dirichlet(np.ones(64), size=nb),
                        rng.uniform(-6, -2, size=(nb, 1))], axis=1)
    t = rng.uniform(-4, 0, size=nb)
    return x, t


def test_forward_brute_force():
    flat = inputs.mlp_init(1).astype(np.float64)
    x, _ = _batch(3, 0)
    y, _ = learned.forward(flat, x)
    assert np.allclose(y, _forward_brute(flat, x), rtol=1e-12, atol=1e-13)


def test_gradient_matches_central_differences():
    flat = inputs.mlp_init(2).astype(np.float64) * 3.0  # larger weights: GELU's curvature matters
    x, t = _batch(5, 1)
    _, g = learned.loss_and_grad(flat, x, t)
    rng = np.random.default_rng(4)
    # every bias, the whole output layer, and a sample of each weight matrix
    idx = np.concatenate([np.arange(128 * 129, 128 * 130), np.arange(128 * 130 + 128 * 128, learned.N_PARAMS),
                          rng.choice(128 * 129, 300, replace=False),
                          128 * 130 + rng.choice(128 * 128, 300, replace=False)])
    h = 1e-6
    for k in idx:
        e = np.zeros_like(flat)
        e[k] = h
        fd = (learned.loss_and_grad(flat + e, x, t)[0] - learned.loss_and_grad(flat - e, x, t)[0]) / (2 * h)
        assert abs(fd - g[k]) <= 1e-7 * max(1.0, abs(g[k])), (k, fd, g[k])


def test_adam_constant_gradient_closed_form():
    # With a constant gradient g the bias-corrected moments equal g and g^2 at
    # every step, so after t steps each parameter has moved by t*lr*g/(|g|+eps).
    rng = np.random.default_rng(5)
    p0 = rng.normal(size=50)
    g = rng.normal(size=50)
    g[0] = 0.0
    p, m, v = p0.copy(), np.zeros(50), np.zeros(50)
    lr, eps = 1e-3, 1e-8
    for step in range(1, 8):
        p, m, v = learned.adam_step(p, g, m, v, step, lr, 0.9, 0.999, eps)
        assert np.allclose(p, p0 - step * lr * g / (np.abs(g) + eps), rtol=0, atol=1e-15)
    assert p[0] == p0[0]


def test_training_reduces_the_loss():
    # a smooth target of the features: the loss must fall by 20x
    flat = inputs.mlp_init(3).astype(np.float64)
    x, _ = _batch(64, 2)
    t = 0.5 * x[:, 128] - 20.0 * x[:, :8].sum(axis=1) + 1.0
    m, v = np.zeros_like(flat), np.zeros_like(flat)
    first = learned.loss_and_grad(flat, x, t)[0]
    for step in range(1, 301):
        loss, g = learned.loss_and_grad(flat, x, t)
        flat, m, v = learned.adam_step(flat, g, m, v, step, 3e-3)
    assert loss < 0.05 * first, (loss, first)


def test_label_is_the_largest_product_meeting_the_target():
    n, leaf = 64, 8
    a, b = inputs.exp_decay(n, 0.2, 60), inputs.exp_decay(n, 0.15, 61)
    na, nb = oracle.leaf_norms(a, leaf), oracle.leaf_norms(b, leaf)
    prods = np.unique((na[:, :, None] * nb[None, :, :]).ravel())
    for target in (1e-6, 1e-4, 1e-2, 0.3):
        tau = learned.label_tau(a, b, leaf, target)
        assert tau in prods
        assert learned.rel_error(a, b, tau, leaf) <= target
        above = prods[prods > tau]
        if above.size:
            # the next product up drops one more triple and misses the target
            assert learned.rel_error(a, b, float(above[0]), leaf) > target
        # positive entries: the error never decreases as tau grows
        errs = [learned.rel_error(a, b, float(p), leaf) for p in prods[:: max(1, prods.size // 25)]]
        assert all(e1 <= e2 + 1e-15 for e1, e2 in zip(errs, errs[1:]))
    # an error target of 1 or more allows dropping everything but the top product
    assert learned.label_tau(a, b, leaf, 1.0) == prods[-1]
