"""Threshold selection on the GPU (through the C ABI) against the FP64 oracle.

Bars:
  - features: bitwise equal to the oracle's rounded to FP32 (both divide
    integer counts in FP64; inputs are checked to have no leaf norm within
    1e-9 of a bin edge, where the two log10 implementations could disagree);
  - network forward: |y - y_oracle| <= 1e-5 * max(1, max|y_oracle|) (FP32
    sums of 129 and 128 terms; erf in FP32);
  - loss gradient: per parameter tensor, max deviation <= 1e-4 of the tensor's
    largest oracle entry; loss within 1e-5 relative;
  - Adam: one step within the FP32 rounding bounds of the oracle's step;
  - sums of squares: 1e-13 relative (exact FP64 squares, another order);
  - relative error of SpAMM at tau: 1e-5 relative (E formed in FP32 from the
    dropped pairs only, ||AB|| from the tau = 0 product);
  - threshold search: the oracle's brute-force label, to 1e-12 relative (both
    are leaf norm products), for targets not within 1e-4 relative of the error
    at any product.
"""

from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle
from oracle import learned
from paper_2103_13042_amd import binding as sp
from paper_2103_13042_amd import inputs

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda", 0)


def gpu(x, dtype=torch.float32) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(x)).to(dtype).to(DEV)


def _batch(nb, seed):
    rng = np.random.default_rng(seed)
    x = np.concatenate([rng.dirichlet(np.ones(64), size=nb), rng.dirichlet(np.ones(64), size=nb),
                        rng.uniform(-6, -2, size=(nb, 1))], axis=1).astype(np.float32)
    t = rng.uniform(-4, 0, size=nb).astype(np.float32)
    return x, t


@pytest.mark.parametrize("n,leaf,alpha", [(1024, 32, 0.05), (2048, 64, 0.3), (1000, 32, 0.01), (512, 64, 0.5)])
def test_features_match_oracle(n, leaf, alpha):
    a, b = inputs.exp_decay(n, alpha, 70), inputs.exp_decay(n, alpha * 0.7, 71)
    for x in (a, b):
        pos = learned.bin_position(oracle.leaf_norms(x, leaf))
        assert np.all(np.abs(pos - np.round(pos)) > 1e-9), "a leaf norm sits on a bin edge"
    target = 3.7e-5
    want = learned.features(a, b, leaf, target).astype(np.float32)
    pa, pb = sp.pyramid(gpu(a), leaf), sp.pyramid(gpu(b), leaf)
    got = sp.tau_features(pa, pb, n, leaf, target).cpu().numpy()
    assert np.array_equal(got, want)


def test_forward_matches_oracle():
    params = inputs.mlp_init(5)
    x, _ = _batch(300, 3)
    y_ref, _ = learned.forward(params.astype(np.float64), x.astype(np.float64))
    y = sp.mlp_forward(gpu(params), gpu(x)).cpu().numpy()
    assert np.max(np.abs(y - y_ref)) <= 1e-5 * max(1.0, np.max(np.abs(y_ref)))


@pytest.mark.parametrize("batch,scale", [(256, 1.0), (37, 3.0), (1, 1.0)])
def test_loss_gradient_matches_oracle(batch, scale):
    params = inputs.mlp_init(6) * np.float32(scale)
    x, t = _batch(batch, 4)
    loss_ref, g_ref = learned.loss_and_grad(params.astype(np.float64), x.astype(np.float64), t.astype(np.float64))
    loss, g = sp.mlp_loss_grad(gpu(params), gpu(x), gpu(t))
    assert float(loss.item()) == pytest.approx(loss_ref, rel=1e-5)
    g = g.cpu().numpy().astype(np.float64)
    got, ref = learned.unpack(g), learned.unpack(g_ref)
    for name in ref:
        bound = 1e-4 * max(np.max(np.abs(ref[name])), 1e-30)
        assert np.max(np.abs(got[name] - ref[name])) <= bound, name


def test_adam_step_matches_oracle():
    rng = np.random.default_rng(8)
    p0 = inputs.mlp_init(7)
    g = rng.normal(size=p0.size).astype(np.float32) * 1e-2
    m0 = rng.normal(size=p0.size).astype(np.float32) * 1e-3
    v0 = np.abs(rng.normal(size=p0.size)).astype(np.float32) * 1e-5
    # the entry point takes FP32 hyper-parameters: give the oracle the same values
    b1, b2, lr, eps = (float(np.float32(v)) for v in (0.9, 0.999, 1e-3, 1e-8))
    want, m1, v1 = learned.adam_step(p0.astype(np.float64), g.astype(np.float64), m0.astype(np.float64),
                                     v0.astype(np.float64), 3, lr, b1, b2, eps)
    p, gm, gv = gpu(p0), gpu(m0), gpu(v0)
    sp.mlp_adam(p, gpu(g), gm, gv, 3, lr, b1, b2, eps)
    # FP32 rounding bounds, u = 2^-24 (1 - b1 and 1 - b2 are exact in FP32):
    # the moments are two-term sums (m can cancel); the update divides
    # m / (1 - b1^3) by sqrt(v / (1 - b2^3)) + eps
    u = 2.0**-24
    g64, m64, v64 = g.astype(np.float64), m0.astype(np.float64), v0.astype(np.float64)
    dm = 3 * u * (b1 * np.abs(m64) + (1 - b1) * np.abs(g64))
    dv = 4 * u * (b2 * v64 + (1 - b2) * g64 * g64)
    assert np.all(np.abs(gm.cpu().numpy() - m1) <= dm)
    assert np.all(np.abs(gv.cpu().numpy() - v1) <= dv)
    c1, c2 = 1 - b1**3, 1 - b2**3
    den = np.sqrt(v1 / c2) + eps
    dden = (0.5 * (dv / np.maximum(v1, 1e-300) + 2 * u) + u) * np.sqrt(v1 / c2) + u * den
    mh = np.abs(m1) / c1
    dp = 2 * u * np.abs(p0) + lr * ((dm / c1 + 2 * u * mh) / den + mh * dden / den**2) * (1 + 1e-6) \
        + 2 * u * lr * mh / den
    assert np.all(np.abs(p.cpu().numpy() - want) <= dp)


def test_training_steps_follow_the_oracle():
    params = inputs.mlp_init(9)
    x, _ = _batch(128, 5)
    t = (0.5 * x[:, 128] - 20.0 * x[:, :8].sum(axis=1) + 1.0).astype(np.float32)
    ref = params.astype(np.float64)
    m_r, v_r = np.zeros_like(ref), np.zeros_like(ref)
    p, m, v = gpu(params), torch.zeros(params.size, device=DEV), torch.zeros(params.size, device=DEV)
    gx, gt = gpu(x), gpu(t)
    for step in range(1, 21):
        loss_r, g_r = learned.loss_and_grad(ref, x.astype(np.float64), t.astype(np.float64))
        ref, m_r, v_r = learned.adam_step(ref, g_r, m_r, v_r, step, 1e-3)
        loss, g = sp.mlp_loss_grad(p, gx, gt)
        sp.mlp_adam(p, g, m, v, step, 1e-3)
        assert float(loss.item()) == pytest.approx(loss_r, rel=1e-2)
    final_r = learned.loss_and_grad(ref, x.astype(np.float64), t.astype(np.float64))[0]
    final = float(sp.mlp_loss_grad(p, gx, gt)[0].item())
    assert final == pytest.approx(final_r, rel=2e-2)


@pytest.mark.parametrize("count", [0, 1, 7, 1000, 1 << 20, 12345677])
def test_sumsq_matches_numpy(count):
    x = np.random.default_rng(count).normal(size=count).astype(np.float32)
    got = float(sp.sumsq(gpu(x)).item())
    want = float(np.sum(x.astype(np.float64) ** 2))
    assert got == pytest.approx(want, rel=1e-13, abs=0.0)
    # an unaligned start takes the scalar path
    if count > 1:
        gx = gpu(x)
        got1 = float(sp.sumsq(gx[1:]).item())
        assert got1 == pytest.approx(float(np.sum(x[1:].astype(np.float64) ** 2)), rel=1e-13)


def _problem(n, leaf, alpha_a, alpha_b, seed):
    a, b = inputs.exp_decay(n, alpha_a, seed), inputs.exp_decay(n, alpha_b, seed + 1)
    ga, gb = gpu(a), gpu(b)
    c0, _ = sp.multiply(ga, gb, 0.0, leaf)
    ab_sq = float(sp.sumsq(c0).item())
    return a, b, ga, gb, sp.pyramid(ga, leaf), sp.pyramid(gb, leaf), ab_sq


@pytest.mark.parametrize("n,leaf", [(256, 32), (300, 32), (512, 64)])
def test_error_for_tau_matches_oracle(n, leaf):
    a, b, ga, gb, pa, pb, ab_sq = _problem(n, leaf, 0.2, 0.1, 80)
    na, nb = oracle.leaf_norms(a, leaf), oracle.leaf_norms(b, leaf)
    prods = np.unique((na[:, :, None] * nb[None, :, :]).ravel())
    bd = oracle.bdim(n, leaf)
    for q in (0.2, 0.5, 0.8, 0.95):
        tau = float(np.sqrt(prods[int(q * len(prods))] * prods[int(q * len(prods)) - 1]))  # between two products
        err, dropped = sp.error_for_tau(ga, gb, tau, leaf, pa, pb, ab_sq)
        _, pairs, _ = oracle.spamm(a, b, tau, leaf, products=False)
        assert dropped == bd**3 - pairs
        assert err == pytest.approx(learned.rel_error(a, b, tau, leaf), rel=1e-5)
    err0, dropped0 = sp.error_for_tau(ga, gb, 0.0, leaf, pa, pb, ab_sq)
    assert err0 == 0.0 and dropped0 == 0


@pytest.mark.parametrize("n,leaf,alphas", [(128, 32, (0.3, 0.2)), (256, 32, (0.15, 0.25)), (256, 64, (0.05, 0.1))])
def test_search_matches_oracle_label(n, leaf, alphas):
    a, b, ga, gb, pa, pb, ab_sq = _problem(n, leaf, *alphas, 90)
    na, nb = oracle.leaf_norms(a, leaf), oracle.leaf_norms(b, leaf)
    prods = np.unique((na[:, :, None] * nb[None, :, :]).ravel())
    errs = np.array([learned.rel_error(a, b, float(p), leaf) for p in prods])
    for target in (1e-6, 1e-4, 1e-3, 1e-2, 0.1):
        if np.any(np.abs(errs / target - 1.0) < 1e-4):
            continue  # the FP32 error could land either side of the target
        want = learned.label_tau(a, b, leaf, target)
        for guess in (0.0, want * 9.0, want / 13.0, 1e-30):
            tau, err, pairs, evals = sp.search_tau_for_error(ga, gb, leaf, target, pa, pb, ab_sq, guess=guess)
            assert tau == pytest.approx(want, rel=1e-12), (target, guess)
            assert err <= target and evals >= 1
            _, count, _ = oracle.spamm(a, b, want, leaf, products=False)
            assert pairs == count


def test_search_edge_cases():
    n, leaf = 256, 32
    a, b, ga, gb, pa, pb, ab_sq = _problem(n, leaf, 0.1, 0.1, 95)
    na, nb = oracle.leaf_norms(a, leaf), oracle.leaf_norms(b, leaf)
    pmax = float(np.max(na[:, :, None] * nb[None, :, :]))
    # a target of 1 or more is met by the largest product (only the top triples kept)
    tau, err, pairs, _ = sp.search_tau_for_error(ga, gb, leaf, 1.0, pa, pb, ab_sq)
    assert tau == pytest.approx(pmax, rel=1e-12) and err <= 1.0
    # the evaluation cap returns a passing product
    tau, err, _, evals = sp.search_tau_for_error(ga, gb, leaf, 1e-3, pa, pb, ab_sq, max_evals=2)
    assert evals == 2 and err <= 1e-3
    with pytest.raises(sp.SpammError):
        sp.search_tau_for_error(ga, gb, leaf, 0.0, pa, pb, ab_sq)
    with pytest.raises(sp.SpammError):
        sp.search_tau_for_error(ga, gb, leaf, 1e-3, pa, pb, 0.0)
