"""Pins of the reduced-precision oracle (oracle/precision.py): rounding against
library conversions (torch's bfloat16 and float16 casts, Python's IEEE half
packing), the scale's closed form, exactness on integer-valued inputs, the
rounding-error bounds of each form, and a pure-Python brute force of the
three-product FP16 form on a tiny problem."""

from __future__ import annotations

import math
import struct

import numpy as np
import pytest
import torch

import oracle
from oracle import precision as pr
from paper_2103_13042_amd import inputs


def _values(seed, count=4000):
    rng = np.random.default_rng(seed)
    v = rng.standard_normal(count) * 10.0 ** rng.uniform(-30, 30, count)
    ties = np.array([1 + 2**-8, 1 + 3 * 2**-8, -(1 + 2**-8), 2**-130, -3.0e-40, 1.0, 0.0, 65504.0, 3.4e38],
                    dtype=np.float64)
    return np.concatenate([v, ties]).astype(np.float32)


def test_bf16_round_matches_torch_cast():
    x = _values(1)
    want = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(pr.bf16_round(x).view(np.uint32), want.view(np.uint32))
    # ties to even
    assert pr.bf16_round(np.float32([1 + 2**-8]))[0] == 1.0
    assert pr.bf16_round(np.float32([1 + 3 * 2**-8]))[0] == np.float32(1 + 2**-6)


@pytest.mark.parametrize("m,e", [(1.0, 15), (1.5, 14), (2.0, 14), (2.0000002, 13), (0.75, 15), (0.5, 16),
                                 (3e-9, 43), (0.0, 0)])
def test_scale_exponent_closed_form(m, e):
    assert pr.f16_scale_exponent(m) == e
    if m > 0:
        assert m * 2.0**e <= 2.0**15 < 2 * m * 2.0**e


def test_f16_split_matches_half_casts_and_bound():
    x = (np.random.default_rng(2).standard_normal(5000) * 10.0 ** np.random.default_rng(3).uniform(-6, 0, 5000)
         ).astype(np.float32)
    e = 12
    hi, lo = pr.f16_split(x, e)
    y = (x * np.float32(2.0**e)).astype(np.float32)  # exact
    want_hi = torch.from_numpy(y).to(torch.float16).to(torch.float32).numpy()
    assert np.array_equal(hi, want_hi)
    want_lo = torch.from_numpy((y - want_hi).astype(np.float32)).to(torch.float16).to(torch.float32).numpy()
    assert np.array_equal(lo, want_lo)
    # |y - (hi + lo)| <= 2^-22 |y| while lo is a normal half, else half the
    # subnormal spacing (2^-25)
    err = np.abs(y.astype(np.float64) - hi - lo)
    assert np.all(err <= np.maximum(2.0**-22 * np.abs(y), 2.0**-25))


@pytest.mark.parametrize("precision", [pr.BF16, pr.F16X3])
def test_integer_inputs_are_exact(precision):
    rng = np.random.default_rng(4)
    n, leaf = 70, 16
    a = rng.integers(-64, 65, size=(n, n)).astype(np.float32)
    b = rng.integers(-64, 65, size=(n, n)).astype(np.float32)
    a[:, 40:] *= 0.0  # some empty tiles
    for tau in (0.0, 500.0, 3000.0):
        c, pairs = pr.spamm_precision(a, b, tau, leaf, precision)
        c64, pairs64, _ = oracle.spamm(a, b, tau, leaf)
        assert pairs == pairs64 and np.array_equal(c, c64)


def _kept_abs(a, b, tau, leaf):
    c, _, _ = oracle.spamm(np.abs(a), np.abs(b), tau, leaf)
    return c


@pytest.mark.parametrize("n,leaf,tau", [(256, 32, 1e-6), (200, 64, 1e-3), (128, 32, 0.0)])
def test_rounding_bounds(n, leaf, tau):
    a, b = inputs.exp_decay(n, 0.05, 30), inputs.algebraic_decay_signed(n, 31)
    c64, pairs64, _ = oracle.spamm(a, b, tau, leaf)
    ab = _kept_abs(a, b, tau, leaf)
    gam = 2 * n * 2.0**-53  # FP64 summation slack on both sides
    cb, pairs = pr.spamm_precision(a, b, tau, leaf, pr.BF16)
    assert pairs == pairs64
    u = 2.0**-8
    assert np.all(np.abs(cb - c64) <= (2 * u + u * u + gam) * ab + 1e-300)
    cf, pairs = pr.spamm_precision(a, b, tau, leaf, pr.F16X3)
    assert pairs == pairs64
    sa = 2.0 ** pr.f16_scale_exponent(pr.max_leaf_norm(a, leaf))
    sb = 2.0 ** pr.f16_scale_exponent(pr.max_leaf_norm(b, leaf))
    # per product: 4 * 2^-22 relative, plus the subnormal-lo absolute term of each operand
    absb = n * (np.max(np.abs(a)) * 2.0**-25 / sb + np.max(np.abs(b)) * 2.0**-25 / sa)
    assert np.all(np.abs(cf - c64) <= (4 * 2.0**-22 + gam) * ab + absb)
    assert np.linalg.norm(cf - c64) <= 1e-6 * np.linalg.norm(c64)


def _half(v: float) -> float:
    return struct.unpack("<e", struct.pack("<e", v))[0]  # IEEE half, round to nearest even


def test_three_product_form_brute_force():
    # 4 x 4 with 2 x 2 leaves, tau = 0: every pair kept; pure Python with the
    # struct module's half rounding
    rng = np.random.default_rng(5)
    a = (rng.standard_normal((4, 4)) * 0.37).astype(np.float32)
    b = (rng.standard_normal((4, 4)) * 1.9).astype(np.float32)
    c, _ = pr.spamm_precision(a, b, 0.0, 2, pr.F16X3)

    def split(x):
        m = max(math.sqrt(sum(float(x[2 * i + r, 2 * j + q]) ** 2 for r in range(2) for q in range(2)))
                for i in range(2) for j in range(2))
        f, ex = math.frexp(m)
        e = 15 - (ex - 1 if f == 0.5 else ex)
        s = 2.0**e
        hi = [[_half(float(x[i, j]) * s) for j in range(4)] for i in range(4)]
        lo = [[_half(float(x[i, j]) * s - hi[i][j]) for j in range(4)] for i in range(4)]
        return hi, lo, s

    ha, la, sa = split(a)
    hb, lb, sb = split(b)
    for i in range(4):
        for j in range(4):
            v = sum(ha[i][k] * hb[k][j] + ha[i][k] * lb[k][j] + la[i][k] * hb[k][j] for k in range(4))
            assert c[i, j] == pytest.approx(v / (sa * sb), rel=1e-15, abs=1e-300)
