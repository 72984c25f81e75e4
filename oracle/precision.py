"""FP64 CPU oracle for the reduced-precision forms of the leaf products (test
infrastructure only: only the test suite may import this module).

The skip mask is the one of the FP32 inputs (Algorithm 1 on the norms of A and
B as given); only the leaf products change precision:

* ``bf16``: every element of A and B is rounded to bfloat16 (round to nearest,
  ties to even); C = sum over kept pairs of bf16(A_ik) bf16(B_kj), products
  exact.
* ``f16x3``: each matrix X gets one power-of-two scale s_X = 2^(15 - ceil(log2
  M_X)), M_X its largest leaf-tile Frobenius norm (so |s_X x| <= 2^15, inside
  the FP16 range); hi = fp16(s_X x), lo = fp16(s_X x - hi), both round to
  nearest even; C = (hiA hiB + hiA loB + loA hiB) / (s_A s_B) over the kept
  pairs, i.e. the product of (hi + lo) / s minus the dropped lo loB term.

The sums are the oracle's FP64 SpAMM (Algorithm 1) of the rounded operands.
"""

from __future__ import annotations

import math

import numpy as np

from . import pyramid, spamm_tiles, all_tiles, bdim

BF16, F16X3 = "bf16", "f16x3"


def bf16_round(x) -> np.ndarray:
    """float32 -> bfloat16 (round to nearest, ties to even), returned as float32."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    r = ((u + np.uint64(0x7FFF) + lsb) & np.uint64(0xFFFF0000)).astype(np.uint32)
    return r.view(np.float32)


def f16_scale_exponent(max_norm: float) -> int:
    """e with s = 2^e = 2^(15 - ceil(log2 max_norm)); 0 when max_norm is 0."""
    if max_norm <= 0.0:
        return 0
    f, x = math.frexp(max_norm)  # max_norm = f 2^x, f in [0.5, 1)
    ceil_log2 = x - 1 if f == 0.5 else x
    return 15 - ceil_log2


def f16_split(x, e: int):
    """(hi, lo) as float32 arrays holding FP16 values of s x, s = 2^e."""
    y = np.ldexp(np.asarray(x, dtype=np.float64), e)  # exact
    hi = y.astype(np.float16)
    lo = (y - hi.astype(np.float64)).astype(np.float16)
    return hi.astype(np.float32), lo.astype(np.float32)


def max_leaf_norm(x, leaf: int) -> float:
    b = bdim(np.asarray(x).shape[0], leaf)
    return float(np.max(pyramid(x, leaf)[-1][:b, :b]))


def spamm_precision(a, b, tau: float, leaf: int, precision: str):
    """C (FP64, N x N) of the reduced-precision form, with the FP32 inputs' mask."""
    a = np.ascontiguousarray(a, dtype=np.float32)
    b = np.ascontiguousarray(b, dtype=np.float32)
    n = a.shape[0]
    pa, pb = pyramid(a, leaf), pyramid(b, leaf)
    tiles = all_tiles(n, leaf)
    bd = bdim(n, leaf)

    def run(x, y):
        ct, counts, _ = spamm_tiles(x, y, tau, leaf, tiles, pyr_a=pa, pyr_b=pb)
        p = bd * leaf
        full = ct.reshape(bd, bd, leaf, leaf).transpose(0, 2, 1, 3).reshape(p, p)
        return np.ascontiguousarray(full[:n, :n]), int(counts.sum())

    if precision == BF16:
        return run(bf16_round(a), bf16_round(b))
    if precision != F16X3:
        raise ValueError(precision)
    ea, eb = f16_scale_exponent(float(np.max(pa[-1]))), f16_scale_exponent(float(np.max(pb[-1])))
    ha, la = f16_split(a, ea)
    hb, lb = f16_split(b, eb)
    # (hi + lo) is exact in FP32 (at most 22 significant bits); rescale exactly
    qa = np.ldexp((ha.astype(np.float64) + la), -ea).astype(np.float32)
    qb = np.ldexp((hb.astype(np.float64) + lb), -eb).astype(np.float32)
    full, pairs = run(qa, qb)
    lolo, _ = run(np.ldexp(la.astype(np.float64), -ea).astype(np.float32),
                  np.ldexp(lb.astype(np.float64), -eb).astype(np.float32))
    return full - lolo, pairs
