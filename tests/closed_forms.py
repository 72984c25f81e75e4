"""Closed forms used as independent pins (no oracle code, no HIP code)."""

from __future__ import annotations

import numpy as np


def toeplitz_tile_norm(d: np.ndarray, leaf: int, power: float = 2.0) -> np.ndarray:
    """Frobenius norm of the leaf tile at tile offset d (column tile - row tile)
    of |A_ij| = 1/(1+|i-j|)^power: the in-tile offsets m = c - r take each value
    with multiplicity leaf - |m|."""
    m = np.arange(-(leaf - 1), leaf, dtype=np.float64)
    w = leaf - np.abs(m)
    dist = np.abs(d[:, None].astype(np.float64) * leaf + m[None, :])
    return np.sqrt((w[None, :] / (1.0 + dist) ** (2 * power)).sum(axis=1))


def closed_form_pair_count(n: int, leaf: int, tau: float) -> tuple[int, float]:
    """Number of kept triples (i,k,j) for the algebraic-decay workload, with the
    smallest relative distance of any product from tau."""
    bd = n // leaf
    d = np.arange(-(bd - 1), bd)
    nrm = toeplitz_tile_norm(d, leaf)
    prod = nrm[:, None] * nrm[None, :]  # [d1 = k - i, d2 = j - k]
    d1, d2 = np.meshgrid(d, d, indexing="ij")
    lo = np.maximum.reduce([np.zeros_like(d1), d1, -d2])
    hi = np.minimum.reduce([np.full_like(d1, bd), bd + d1, bd - d2])
    mult = np.maximum(0, hi - lo)
    keep = prod >= tau
    gap = float(np.min(np.abs(prod[mult > 0] / tau - 1.0)))
    return int(mult[keep].sum()), gap
