"""The largest tile grids the GPU path accepts, checked against a closed form.

The library takes at most 1024 tiles per side (512 on the leaf-128 macro-tile
path); at that size the packed schedule items of the macro-tile multiply use
every value of their macro-row, macro-column and k fields.

Closed form: A = I and B = the exchange matrix (ones on the anti-diagonal).  The
only nonzero leaf tiles are A's diagonal tiles and B's anti-diagonal tiles
(k, bdim-1-k), each holding `leaf` ones, so each has Frobenius norm sqrt(leaf)
(Eq. 2) and every nonzero norm product equals leaf.  With tau slightly below
leaf exactly the bdim triples (i, i, bdim-1-i) survive the test of Algorithm 1,
every kept tile product is exact in FP32, and C = A B = B bitwise.  With tau
slightly above leaf nothing survives and C = 0.  The margins (1e-9 relative)
are far outside FP64 rounding of the norm product.
"""

from __future__ import annotations

import pytest
import torch

from paper_2103_13042_amd import binding as sp

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda", 0)


@pytest.mark.parametrize("n,leaf", [(65536, 64), (32768, 32), (65536, 128)])
def test_largest_tile_grid_identity_times_exchange(n, leaf):
    bdim = n // leaf
    need = sp.workspace_bytes(n, leaf)
    assert need > 0
    if leaf != 128:
        assert bdim == 1024 and sp.workspace_bytes(n + leaf, leaf) == 0
    print(f"largest grid: n={n} leaf={leaf} bdim={bdim}", flush=True)
    torch.cuda.empty_cache()
    idx = torch.arange(n, device=DEV)
    a = torch.zeros((n, n), dtype=torch.float32, device=DEV)
    a[idx, idx] = 1.0
    b = torch.zeros_like(a)
    b[idx, n - 1 - idx] = 1.0
    ws = torch.empty(need, dtype=torch.uint8, device=DEV)
    try:
        c, pairs = sp.multiply(a, b, leaf * (1.0 - 1e-9), leaf, ws=ws)
        assert pairs == bdim
        assert torch.equal(c, b)
        c, pairs = sp.multiply(a, b, leaf * (1.0 + 1e-9), leaf, c=c, ws=ws)
        assert pairs == 0
        assert not bool(c.any())
    finally:
        del a, b, ws
        torch.cuda.empty_cache()
