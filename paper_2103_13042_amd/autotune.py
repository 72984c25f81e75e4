"""Leaf-size tuner for batches of products.

The leaf edge is part of a SpAMM problem (it decides which tile pairs are
tested and kept), so the tuner does not change a product behind the caller's
back: it proposes a leaf per product from measured speed, the caller adopts it
as part of the problem, and results are checked at the chosen leaf.

``tune`` times the batched path itself (spamm_batch_run, every stage) for
each candidate leaf on a batch of copies of one exponential-decay pair per
(size, decay-rate) bucket; a bucket keeps the default leaf unless another is
faster by more than ``MARGIN`` (so timing noise does not flip the choice).
Buckets are keyed on what the library measures of a product, not on how it
was generated: its size and its density, the fraction of leaf-32 tile
triples the plan keeps at the product's tau (``density``: norm pass, pyramid
and plan at leaf 32, pairs / bdim^3).  ``choose`` maps a product to the
nearest bucket in (log n, log density).  The table of the last tuning run is
kept in ``data/leaf_table.json`` so that the same batch gets the same leaves
from run to run.
"""

from __future__ import annotations

import json
import math
from pathlib import Path

import numpy as np
import torch

from . import binding as sp
from . import inputs

SIZES = (256, 512, 1024, 2048, 4096)
ALPHAS = (0.01, 0.05, 0.2, 0.5)
LEAVES = (32, 64, 128)
DEFAULT_LEAF = 64
MARGIN = 0.10
PROBE_LEAF = 32  # the leaf at which a product's density is measured
COPIES = 8       # products per timed batch
TABLE_FILE = Path(__file__).resolve().parent / "data" / "leaf_table.json"


def _time_ms(fn, reps: int) -> float:
    for _ in range(2):
        fn()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for e0, e1 in evs:
        e0.record()
        fn()
        e1.record()
    torch.cuda.synchronize()
    return float(np.median([e0.elapsed_time(e1) for e0, e1 in evs]))


def density(a: torch.Tensor, b: torch.Tensor, tau: float) -> float:
    """Fraction of the leaf-32 tile triples of (a, b) whose norm product is at
    least tau (the plan's kept pairs / bdim^3), at least one triple."""
    n = a.shape[0]
    _, _, pairs = sp.prepare(a, b, tau, PROBE_LEAF)
    return max(int(pairs.item()), 1) / float(sp.bdim(n, PROBE_LEAF)) ** 3


def tune(device, *, tau: float = 1e-6, sizes=SIZES, alphas=ALPHAS, leaves=LEAVES, reps: int = 9) -> dict:
    """{"buckets": [{"n", "alpha", "density", "ms": {leaf: ms per product}, "leaf"}], ...}"""
    rows = []
    for n in sizes:
        for al in alphas:
            a = inputs.exp_decay_torch(n, al, 900, device)
            b = inputs.exp_decay_torch(n, al, 901, device)
            ms = {}
            for leaf in leaves:
                bt = sp.Batch([a] * COPIES, [b] * COPIES, [leaf] * COPIES, [tau] * COPIES)
                ms[leaf] = _time_ms(bt.run, reps) / COPIES
                del bt
            best = min(ms, key=ms.get)
            if DEFAULT_LEAF in ms and ms[best] > (1.0 - MARGIN) * ms[DEFAULT_LEAF]:
                best = DEFAULT_LEAF
            rows.append({"n": n, "alpha": al, "density": density(a, b, tau), "ms": {str(k): v for k, v in ms.items()},
                         "leaf": int(best)})
    return {"tau": tau, "leaves": list(leaves), "margin": MARGIN, "default": DEFAULT_LEAF, "probe_leaf": PROBE_LEAF,
            "copies": COPIES, "buckets": rows}


def choose(table: dict, n: int, dens: float) -> int:
    """The leaf of the bucket nearest to (n, density) in (log n, log density)."""
    best, dist = None, math.inf
    for r in table["buckets"]:
        d = (math.log(n / r["n"])) ** 2 + (math.log(dens / r["density"])) ** 2
        if d < dist:
            best, dist = r["leaf"], d
    return int(best)


def save(table: dict, path) -> None:
    Path(path).write_text(json.dumps(table, indent=1) + "\n")


def load(path) -> dict:
    return json.loads(Path(path).read_text())
