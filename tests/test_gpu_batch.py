"""Batched products on the GPU (spamm_batch_setup / spamm_batch_run): every
product equals the oracle (pairs exactly; C within the FP32 accumulation bound
of the single-product tests) or, at sizes the oracle is slow for, the
single-product path (same pairs; relative Frobenius difference <= 1e-6, the two
only differ in accumulation order); replays of a captured graph equal the eager
run bitwise."""

from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle
from paper_2103_13042_amd import binding as sp
from paper_2103_13042_amd import inputs

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda", 0)
U32 = 2.0**-24

# (n, leaf, tau, generator) — ragged sizes, n < leaf, a single element, all leaf classes;
# products with more than 64 tiles per side (2100 and 2200 at leaf 32) are planned by
# the staged launches, the others by one workgroup each, so both kinds sit in one batch
SPECS = [
    (300, 32, 1e-6, "exp"), (1024, 64, 1e-6, "exp"), (777, 128, 1e-6, "exp"), (2100, 32, 1e-6, "exp"),
    (256, 32, 1e-3, "alg"), (100, 128, 1e-6, "exp"), (1, 32, 0.0, "exp"), (512, 64, 0.0, "alg"),
    (640, 32, 1e-6, "alg"), (2048, 64, 1e-6, "alg"), (1536, 128, 1e-5, "exp"), (2200, 32, 0.0, "alg"),
]


def _mats(n, kind, seed):
    if kind == "exp":
        return inputs.exp_decay(n, 0.05, seed), inputs.exp_decay(n, 0.08, seed + 1)
    return inputs.algebraic_decay_signed(n, seed), inputs.algebraic_decay_signed(n, seed + 1)


@pytest.fixture(scope="module")
def batch():
    mats = [_mats(n, kind, 10 * q) for q, (n, _, _, kind) in enumerate(SPECS)]
    ga = [torch.from_numpy(a).to(DEV) for a, _ in mats]
    gb = [torch.from_numpy(b).to(DEV) for _, b in mats]
    bt = sp.Batch(ga, gb, [s[1] for s in SPECS], [s[2] for s in SPECS])
    bt.run()
    torch.cuda.synchronize()
    return mats, bt


def test_batch_matches_oracle_and_single_products(batch):
    mats, bt = batch
    pairs = bt.pairs.cpu().tolist()
    for q, ((n, leaf, tau, _), (a, b)) in enumerate(zip(SPECS, mats)):
        c = bt.c[q].cpu().numpy()
        if n <= 1024:
            c_ref, count, _ = oracle.spamm(a, b, tau, leaf)
            abs_ref, _, _ = oracle.spamm(np.abs(a), np.abs(b), tau, leaf)
            assert pairs[q] == count, q
            bound = n * U32 / (1 - n * U32) * abs_ref + 1e-38
            assert np.all(np.abs(c.astype(np.float64) - c_ref) <= bound), q
        else:
            _, counts, _ = oracle.spamm_tiles(a, b, tau, leaf, oracle.all_tiles(n, leaf), products=False)
            assert pairs[q] == int(counts.sum()), q
        c1, p1 = sp.multiply(torch.from_numpy(a).to(DEV), torch.from_numpy(b).to(DEV), tau, leaf)
        assert pairs[q] == p1, q
        c1 = c1.cpu().numpy().astype(np.float64)
        den = np.linalg.norm(c1)
        assert np.linalg.norm(c - c1) <= 1e-6 * den + 1e-30, q


def test_batch_reruns_are_bitwise_equal(batch):
    _, bt = batch
    first = [c.clone() for c in bt.c]
    for c in bt.c:
        c.fill_(7.0)
    bt.run()
    torch.cuda.synchronize()
    assert all(torch.equal(x, y) for x, y in zip(first, bt.c))


def test_graph_replays_equal_eager_run(batch):
    _, bt = batch
    eager = [c.clone() for c in bt.c]
    eager_pairs = bt.pairs.clone()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        bt.run()  # warm-up on the capture stream
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        bt.run()
    for r in range(3):
        for c in bt.c:
            c.zero_()  # eager work between replays
        bt.pairs.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert all(torch.equal(x, y) for x, y in zip(eager, bt.c)), r
        assert torch.equal(eager_pairs, bt.pairs), r


def test_batch_argument_errors():
    a = torch.ones(64, 64, device=DEV)
    with pytest.raises(sp.SpammError):
        sp.Batch([a], [a], [16], [1e-6])  # leaf 16 is not a batched leaf class
    with pytest.raises(sp.SpammError):
        sp.Batch([a], [a], [32], [-1.0])
    with pytest.raises(ValueError):
        sp.Batch([a], [torch.ones(32, 32, device=DEV)], [32], [1e-6])
    with pytest.raises(sp.SpammError):
        sp.Batch([a, a], [a, a], [32, 64], [1e-6, 1e-6], c_list=[a, torch.ones(64, 64, device=DEV)])  # c aliases a


def _offset_view(x: np.ndarray, offset: int) -> torch.Tensor:
    n = x.shape[0]
    buf = torch.zeros(n * n + offset, dtype=torch.float32, device=DEV)
    buf[offset:] = torch.from_numpy(x).to(DEV).reshape(-1)
    return buf[offset:].view(n, n)


def test_batch_with_members_that_are_only_4_byte_aligned():
    """Members whose A and B start 4, 8 or 12 bytes past a 16-byte boundary sit
    beside aligned ones in every leaf class; each takes the unaligned norm and
    multiply paths and must still equal the oracle."""
    specs = [(640, 32, 1), (640, 32, 0), (1024, 64, 2), (512, 64, 0), (777, 128, 3), (1000, 64, 1)]
    mats = [inputs.exp_decay(n, 0.05, 60 + q) for q, (n, _, _) in enumerate(specs)]
    matsb = [inputs.exp_decay(n, 0.08, 70 + q) for q, (n, _, _) in enumerate(specs)]
    ga = [_offset_view(a, off) if off else torch.from_numpy(a).to(DEV) for a, (_, _, off) in zip(mats, specs)]
    gb = [_offset_view(b, off) if off else torch.from_numpy(b).to(DEV) for b, (_, _, off) in zip(matsb, specs)]
    tau = 1e-6
    bt = sp.Batch(ga, gb, [s[1] for s in specs], [tau] * len(specs))
    bt.run()
    torch.cuda.synchronize()
    pairs = bt.pairs.cpu().tolist()
    for q, ((n, leaf, _), a, b) in enumerate(zip(specs, mats, matsb)):
        c_ref, count, _ = oracle.spamm(a, b, tau, leaf)
        abs_ref, _, _ = oracle.spamm(np.abs(a), np.abs(b), tau, leaf)
        assert pairs[q] == count, q
        bound = n * U32 / (1 - n * U32) * abs_ref + 1e-38
        c = bt.c[q].cpu().numpy().astype(np.float64)
        assert np.all(np.abs(c - c_ref) <= bound), q


# --------------------------------------------------------------------------
# The benchmark batch at its real shape: 256 products, n log-uniform in
# [256, 4096], exponential decay with rates uniform in [0.01, 0.5), tau = 1e-6,
# leaves from the committed tuner table (as the benchmark picks them).  Every
# product's pair count equals the oracle's (the count-only recursion over all
# its output tiles); sampled output tiles of every product equal the oracle's
# within the FP32 accumulation bound.

BATCH_COUNT, BATCH_TAU, CHUNKS = 256, 1e-6, 4


@pytest.fixture(scope="module")
def bench_batch():
    from paper_2103_13042_amd import autotune

    specs = inputs.batch_specs(BATCH_COUNT)
    table = autotune.load(autotune.TABLE_FILE)
    a_l = [inputs.exp_decay_torch(n, aa, sa, DEV) for n, aa, _, sa, _ in specs]
    b_l = [inputs.exp_decay_torch(n, ab, sb, DEV) for n, _, ab, _, sb in specs]
    leaves = [autotune.choose(table, n, autotune.density(a, b, BATCH_TAU)) for (n, *_), a, b in zip(specs, a_l, b_l)]
    bt = sp.Batch(a_l, b_l, leaves, [BATCH_TAU] * len(specs))
    bt.run()
    torch.cuda.synchronize()
    print(f"batch of {len(specs)}: leaves {sorted(set(leaves))}, pairs {int(bt.pairs.sum())}", flush=True)
    return specs, leaves, a_l, b_l, bt


def _batch_tiles(bd: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    pick = {(0, 0), (bd - 1, bd - 1), (0, bd - 1)}
    pick |= {(i, min(bd - 1, i + d)) for i in range(0, bd, max(1, bd // 3)) for d in (0, 1)}
    pick |= {tuple(int(v) for v in rng.integers(0, bd, 2)) for _ in range(3)}
    return np.array(sorted(pick), dtype=np.int64)


@pytest.mark.parametrize("chunk", range(CHUNKS))
def test_benchmark_batch_matches_oracle(bench_batch, chunk):
    specs, leaves, a_l, b_l, bt = bench_batch
    per = len(specs) // CHUNKS
    pairs = bt.pairs.cpu().tolist()
    for q in range(chunk * per, (chunk + 1) * per):
        n, leaf = specs[q][0], leaves[q]
        a, b = a_l[q].cpu().numpy(), b_l[q].cpu().numpy()
        pa, pb = oracle.pyramid(a, leaf), oracle.pyramid(b, leaf)
        _, counts, _ = oracle.spamm_tiles(a, b, BATCH_TAU, leaf, oracle.all_tiles(n, leaf), products=False,
                                          pyr_a=pa, pyr_b=pb)
        assert pairs[q] == int(counts.sum()), (q, n, leaf)
        tiles = _batch_tiles(oracle.bdim(n, leaf), q)
        ct, _, _ = oracle.spamm_tiles(a, b, BATCH_TAU, leaf, tiles, pyr_a=pa, pyr_b=pb)
        abs_t, _, _ = oracle.spamm_tiles(np.abs(a), np.abs(b), BATCH_TAU, leaf, tiles)
        c = bt.c[q]
        for (r0, c0, blk), (_, _, ab) in zip(oracle.tiles_to_matrix_view(ct, tiles, n, leaf),
                                             oracle.tiles_to_matrix_view(abs_t, tiles, n, leaf)):
            got = c[r0:r0 + blk.shape[0], c0:c0 + blk.shape[1]].cpu().numpy().astype(np.float64)
            bound = n * U32 / (1 - n * U32) * ab + 1e-38
            assert np.all(np.abs(got - blk) <= bound), (q, n, leaf, r0, c0)
    print(f"products {chunk * per}..{(chunk + 1) * per - 1}: pairs and sampled tiles equal the oracle", flush=True)
