"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Bars:
  - norms and pyramids: relative difference <= 1e-13 (both sum exact FP64
    squares; only the summation order differs);
  - skip masks: identical, except triples whose oracle norm product lies within
    1e-12 relative of tau (either outcome is correct there);
  - pairs: identical to the oracle's count (and to the closed form for the
    algebraic-decay workload);
  - C: every element within gamma_K * (|A||B| restricted to the kept pairs),
    the FP32 accumulation bound with K = N terms and u = 2^-24, where the
    restricted |A||B| is the oracle's SpAMM of |A| and |B| (same norms, so the
    same mask); and relative Frobenius difference <= 1e-5 (the target for the
    method is 1e-4).
"""

from __future__ import annotations

import math

import numpy as np
import pytest
import torch

import oracle
from closed_forms import closed_form_pair_count
from paper_2103_13042_amd import binding as sp
from paper_2103_13042_amd import inputs

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda", 0)
U32 = 2.0**-24
TIE = 1e-12
REL_FRO = 1e-5


def gpu(x: np.ndarray) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(DEV)


def gamma32(k: int) -> float:
    return k * U32 / (1.0 - k * U32)


def mask_from_plan(offsets: torch.Tensor, klist: torch.Tensor, bd: int) -> np.ndarray:
    off = offsets.cpu().numpy().astype(np.int64)
    total = int(off[-1])
    kl = klist[:total].cpu().numpy().astype(np.int64)
    counts = np.diff(off)
    tiles = np.repeat(np.arange(bd * bd), counts)
    mask = np.zeros((bd * bd, bd), dtype=bool)
    mask[tiles, kl] = True
    # ascending and unique within each tile
    if total:
        same = tiles[1:] == tiles[:-1]
        assert np.all(kl[1:][same] > kl[:-1][same])
        assert kl.min() >= 0 and kl.max() < bd
    return mask.reshape(bd, bd, bd)


def oracle_products(a, b, leaf):
    na, nb = oracle.leaf_norms(a, leaf), oracle.leaf_norms(b, leaf)
    return na[:, None, :] * nb.T[None, :, :]  # [i, j, k] = nA[i,k] * nB[k,j]


def off_tie(prod, tau):
    if tau == 0.0 or math.isinf(tau):
        return np.ones_like(prod, dtype=bool)
    return np.abs(prod / tau - 1.0) > TIE


def check_c(c_gpu: np.ndarray, a, b, tau, leaf, c_ref=None):
    """C against the oracle: elementwise FP32 accumulation bound and rel. Frobenius."""
    n = a.shape[0]
    if c_ref is None:
        c_ref, _, _ = oracle.spamm(a, b, tau, leaf)
    abs_ref, _, _ = oracle.spamm(np.abs(a), np.abs(b), tau, leaf)
    err = np.abs(c_gpu.astype(np.float64) - c_ref)
    bound = gamma32(n) * abs_ref + 1e-38
    worst = float(np.max(err - bound))
    assert worst <= 0.0, f"elementwise bound exceeded by {worst:.3e}"
    den = np.linalg.norm(c_ref)
    rel = np.linalg.norm(c_gpu.astype(np.float64) - c_ref) / den if den > 0 else np.linalg.norm(c_gpu)
    assert rel <= REL_FRO, rel
    return rel


# --------------------------------------------------------------------------
# norm pass and pyramid


@pytest.mark.parametrize(
    "n,leaf,offset",
    [(1024, 32, 0), (1000, 64, 0), (1001, 32, 0), (1024, 64, 1), (1024, 128, 2), (1001, 32, 3), (2050, 64, 1),
     (300, 128, 0), (77, 16, 0), (130, 7, 0), (5, 8, 0)],
)
def test_leaf_norms_match_oracle(n, leaf, offset):
    a = inputs.exp_decay(n, 0.05, 0)
    if offset:  # a view that is only 4-byte aligned takes the path for unaligned rows
        buf = torch.zeros(n * n + offset, dtype=torch.float32, device=DEV)
        buf[offset:] = gpu(a).reshape(-1)
        x = buf[offset:].view(n, n)
    else:
        x = gpu(a)
    got = sp.norms(x, leaf).cpu().numpy()
    want = oracle.leaf_norms(a, leaf)
    np.testing.assert_allclose(got, want, rtol=1e-13, atol=0)


def test_leaf_norms_keep_fp32_subnormals():
    # exp(-1.2*|i-j|) falls through the FP32 subnormal range (< 1.18e-38) a few
    # tiles off the diagonal; those tiles must keep their tiny, non-zero norms.
    n, leaf = 256, 32
    a = inputs.exp_decay(n, 1.2, 3)
    assert np.any((a > 0) & (a < np.finfo(np.float32).tiny))
    got = sp.norms(gpu(a), leaf).cpu().numpy()
    want = oracle.leaf_norms(a, leaf)
    assert np.all((want > 0) == (got > 0))
    np.testing.assert_allclose(got, want, rtol=1e-13, atol=0)


@pytest.mark.parametrize("n,leaf", [(1024, 32), (1000, 64), (1100, 32), (20, 32), (8192, 64)])
def test_pyramid_matches_oracle_and_is_monotone(n, leaf):
    a = inputs.algebraic_decay_signed(n, 0) if n == 8192 else inputs.exp_decay(n, 0.03, 1)
    flat = sp.pyramid(gpu(a), leaf)
    got = [p.cpu().numpy() for p in sp.pyramid_levels(flat, n, leaf)]
    want = oracle.pyramid(a, leaf)
    assert len(got) == len(want)
    for g, w in zip(got, want):
        np.testing.assert_allclose(g, w, rtol=1e-13, atol=0)
    # a parent is never below any of its children (exactly, in the GPU values)
    for l in range(len(got) - 1):
        kids = got[l + 1]
        m = kids.shape[0] // 2
        kmax = kids.reshape(m, 2, m, 2).max(axis=(1, 3))
        assert np.all(got[l] >= kmax)


# --------------------------------------------------------------------------
# plan


def _plan(a, b, leaf, tau):
    n = a.shape[0]
    ga, gb = gpu(a), gpu(b)
    pa, pb = sp.pyramid(ga, leaf), sp.pyramid(gb, leaf)
    offsets, klist, pairs = sp.plan(pa, pb, n, leaf, tau)
    return offsets, klist, int(pairs.item())


@pytest.mark.parametrize(
    "n,leaf,tau,kind",
    [
        (1024, 32, 1e-6, "exp"),
        (1024, 32, 1e-2, "exp"),
        (1000, 64, 0.0, "exp"),
        (1000, 64, 3.0, "rand"),
        (4096, 32, 1e-6, "exp"),  # 128 x 128 grid: two k-chunks and pyramid skipping
        (1100, 16, 1e-5, "exp"),  # 69 x 69 grid padded to 128
    ],
)
def test_plan_mask_matches_oracle(n, leaf, tau, kind):
    if kind == "exp":
        a, b = inputs.exp_decay(n, 0.05, 0), inputs.exp_decay(n, 0.05, 1)
    else:
        a, b = inputs.uniform_pm1(n, 4), inputs.uniform_pm1(n, 5)
    bd = oracle.bdim(n, leaf)
    offsets, klist, pairs = _plan(a, b, leaf, tau)
    got = mask_from_plan(offsets, klist, bd)
    _, count, want = oracle.spamm(a, b, tau, leaf, products=False)
    ok = off_tie(oracle_products(a, b, leaf), tau)
    assert np.array_equal(got[ok], want[ok])
    assert pairs == int(got.sum())
    if ok.all():
        assert pairs == count


@pytest.mark.parametrize("tau", [1e-8, 1e-6, 1e-4])
def test_plan_counts_algebraic_8192(tau, alg8192):
    a, b = alg8192
    offsets, klist, pairs = _plan(a, b, 64, tau)
    want, _ = closed_form_pair_count(8192, 64, tau)
    assert pairs == want
    # masks of sampled tiles against the oracle's recursion
    tiles = _sample_tiles(128, seed=7)
    _, counts, omask = oracle.spamm_tiles(a, b, tau, 64, tiles, products=False)
    got = mask_from_plan(offsets, klist, 128)
    for t, (i, j) in enumerate(tiles):
        assert np.array_equal(got[i, j], omask[t])


# --------------------------------------------------------------------------
# multiply and the whole path


def test_multiply_c1_full_parity(c1):
    a, b, c_ref, count = c1
    c, pairs = sp.multiply(gpu(a), gpu(b), 1e-6, 32)
    assert pairs == count
    rel = check_c(c.cpu().numpy(), a, b, 1e-6, 32, c_ref=c_ref)
    print(f"C1 rel Frobenius vs oracle: {rel:.3e}")


@pytest.mark.parametrize(
    "n,leaf,q,kind",
    [
        (1000, 64, 0.5, "rand"),   # ragged last tile row/column
        (1001, 32, 0.3, "rand"),   # N not a multiple of 4: rows read at 4-byte alignment
        (1003, 64, 0.5, "exp"),    # the same at leaf 64
        (777, 128, 0.6, "exp"),
        (96, 32, 0.0, "rand"),     # tau = 0: the dense product
        (20, 64, 0.0, "rand"),     # one tile smaller than the leaf
        (520, 64, 0.9, "exp"),
        (1024, 128, 0.7, "rand"),
    ],
)
def test_multiply_matches_oracle(n, leaf, q, kind):
    if kind == "exp":
        a, b = inputs.exp_decay(n, 0.02, 8), inputs.exp_decay(n, 0.02, 9)
    else:
        a, b = inputs.uniform_pm1(n, 8), inputs.uniform_pm1(n, 9)
    prod = oracle_products(a, b, leaf)
    tau = float(np.quantile(prod, q)) if q > 0 else 0.0
    c_ref, count, mask = oracle.spamm(a, b, tau, leaf)
    c, pairs = sp.multiply(gpu(a), gpu(b), tau, leaf)
    if off_tie(prod, tau).all():
        assert pairs == count
    check_c(c.cpu().numpy(), a, b, tau, leaf, c_ref=c_ref)


def _offset_view(x: np.ndarray, offset: int) -> torch.Tensor:
    """x on the GPU as a view that starts `offset` floats into its buffer."""
    n = x.shape[0]
    buf = torch.zeros(n * n + offset, dtype=torch.float32, device=DEV)
    buf[offset:] = gpu(x).reshape(-1)
    return buf[offset:].view(n, n)


@pytest.mark.parametrize("n,leaf,offset", [(1024, 64, 1), (1024, 32, 2), (1024, 128, 3), (1000, 64, 1)])
def test_multiply_on_views_that_are_only_4_byte_aligned(n, leaf, offset):
    """A and B start 4, 8 or 12 bytes past a 16-byte boundary: the norm pass and
    the multiply take their paths for unaligned operands, and C must be the
    oracle's and the same, bitwise in the pair count and to the accumulation
    bound in C, as for the aligned copies."""
    a, b = inputs.exp_decay(n, 0.02, 8), inputs.exp_decay(n, 0.02, 9)
    prod = oracle_products(a, b, leaf)
    tau = float(np.quantile(prod, 0.5))
    c_ref, count, _ = oracle.spamm(a, b, tau, leaf)
    ga, gb = _offset_view(a, offset), _offset_view(b, offset)
    assert ga.data_ptr() % 16 != 0 and gb.data_ptr() % 16 != 0
    c, pairs = sp.multiply(ga, gb, tau, leaf)
    if off_tie(prod, tau).all():
        assert pairs == count
    check_c(c.cpu().numpy(), a, b, tau, leaf, c_ref=c_ref)
    c_al, pairs_al = sp.multiply(gpu(a), gpu(b), tau, leaf)
    assert pairs_al == pairs


def test_tau_zero_is_dense_and_counts_every_triple():
    n, leaf = 512, 64
    a, b = inputs.uniform_pm1(n, 1), inputs.uniform_pm1(n, 2)
    c, pairs = sp.multiply(gpu(a), gpu(b), 0.0, leaf)
    assert pairs == (n // leaf) ** 3
    dense = a.astype(np.float64) @ b.astype(np.float64)
    bound = gamma32(n) * (np.abs(a).astype(np.float64) @ np.abs(b).astype(np.float64))
    assert np.all(np.abs(c.cpu().numpy() - dense) <= bound)


@pytest.mark.parametrize("n,leaf", [(4096, 64), (2048, 32), (8192, 128)])
def test_many_pairs_per_workgroup(n, leaf):
    """tau = 0 on a dense random matrix: every workgroup of the multiply owns
    hundreds of pairs, so its pair stream wraps around its LDS ring several
    times.  At tau = 0 SpAMM is the dense product (pinned for the oracle), so
    the reference is the FP64 product of the same FP32 inputs; every element is
    checked against the FP32 accumulation bound."""
    a, b = inputs.uniform_pm1(n, 21), inputs.uniform_pm1(n, 22)
    ga, gb = gpu(a), gpu(b)
    c, pairs = sp.multiply(ga, gb, 0.0, leaf)
    assert pairs == (n // leaf) ** 3
    ref = ga.double() @ gb.double()
    bound = gamma32(n) * (ga.abs().double() @ gb.abs().double())
    excess = float(((c.double() - ref).abs() - bound).max())
    assert excess <= 0.0, excess
    rel = float(torch.linalg.norm(c.double() - ref) / torch.linalg.norm(ref))
    assert rel <= REL_FRO, rel


@pytest.mark.parametrize("leaf", [64, 128])
@pytest.mark.parametrize("kind", ["one_block", "scattered"])
def test_macro_tiles_shared_between_workgroups(kind, leaf):
    """Leaf 64 or 128, N a multiple of 128: the multiply splits its item list
    between workgroups by cost, so one 128x128 macro tile can be computed by
    several workgroups whose partial sums a second kernel adds (leaf 128: one
    macro tile per output tile).
    one_block: all the work sits in one 128x128 block of C (A nonzero in its
    first 128 rows, B in its first 128 columns), so that block is shared by
    many workgroups with about one item each; scattered: random tile-level
    sparsity, many blocks split between two workgroups.  Checked against the
    oracle, and run twice for bitwise equality (the partials are added in
    workgroup order)."""
    rng = np.random.default_rng(31)
    n, tau = 1024, 1e-6
    a, b = inputs.uniform_pm1(n, 41), inputs.uniform_pm1(n, 42)
    if kind == "one_block":
        a[128:, :] = 0.0
        b[:, 128:] = 0.0
    else:
        bd = n // leaf
        ka = np.kron(rng.random((bd, bd)) < 0.15, np.ones((leaf, leaf), dtype=bool))
        kb = np.kron(rng.random((bd, bd)) < 0.15, np.ones((leaf, leaf), dtype=bool))
        a = np.where(ka, a, 0.0).astype(np.float32)
        b = np.where(kb, b, 0.0).astype(np.float32)
    c_ref, count, _ = oracle.spamm(a, b, tau, leaf)
    ga, gb = gpu(a), gpu(b)
    c1, p1 = sp.multiply(ga, gb, tau, leaf)
    c2, p2 = sp.multiply(ga, gb, tau, leaf)
    assert p1 == p2 == count
    assert torch.equal(c1, c2)
    check_c(c1.cpu().numpy(), a, b, tau, leaf, c_ref=c_ref)


def test_tau_above_every_product_gives_exact_zero():
    n, leaf = 700, 64
    a, b = inputs.uniform_pm1(n, 3), inputs.uniform_pm1(n, 4)
    ga, gb = gpu(a), gpu(b)
    big = 2.0 * float(np.linalg.norm(a.astype(np.float64)) * np.linalg.norm(b.astype(np.float64)))
    for tau in (big, math.inf):
        c = torch.full((n, n), 7.0, device=DEV)
        _, pairs = sp.multiply(ga, gb, tau, leaf, c=c)
        assert pairs == 0
        assert torch.count_nonzero(c).item() == 0


def test_zero_matrix():
    n, leaf = 300, 32
    z = torch.zeros((n, n), device=DEV)
    b = gpu(inputs.uniform_pm1(n, 5))
    c, pairs = sp.multiply(z, b, 1e-9, leaf)
    assert pairs == 0 and torch.count_nonzero(c).item() == 0
    c, pairs = sp.multiply(z, b, 0.0, leaf)  # 0 >= 0: every triple is multiplied
    assert pairs == oracle.bdim(n, leaf) ** 3 and torch.count_nonzero(c).item() == 0


def test_runs_are_bitwise_deterministic(c1):
    a, b, _, _ = c1
    ga, gb = gpu(a), gpu(b)
    c1_, p1 = sp.multiply(ga, gb, 1e-6, 32)
    c2_, p2 = sp.multiply(ga, gb, 1e-6, 32)
    assert p1 == p2 and torch.equal(c1_, c2_)


def test_staged_calls_equal_the_fused_call(c1):
    """The staged calls (pyramids, plan, execute; prepare, execute) agree
    bitwise.  The one-call path takes the small-product kernel at this size:
    the same pairs, and C equal up to the order of the FP32 additions (the
    k-range of a tile is split between four wave groups)."""
    a, b, c_ref, _ = c1
    ga, gb = gpu(a), gpu(b)
    c_fused, pairs = sp.multiply(ga, gb, 1e-6, 32)
    pa, pb = sp.pyramid(ga, 32), sp.pyramid(gb, 32)
    offsets, klist, p = sp.plan(pa, pb, 1024, 32, 1e-6)
    c_staged = sp.execute(ga, gb, 32, offsets, klist)
    assert int(p.item()) == pairs
    rel = float(torch.linalg.norm((c_fused - c_staged).double()) / torch.linalg.norm(c_staged.double()))
    assert rel <= 1e-6, rel
    check_c(c_fused.cpu().numpy(), a, b, 1e-6, 32, c_ref=c_ref)
    o2, k2, p2 = sp.prepare(ga, gb, 1e-6, 32)
    assert torch.equal(o2, offsets) and int(p2.item()) == pairs
    assert torch.equal(k2[:pairs], klist[:pairs])
    assert torch.equal(sp.execute(ga, gb, 32, o2, k2), c_staged)


@pytest.mark.parametrize(
    "n,q,kind",
    [
        (1024, 0.5, "exp"),
        (1000, 0.7, "rand"),   # ragged last tile row and column
        (2048, 0.9, "exp"),    # 64 tiles per side: the largest small-product grid
        (996, 0.0, "rand"),    # tau = 0: every triple
        (36, 0.3, "rand"),     # 2 x 2 tiles, the second 4 wide
        (4, 0.0, "rand"),      # one tile of 4 x 4
        (2052, 0.5, "exp"),    # 65 tiles per side: the general path
    ],
)
def test_small_product_path_matches_oracle_and_staged_path(n, q, kind):
    """Leaf 32 with at most 64 tiles per side goes through one norm launch and
    one threshold-and-multiply launch.  Pairs equal the oracle's and the staged
    path's exactly; C is within the FP32 accumulation bound of the oracle and
    within 1e-6 (relative Frobenius) of the staged path; every element of C is
    written; two runs are bitwise equal."""
    leaf = 32
    if kind == "exp":
        a, b = inputs.exp_decay(n, 0.02, 18), inputs.exp_decay(n, 0.02, 19)
    else:
        a, b = inputs.uniform_pm1(n, 18), inputs.uniform_pm1(n, 19)
    prod = oracle_products(a, b, leaf)
    tau = float(np.quantile(prod, q)) if q > 0 else 0.0
    c_ref, count, _ = oracle.spamm(a, b, tau, leaf)
    ga, gb = gpu(a), gpu(b)
    c = torch.full((n, n), 7.0, device=DEV)
    pairs_dev = torch.full((1,), 12345, dtype=torch.int64, device=DEV)
    c, pairs = sp.multiply(ga, gb, tau, leaf, c=c, pairs=pairs_dev)
    if off_tie(prod, tau).all():
        assert pairs == count
    check_c(c.cpu().numpy(), a, b, tau, leaf, c_ref=c_ref)
    offsets, klist, p = sp.prepare(ga, gb, tau, leaf)
    assert int(p.item()) == pairs
    c_staged = sp.execute(ga, gb, leaf, offsets, klist)
    den = float(torch.linalg.norm(c_staged.double()))
    diff = float(torch.linalg.norm((c - c_staged).double()))
    assert diff <= 1e-6 * den + 1e-30, (diff, den)
    c2, p2 = sp.multiply(ga, gb, tau, leaf)
    assert p2 == pairs and torch.equal(c2, c)


def test_small_product_path_with_nothing_kept():
    n, leaf = 1024, 32
    a, b = inputs.uniform_pm1(n, 3), inputs.uniform_pm1(n, 4)
    ga, gb = gpu(a), gpu(b)
    for tau in (1e30, math.inf):
        c = torch.full((n, n), 7.0, device=DEV)
        _, pairs = sp.multiply(ga, gb, tau, leaf, c=c)
        assert pairs == 0
        assert torch.count_nonzero(c).item() == 0


@pytest.mark.parametrize("n,leaf", [(1024, 32), (1000, 32), (2048, 64), (1100, 64), (1024, 128)])
def test_schedule_then_multiply_kernel_equals_execute(n, leaf):
    a, b = inputs.exp_decay(n, 0.05, 50), inputs.exp_decay(n, 0.05, 51)
    ga, gb = gpu(a), gpu(b)
    ws = sp.workspace(n, leaf, DEV)
    offsets, klist, _ = sp.prepare(ga, gb, 1e-6, leaf, ws=ws)
    c_exec = sp.execute(ga, gb, leaf, offsets, klist, ws=ws)
    sp.schedule(offsets, klist, n, leaf, ws=ws)
    c_two = sp.execute_scheduled(ga, gb, leaf, offsets, klist, ws=ws)
    assert torch.equal(c_exec, c_two)
    # the multiply kernel alone, run again on the same schedule
    c_again = sp.execute_scheduled(ga, gb, leaf, offsets, klist, ws=ws)
    assert torch.equal(c_exec, c_again)


@pytest.mark.parametrize("tau", [1e-8, 1e-6, 1e-4])
def test_algebraic_8192_full_size_sampled_tiles(tau, alg8192):
    """The benchmark workload at full size and in the benchmark's launch
    configuration: pair count against the closed form, sampled output tiles
    against the oracle's recursion for those tiles."""
    a, b = alg8192
    n, leaf = 8192, 64
    c, pairs = sp.multiply(gpu(a), gpu(b), tau, leaf)
    assert pairs == closed_form_pair_count(n, leaf, tau)[0]
    tiles = _sample_tiles(n // leaf, seed=11)
    ct, counts, _ = oracle.spamm_tiles(a, b, tau, leaf, tiles)
    abs_t, _, _ = oracle.spamm_tiles(np.abs(a), np.abs(b), tau, leaf, tiles)
    cg = c.cpu().numpy()
    num = den = 0.0
    for t, (i, j) in enumerate(tiles):
        blk = cg[i * leaf : (i + 1) * leaf, j * leaf : (j + 1) * leaf].astype(np.float64)
        err = np.abs(blk - ct[t])
        assert np.all(err <= gamma32(n) * abs_t[t] + 1e-38), (i, j)
        num += float(np.sum((blk - ct[t]) ** 2))
        den += float(np.sum(ct[t] ** 2))
    assert math.sqrt(num / den) <= REL_FRO


def _sample_tiles(bd: int, seed: int) -> np.ndarray:
    """Diagonal and near-diagonal tiles, the corners, and a seeded random set."""
    rng = np.random.default_rng(seed)
    pick = {(i, i) for i in range(0, bd, max(1, bd // 16))}
    pick |= {(i, min(bd - 1, i + d)) for i in range(0, bd, max(1, bd // 8)) for d in (1, 2, 5)}
    pick |= {(0, bd - 1), (bd - 1, 0), (bd - 1, bd - 1)}
    pick |= {tuple(int(v) for v in rng.integers(0, bd, 2)) for _ in range(24)}
    return np.array(sorted(pick), dtype=np.int64)


# --------------------------------------------------------------------------
# fixtures


@pytest.fixture(scope="module")
def c1():
    a, b = inputs.workload_exp1024()
    c_ref, count, _ = oracle.spamm(a, b, 1e-6, 32)
    return a, b, c_ref, count


@pytest.fixture(scope="module")
def alg8192():
    return inputs.workload_alg8192()


@pytest.mark.parametrize("n,leaf", [(1024, 32), (1000, 64), (1024, 64), (2048, 128)])
def test_one_call_graph_replays_equal_eager_run(n, leaf):
    """spamm_multiply captured in a graph (the small-product path at leaf 32;
    at leaf 64 the register-staged multiply for n = 1000 and, for n a
    multiple of 128, the one-launch plan with its look-back state and the
    LDS-DMA multiply with its fixup kernel; the leaf-128 DMA path) and
    replayed three times with eager work in between: every replay equals the
    eager call bitwise, C and pairs (the pair counter and the plan's state are
    cleared by a kernel, not a memset)."""
    a, b = inputs.exp_decay(n, 0.02, 28), inputs.exp_decay(n, 0.02, 29)
    ga, gb = gpu(a), gpu(b)
    ws = sp.workspace(n, leaf, DEV)
    c = torch.empty((n, n), device=DEV)
    pairs = torch.empty(1, dtype=torch.int64, device=DEV)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        sp.multiply(ga, gb, 1e-6, leaf, c=c, pairs=pairs, ws=ws, sync=False)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    eager_c, eager_pairs = c.clone(), pairs.clone()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        sp.multiply(ga, gb, 1e-6, leaf, c=c, pairs=pairs, ws=ws, sync=False)
    for r in range(3):
        c.fill_(7.0)
        pairs.fill_(-5)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(c, eager_c), r
        assert torch.equal(pairs, eager_pairs), r


@pytest.mark.parametrize("n,leaf", [(1024, 32), (1000, 64)])
def test_one_call_without_a_pair_counter(n, leaf):
    """spamm_multiply with pairs = NULL counts into the workspace instead (the
    small-product path clears that slot in its norm pass): C equals the call
    that returns the count, bitwise, on repeated calls."""
    a, b = inputs.exp_decay(n, 0.02, 38), inputs.exp_decay(n, 0.02, 39)
    ga, gb = gpu(a), gpu(b)
    ws = sp.workspace(n, leaf, DEV)
    c_ref, _ = sp.multiply(ga, gb, 1e-6, leaf, ws=ws)
    for _ in range(2):
        c = torch.full((n, n), 7.0, device=DEV)
        st = sp._lib.spamm_multiply(sp._ptr(ga), sp._ptr(gb), n, 1e-6, leaf, sp._ptr(c), None, sp._ptr(ws),
                                    ws.numel(), sp._stream(DEV))
        assert st == 0
        torch.cuda.synchronize()
        assert torch.equal(c, c_ref)


# --------------------------------------------------------------------------
# leaf 16 (one wave per output tile, 16x16x4 MFMA)


@pytest.mark.parametrize(
    "n,kind,tau",
    [(1024, "c1", 1e-6), (1000, "exp", 1e-6), (1001, "uni", 0.0), (300, "exp", math.inf), (5, "uni", 0.0),
     (17, "uni", 1.0), (2048, "alg", 1e-4), (513, "alg", 1e-3)],
)
def test_leaf16_matches_oracle(n, kind, tau):
    """Leaf 16 through spamm_multiply: ragged N (a partial last tile), N below
    the leaf, tau = 0 (every pair kept), tau = inf (C = 0), the N = 1024
    exponential-decay inputs at leaf 16: pairs equal the oracle's count, C
    within the FP32 accumulation bound."""
    if kind == "c1":
        a, b = inputs.workload_exp1024()
    elif kind == "exp":
        a, b = inputs.exp_decay(n, 0.05, 3), inputs.exp_decay(n, 0.08, 4)
    elif kind == "alg":
        a, b = inputs.algebraic_decay_signed(n, 5), inputs.algebraic_decay_signed(n, 6)
    else:
        a, b = inputs.uniform_pm1(n, 7), inputs.uniform_pm1(n, 8)
    c_ref, count, _ = oracle.spamm(a, b, tau, 16)
    c, pairs = sp.multiply(gpu(a), gpu(b), tau, 16)
    assert pairs == count
    if math.isinf(tau):
        assert pairs == 0 and int(torch.count_nonzero(c)) == 0
    check_c(c.cpu().numpy(), a, b, tau, 16, c_ref=c_ref)


def test_leaf16_staged_calls_equal_one_call():
    n, leaf, tau = 777, 16, 1e-5
    a, b = gpu(inputs.exp_decay(n, 0.03, 1)), gpu(inputs.exp_decay(n, 0.03, 2))
    c1, p1 = sp.multiply(a, b, tau, leaf)
    offsets, klist, pairs = sp.prepare(a, b, tau, leaf)
    c2 = sp.execute(a, b, leaf, offsets, klist)
    assert int(pairs.item()) == p1 and torch.equal(c1, c2)


# --------------------------------------------------------------------------
# a NULL workspace: the library's cached per-device workspace, spamm_release


def test_null_workspace_equals_caller_workspace_and_release():
    cases = [(1024, 32, 1e-6), (2000, 64, 1e-5), (777, 128, 1e-6), (300, 16, 1e-6)]
    for n, leaf, tau in cases:  # growing and shrinking requests on one device
        a, b = gpu(inputs.exp_decay(n, 0.05, 11)), gpu(inputs.exp_decay(n, 0.05, 12))
        c_own, p_own = sp.multiply(a, b, tau, leaf)
        c_lib, p_lib = sp.multiply(a, b, tau, leaf, ws=sp.LIBRARY_WORKSPACE)
        assert p_own == p_lib and torch.equal(c_own, c_lib), (n, leaf)
    sp.release()
    sp.release()  # nothing cached: a no-op
    n, leaf, tau = 512, 32, 1e-4
    a, b = gpu(inputs.exp_decay(n, 0.05, 13)), gpu(inputs.exp_decay(n, 0.05, 14))
    c_own, p_own = sp.multiply(a, b, tau, leaf)
    c_lib, p_lib = sp.multiply(a, b, tau, leaf, ws=sp.LIBRARY_WORKSPACE)  # allocates again
    assert p_own == p_lib and torch.equal(c_own, c_lib)
    sp.release()


# --------------------------------------------------------------------------
# the plan and the multiply schedule from one launch (spamm_prepare_schedule)


@pytest.mark.parametrize(
    "n,leaf,tau,kind",
    [(1000, 64, 1e-6, "exp"), (8192, 64, 1e-6, "alg"), (4160, 32, 1e-5, "exp"), (2080, 32, 0.0, "uni"),
     (300, 32, math.inf, "exp"), (64, 64, 0.0, "uni"), (70, 64, 1e-3, "uni"), (6400, 64, 1e-4, "alg"),
     (3000, 32, 1e-6, "alg")],
)
def test_fused_plan_equals_staged_plan(n, leaf, tau, kind):
    """Offsets, k-lists and pairs of spamm_prepare_schedule equal those of
    spamm_prepare bitwise (odd and even tile grids, one or several 64-tile
    column blocks, tau = 0 and inf), and the multiply after each gives
    bitwise the same C; a second call on the same workspace gives the same
    again (the look-back state is cleared by every call)."""
    if kind == "exp":
        a, b = inputs.exp_decay(n, 0.05, 1), inputs.exp_decay(n, 0.03, 2)
    elif kind == "alg":
        a, b = inputs.algebraic_decay_signed(n, 0), inputs.algebraic_decay_signed(n, 1)
    else:
        a, b = inputs.uniform_pm1(n, 3), inputs.uniform_pm1(n, 4)
    ga, gb = gpu(a), gpu(b)
    ws1 = sp.workspace(n, leaf, DEV).clone()
    ws2 = sp.workspace(n, leaf, DEV).clone()
    o1, k1, p1 = sp.prepare(ga, gb, tau, leaf, ws=ws1)
    c1 = sp.execute(ga, gb, leaf, o1, k1, ws=ws1)
    bd = sp.bdim(n, leaf)
    for rep in range(2):
        o2, k2, p2 = sp.prepare(ga, gb, tau, leaf, ws=ws2, schedule=True)
        c2 = sp.execute_scheduled(ga, gb, leaf, o2, k2, ws=ws2)
        total = int(p1.item())
        assert int(p2.item()) == total, rep
        assert torch.equal(o1[: bd * bd + 1], o2[: bd * bd + 1]), rep
        assert torch.equal(k1[:total], k2[:total]), rep
        assert torch.equal(c1, c2), rep
    if n == 8192:
        assert total == closed_form_pair_count(n, leaf, tau)[0]
