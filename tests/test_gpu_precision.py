"""Reduced-precision leaf products on the GPU (through the C ABI) against the
FP64 oracle of oracle/precision.py.

Bars:
  - split operands: bitwise equal to the oracle's rounding (bf16; FP16 hi and
    lo with the same scale exponents), B planes transposed;
  - skip mask / pairs: identical to the FP32 path's;
  - C: every element within gamma_K * (|A||B| restricted to the kept pairs)
    * (1 + 2^-7) of the oracle's reduced-precision result, with K the number
    of FP32 accumulations per element (n for bf16, 3n for the three FP16
    products), i.e. only the FP32 accumulation differs;
  - and, stated as the accuracy of each form against the FP64 SpAMM oracle of
    the FP32 inputs: relative Frobenius error <= 1e-6 for f16x3, and for bf16
    the bound its operand rounding allows, (2u + u^2 + gamma_n) * ||(|A||B|)||
    / ||C|| with u = 2^-9 (measured values printed).
"""

from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle
from oracle import precision as pr
from paper_2103_13042_amd import binding as sp
from paper_2103_13042_amd import inputs

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda", 0)
U32 = 2.0**-24


def gpu(x: np.ndarray) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(DEV)


def gamma(k: int) -> float:
    return k * U32 / (1.0 - k * U32)


U_BF16 = 2.0**-9  # unit roundoff of bfloat16 (8 significand bits)


def bf16_bar(abs_norm: float, exact_norm: float, k: int) -> float:
    """Relative Frobenius error BF16 products may reach against the FP64 SpAMM
    of the FP32 inputs: each operand rounded to BF16 moves by at most U_BF16
    relative, so each product a*b by at most 2u + u^2, plus the FP32
    accumulation of k terms; both relative to ||(|A||B|) on the kept pairs||."""
    return (2 * U_BF16 + U_BF16**2 + gamma(k)) * abs_norm / exact_norm


@pytest.mark.parametrize("precision", ["bf16", "f16x3"])
@pytest.mark.parametrize("n", [256, 1024])
def test_split_operands_match_oracle(precision, n):
    a, b = inputs.exp_decay(n, 0.05, 11), inputs.algebraic_decay_signed(n, 12)
    ga, gb = gpu(a), gpu(b)
    pa, pb = sp.pyramid(ga, 64), sp.pyramid(gb, 64)
    buf = sp.split(ga, gb, 64, precision, pa, pb)
    exps, planes = sp.split_views(buf, n, precision)
    planes = [p.cpu().numpy().view(np.float16).astype(np.float32) if precision == "f16x3"
              else (p.cpu().numpy().view(np.uint16).astype(np.uint32) << 16).view(np.float32) for p in planes]
    if precision == "bf16":
        assert np.array_equal(planes[0], pr.bf16_round(a))
        assert np.array_equal(planes[1], pr.bf16_round(b).T)
    else:
        ea, eb = (pr.f16_scale_exponent(pr.max_leaf_norm(x, 64)) for x in (a, b))
        assert exps.cpu().tolist() == [ea, eb]
        ha, la = pr.f16_split(a, ea)
        hb, lb = pr.f16_split(b, eb)
        for got, want in zip(planes, (ha, la, hb.T, lb.T)):
            assert np.array_equal(got, want)


def _check(c_gpu, a, b, tau, leaf, precision):
    n = a.shape[0]
    c_or, pairs = pr.spamm_precision(a, b, tau, leaf, precision)
    abs_ref, _, _ = oracle.spamm(np.abs(a), np.abs(b), tau, leaf)
    k = n if precision == "bf16" else 3 * n
    err = np.abs(c_gpu.astype(np.float64) - c_or)
    assert np.all(err <= gamma(k) * abs_ref * (1 + 2.0**-7) + 1e-300), float(np.max(err - gamma(k) * abs_ref))
    c64, _, _ = oracle.spamm(a, b, tau, leaf)
    rel = float(np.linalg.norm(c_gpu.astype(np.float64) - c64) / np.linalg.norm(c64))
    print(f"{precision} n={n} tau={tau:g}: rel. Frobenius error vs the FP64 SpAMM oracle {rel:.2e}")
    if precision == "f16x3":
        assert rel <= 1e-6
    else:
        assert rel <= bf16_bar(np.linalg.norm(abs_ref), np.linalg.norm(c64), n)
    return pairs


@pytest.mark.parametrize("precision", ["bf16", "f16x3"])
@pytest.mark.parametrize("n,kind,tau", [(1024, "exp", 1e-6), (2048, "alg", 1e-6), (256, "exp", 0.0),
                                        (768, "relu", 1e-6), (1024, "alg", 1e-3)])
def test_multiply_precision_matches_oracle(precision, n, kind, tau):
    if kind == "exp":
        a, b = inputs.exp_decay(n, 0.05, 0), inputs.exp_decay(n, 0.05, 1)
    elif kind == "alg":
        a, b = inputs.algebraic_decay_signed(n, 0), inputs.algebraic_decay_signed(n, 1)
    else:
        a, b = inputs.relu_like(n, 0), inputs.relu_like(n, 1)
    c, pairs = sp.multiply_precision(gpu(a), gpu(b), tau, 64, precision)
    _, pairs32 = sp.multiply(gpu(a), gpu(b), tau, 64)
    assert pairs == pairs32
    assert _check(c.cpu().numpy(), a, b, tau, 64, precision) == pairs


def _signed_with_zeros_and_tiny(n, seed):
    # signed entries, negative zeros and entries scaled down by 2^-20 (their
    # FP16 lo parts are subnormal or zero), to pin the in-register rounding
    x = inputs.algebraic_decay_signed(n, seed)
    x[::7, ::5] = -0.0
    x[1::9, ::3] *= np.float32(2.0**-20)
    return x


@pytest.mark.parametrize("kind", ["exp", "signed"])
@pytest.mark.parametrize("precision", ["bf16", "f16x3"])
def test_staged_split_path_equals_fused(precision, kind):
    n, leaf, tau = 1024, 64, 1e-6
    if kind == "exp":
        a, b = inputs.exp_decay(n, 0.02, 5), inputs.exp_decay(n, 0.02, 6)
    else:
        a, b = _signed_with_zeros_and_tiny(n, 5), _signed_with_zeros_and_tiny(n, 6)
    ga, gb = gpu(a), gpu(b)
    c_fused, _ = sp.multiply_precision(ga, gb, tau, leaf, precision)
    ws = sp.workspace(n, leaf, DEV)
    offsets, klist, _ = sp.prepare(ga, gb, tau, leaf, ws=ws)
    pa, pb = sp.pyramid(ga, leaf), sp.pyramid(gb, leaf)
    buf = sp.split(ga, gb, leaf, precision, pa, pb)
    c1 = sp.execute_split(buf, n, leaf, precision, offsets, klist, ws=ws)
    sp.schedule(offsets, klist, n, leaf, ws=ws)
    c2 = sp.execute_split(buf, n, leaf, precision, offsets, klist, ws=ws, scheduled=True)
    assert torch.equal(c_fused, c1) and torch.equal(c1, c2)
    if precision == "f16x3":  # the stages of the in-register split: bitwise the same C
        header = torch.zeros(256, dtype=torch.uint8, device=DEV)
        o3, k3, _ = sp.prepare_scales(ga, gb, tau, leaf, header, ws=ws)
        assert torch.equal(header[:8], buf[:8])
        sp.schedule(o3, k3, n, leaf, ws=ws)
        assert torch.equal(sp.execute_f16x3(ga, gb, leaf, header, o3, k3, ws=ws), c1)
    else:  # BF16 rounded in registers from the FP32 tiles: bitwise the same C
        sp.schedule(offsets, klist, n, leaf, ws=ws)
        assert torch.equal(sp.execute_bf16(ga, gb, leaf, offsets, klist, ws=ws), c1)


@pytest.mark.parametrize("n,kind", [(1024, "exp"), (1024, "signed"), (640, "exp")])
def test_prepare_schedule_scales_equals_the_staged_calls(n, kind):
    """spamm_prepare_schedule_scales (one-launch plan and schedule, then the
    scale exponents) gives the offsets, k-lists, pairs and header of
    spamm_prepare_scales + spamm_schedule, and the in-register FP16 hi+lo
    multiply after it gives bitwise the same C."""
    leaf, tau = 64, 1e-6
    if kind == "exp":
        a, b = inputs.exp_decay(n, 0.02, 11), inputs.exp_decay(n, 0.02, 12)
    else:
        a, b = _signed_with_zeros_and_tiny(n, 11), _signed_with_zeros_and_tiny(n, 12)
    ga, gb = gpu(a), gpu(b)
    ws1, ws2 = sp.workspace(n, leaf, DEV), sp.workspace(n, leaf, DEV)
    h1 = torch.zeros(256, dtype=torch.uint8, device=DEV)
    h2 = torch.full((256,), 7, dtype=torch.uint8, device=DEV)
    o1, k1, p1 = sp.prepare_scales(ga, gb, tau, leaf, h1, ws=ws1)
    sp.schedule(o1, k1, n, leaf, ws=ws1)
    o2, k2, p2 = sp.prepare_scales(ga, gb, tau, leaf, h2, ws=ws2, schedule=True)
    pairs = int(p1.item())
    assert pairs == int(p2.item()) and pairs > 0
    assert torch.equal(o1, o2) and torch.equal(k1[:pairs], k2[:pairs])
    assert torch.equal(h1[:8], h2[:8])
    c1 = sp.execute_f16x3(ga, gb, leaf, h1, o1, k1, ws=ws1)
    c2 = sp.execute_f16x3(ga, gb, leaf, h2, o2, k2, ws=ws2)
    assert torch.equal(c1, c2)
    ea, eb = (pr.f16_scale_exponent(pr.max_leaf_norm(x, leaf)) for x in (a, b))
    assert h2[:8].view(torch.int32).cpu().tolist() == [ea, eb]
    # the header is checked before anything is enqueued
    with pytest.raises(sp.SpammError) as e:
        sp.prepare_scales(ga, gb, tau, leaf, torch.zeros(255, dtype=torch.uint8, device=DEV), ws=ws2, schedule=True)
    assert e.value.status == 2


def test_f16x3_whole_path_needs_only_the_split_header():
    n, leaf, tau = 512, 64, 1e-6
    a, b = gpu(inputs.exp_decay(n, 0.05, 7)), gpu(inputs.exp_decay(n, 0.05, 8))
    c_full, p_full = sp.multiply_precision(a, b, tau, leaf, "f16x3", split_buf=sp.split_buffer(n, "f16x3", DEV))
    header = torch.zeros(256, dtype=torch.uint8, device=DEV)
    c_head, p_head = sp.multiply_precision(a, b, tau, leaf, "f16x3", split_buf=header)
    assert p_full == p_head and torch.equal(c_full, c_head)
    ea, eb = (pr.f16_scale_exponent(pr.max_leaf_norm(x.cpu().numpy(), leaf)) for x in (a, b))
    assert header[:8].view(torch.int32).cpu().tolist() == [ea, eb]
    with pytest.raises(sp.SpammError) as e:
        sp.multiply_precision(a, b, tau, leaf, "f16x3", split_buf=torch.zeros(255, dtype=torch.uint8, device=DEV))
    assert e.value.status == 2
    big = torch.zeros(1024, dtype=torch.uint8, device=DEV)
    with pytest.raises(sp.SpammError) as e:
        sp.multiply_precision(a, b, tau, leaf, "f16x3", split_buf=big[16:])  # not 256-byte aligned
    assert e.value.status == 1


@pytest.mark.parametrize("precision", ["f16x3", "bf16"])
@pytest.mark.parametrize("tau", [0.0, 1e-6])
def test_whole_path_picks_either_form_with_the_same_result(precision, tau):
    # n = 3072, leaf 64: the planes are used from 45 (FP16 hi+lo) or 16 (BF16)
    # pairs per output tile (tau = 0: 48 per tile), the in-register conversion
    # below (tau = 1e-6 on this exponential decay: about 13 per tile); a call
    # with only 256 bytes of split buffer always converts in registers
    n, leaf = 3072, 64
    a, b = gpu(inputs.exp_decay(n, 0.02, 21)), gpu(inputs.exp_decay(n, 0.02, 22))
    c_adapt, p_adapt = sp.multiply_precision(a, b, tau, leaf, precision)
    c_reg, p_reg = sp.multiply_precision(a, b, tau, leaf, precision,
                                         split_buf=torch.zeros(256, dtype=torch.uint8, device=DEV))
    assert p_adapt == p_reg and torch.equal(c_adapt, c_reg)
    assert (p_adapt >= {"f16x3": 45, "bf16": 16}[precision] * (n // leaf) ** 2) == (tau == 0.0)


@pytest.mark.parametrize("precision", ["f16x3", "bf16"])
@pytest.mark.parametrize("tau", [0.0, 1e-6])
def test_whole_path_graph_replays_equal_eager_run(precision, tau):
    """spamm_multiply_precision captured in a graph and replayed three times
    with eager work in between: the form is picked on the device from the
    plan's pair count (tau = 0: the planes; 1e-6: in registers), so every
    replay equals the eager call bitwise, C and pairs."""
    n, leaf = 3072, 64
    a, b = gpu(inputs.exp_decay(n, 0.02, 41)), gpu(inputs.exp_decay(n, 0.02, 42))
    ws = sp.workspace(n, leaf, DEV)
    split_buf = sp.split_buffer(n, precision, DEV)
    c = torch.empty((n, n), device=DEV)
    pairs = torch.empty(1, dtype=torch.int64, device=DEV)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        sp.multiply_precision(a, b, tau, leaf, precision, c=c, pairs=pairs, split_buf=split_buf, ws=ws, sync=False)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    eager_c, eager_pairs = c.clone(), pairs.clone()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        sp.multiply_precision(a, b, tau, leaf, precision, c=c, pairs=pairs, split_buf=split_buf, ws=ws, sync=False)
    for r in range(3):
        c.fill_(7.0)
        pairs.fill_(-5)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(c, eager_c), r
        assert torch.equal(pairs, eager_pairs), r


def test_zero_and_tau_above_every_product():
    n = 512
    z = torch.zeros(n, n, device=DEV)
    c, pairs = sp.multiply_precision(z, z, 0.0, 64, "f16x3")
    assert pairs == (n // 64) ** 3 and int(torch.count_nonzero(c)) == 0
    a = gpu(inputs.exp_decay(n, 0.1, 3))
    c, pairs = sp.multiply_precision(a, a, float("inf"), 64, "bf16")
    assert pairs == 0 and int(torch.count_nonzero(c)) == 0


def test_unsupported_shapes_and_arguments():
    a = gpu(inputs.exp_decay(320, 0.1, 1))
    with pytest.raises(sp.SpammError) as e:
        sp.multiply_precision(a, a, 1e-6, 64, "f16x3")  # 320 is not a multiple of 128
    assert e.value.status == 4
    b = gpu(inputs.exp_decay(256, 0.1, 1))
    with pytest.raises(sp.SpammError):
        sp.multiply_precision(b, b, 1e-6, 32, "bf16")  # leaf 32
    with pytest.raises(sp.SpammError):
        sp.multiply_precision(b, b, 1e-6, 64, 7)
    # FP32 through the same entry point is the plain path
    c0, p0 = sp.multiply_precision(b, b, 1e-6, 64, "fp32")
    c1, p1 = sp.multiply(b, b, 1e-6, 64)
    assert p0 == p1 and torch.equal(c0, c1)


def _sample_tiles(bd, seed):
    rng = np.random.default_rng(seed)
    ii, jj = np.meshgrid(np.arange(bd), np.arange(bd), indexing="ij")
    band = np.stack([ii.ravel(), jj.ravel()], 1)
    band = band[np.abs(band[:, 0] - band[:, 1]) <= 2]
    pick = rng.choice(len(band), 48, replace=False)
    rand = rng.integers(0, bd, size=(16, 2))
    return np.concatenate([band[pick], rand])


@pytest.mark.parametrize("kind", ["exp0.01", "exp0.05", "relu"])
def test_precision_forms_full_size_sampled_tiles(kind):
    # N = 16384, leaf 64, tau = 1e-6: every form on the GPU; the oracle on
    # sampled output tiles (the band |i - j| <= 2 and random tiles).  The
    # exponential-decay rates are those of the precision workload (0.01: 530,860
    # kept pairs, the widest band; 0.05: 27,440), plus the dense ReLU-like pair.
    n, leaf, tau = 16384, 64, 1e-6
    if kind == "relu":
        ga, gb = inputs.relu_like_torch(n, 0, DEV), inputs.relu_like_torch(n, 1, DEV)
    else:
        alpha = float(kind[3:])
        ga, gb = inputs.exp_decay_torch(n, alpha, 0, DEV), inputs.exp_decay_torch(n, alpha, 1, DEV)
    a, b = ga.cpu().numpy(), gb.cpu().numpy()
    bd = n // leaf
    tiles = _sample_tiles(bd, 3)
    pa, pb = oracle.pyramid(a, leaf), oracle.pyramid(b, leaf)
    ea = pr.f16_scale_exponent(float(np.max(pa[-1])))
    eb = pr.f16_scale_exponent(float(np.max(pb[-1])))
    ha, la = pr.f16_split(a, ea)
    hb, lb = pr.f16_split(b, eb)
    qa = np.ldexp(ha.astype(np.float64) + la, -ea).astype(np.float32)
    qb = np.ldexp(hb.astype(np.float64) + lb, -eb).astype(np.float32)
    del ha, hb
    lla = np.ldexp(la.astype(np.float64), -ea).astype(np.float32)
    llb = np.ldexp(lb.astype(np.float64), -eb).astype(np.float32)
    del la, lb
    ref = {
        "fp32": oracle.spamm_tiles(a, b, tau, leaf, tiles, pyr_a=pa, pyr_b=pb)[0],
        "f16x3": oracle.spamm_tiles(qa, qb, tau, leaf, tiles, pyr_a=pa, pyr_b=pb)[0]
        - oracle.spamm_tiles(lla, llb, tau, leaf, tiles, pyr_a=pa, pyr_b=pb)[0],
        "bf16": oracle.spamm_tiles(pr.bf16_round(a), pr.bf16_round(b), tau, leaf, tiles, pyr_a=pa, pyr_b=pb)[0],
    }
    exact = ref["fp32"]
    abs_ref = oracle.spamm_tiles(np.abs(a), np.abs(b), tau, leaf, tiles, pyr_a=pa, pyr_b=pb)[0]
    _, pairs32 = sp.multiply(ga, gb, tau, leaf)
    for prec, k in (("fp32", n), ("f16x3", 3 * n), ("bf16", n)):
        c, pairs = sp.multiply_precision(ga, gb, tau, leaf, prec)
        assert pairs == pairs32
        got = np.stack([c[i * leaf:(i + 1) * leaf, j * leaf:(j + 1) * leaf].cpu().numpy() for i, j in tiles])
        err = np.abs(got.astype(np.float64) - ref[prec])
        assert np.all(err <= gamma(k) * abs_ref * (1 + 2.0**-7) + 1e-300), prec
        rel = float(np.linalg.norm(got - exact) / np.linalg.norm(exact))
        print(f"{kind} {prec}: pairs {pairs}, sampled rel. error vs FP64 SpAMM {rel:.2e}")
        bar = {"fp32": 1e-5, "f16x3": 1e-6,
               "bf16": bf16_bar(float(np.linalg.norm(abs_ref)), float(np.linalg.norm(exact)), n)}[prec]
        assert rel <= bar, (prec, rel, bar)
