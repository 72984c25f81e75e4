"""Seeded synthetic inputs for SpAMM: decay matrices in FP32, row-major, N x N.

This module holds no SpAMM arithmetic. It only draws matrices; both the HIP path
(tests, bench) and the CPU oracle consume exactly the arrays it returns.

Decay classes follow the paper's definitions in its background section (decay
matrices): exponential decay |A_ij| < c*lambda^|i-j| and algebraic decay
|A_ij| < c/(|i-j|^lambda + 1).

Random numbers come from one counter-based generator: the SplitMix64 output
function (Steele, Lea, Flood, "Fast splittable pseudorandom number generators",
OOPSLA 2014) applied to a counter built from (seed, row, column).  Each element
is a pure function of (seed, i, j), so the upper-left block of a larger matrix
equals the smaller matrix, and any row range can be generated on its own.
Values are computed in float64 and rounded once to float32.
"""

from __future__ import annotations

import numpy as np

_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_ROWS_PER_CHUNK = 256


def _mix64(z: np.ndarray) -> np.ndarray:
    """SplitMix64 finaliser on a uint64 array (wrapping arithmetic)."""
    z = (z ^ (z >> np.uint64(30))) * _M1
    z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def hash64(seed: int, rows: np.ndarray, cols: np.ndarray) -> np.ndarray:
    """64-bit hash of (seed, i, j); rows/cols broadcast against each other."""
    ctr = (rows.astype(np.uint64) << np.uint64(32)) | cols.astype(np.uint64)
    key = np.uint64(((seed + 1) * 0x9E3779B97F4A7C15) & 0xFFFFFFFFFFFFFFFF)
    with np.errstate(over="ignore"):
        return _mix64(ctr + key)


def uniform01(seed: int, rows: np.ndarray, cols: np.ndarray) -> np.ndarray:
    """u in [0, 1) with 53 random bits: (h >> 11) * 2^-53."""
    h = hash64(seed, rows, cols)
    return (h >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


def sign_pm1(seed: int, rows: np.ndarray, cols: np.ndarray) -> np.ndarray:
    """+1 or -1 from the top bit of the hash."""
    h = hash64(seed, rows, cols)
    return 1.0 - 2.0 * (h >> np.uint64(63)).astype(np.float64)


def _build(n: int, fn) -> np.ndarray:
    """Fill an n x n float32 matrix chunk by chunk of rows; fn(rows, cols, dist) -> float64."""
    if n < 0:
        raise ValueError("n must be >= 0")
    out = np.empty((n, n), dtype=np.float32)
    cols = np.arange(n, dtype=np.int64)[None, :]
    for r0 in range(0, n, _ROWS_PER_CHUNK):
        r1 = min(n, r0 + _ROWS_PER_CHUNK)
        rows = np.arange(r0, r1, dtype=np.int64)[:, None]
        dist = np.abs(rows - cols).astype(np.float64)
        out[r0:r1] = fn(rows, cols, dist).astype(np.float32)
    return out


def exp_decay(n: int, alpha: float, seed: int) -> np.ndarray:
    """A_ij = exp(-alpha*|i-j|) * (0.5 + 0.5*u_ij), u ~ U[0,1) from `seed`."""
    return _build(n, lambda r, c, d: np.exp(-alpha * d) * (0.5 + 0.5 * uniform01(seed, r, c)))


def algebraic_decay_signed(n: int, seed: int, power: float = 2.0) -> np.ndarray:
    """A_ij = s_ij / (1 + |i-j|)^power with s_ij = +-1 from `seed`."""
    return _build(n, lambda r, c, d: sign_pm1(seed, r, c) / (1.0 + d) ** power)


def paper_algebraic_band(n: int) -> np.ndarray:
    """v[d] = 0.1 / (d^0.1 + 1) for d = 0 .. n-1, rounded to float32: the
    distinct entries of the paper's synthetic matrix (section 4.1)."""
    d = np.arange(max(n, 0), dtype=np.float64)
    return (0.1 / (d ** 0.1 + 1.0)).astype(np.float32)


def paper_algebraic(n: int) -> np.ndarray:
    """The paper's synthetic evaluation matrix, a_ij = 0.1 / (|i-j|^0.1 + 1) (section 4.1),
    as the symmetric Toeplitz matrix of paper_algebraic_band(n)."""
    if n < 0:
        raise ValueError("n must be >= 0")
    v = paper_algebraic_band(n)
    out = np.empty((n, n), dtype=np.float32)
    cols = np.arange(n, dtype=np.int64)[None, :]
    for r0 in range(0, n, _ROWS_PER_CHUNK):
        r1 = min(n, r0 + _ROWS_PER_CHUNK)
        rows = np.arange(r0, r1, dtype=np.int64)[:, None]
        out[r0:r1] = v[np.abs(rows - cols)]
    return out


def paper_algebraic_torch(n: int, device):
    """paper_algebraic(n) built on the device from the same float32 band (bitwise
    the host generator's entries, without an N^2 host array)."""
    import torch

    v = torch.from_numpy(paper_algebraic_band(n)).to(device)
    w = torch.cat([v.flip(0), v[1:]])  # w[m] = v[|m - (n-1)|]
    # y[i, j'] = w[i + j'];  x[i, j] = y[i, n-1-j] = w[i - j + n - 1] = v[|i - j|]
    return torch.as_strided(w, (n, n), (1, 1)).flip(1).contiguous()


def uniform_pm1(n: int, seed: int) -> np.ndarray:
    """Dense test matrix, entries uniform in [-1, 1)."""
    return _build(n, lambda r, c, d: 2.0 * uniform01(seed, r, c) - 1.0)


def uniform_pm1_rect(rows: int, cols: int, seed: int) -> np.ndarray:
    """Rectangular variant of uniform_pm1 (used to build structured test tiles)."""
    r = np.arange(rows, dtype=np.int64)[:, None]
    c = np.arange(cols, dtype=np.int64)[None, :]
    return (2.0 * uniform01(seed, r, c) - 1.0).astype(np.float32)


# Named workloads.  Sizes and parameters mirror the configurations the method is
# measured on; every matrix is synthetic and seeded.
def workload_exp1024() -> tuple[np.ndarray, np.ndarray]:
    """N=1024 exponential decay, alpha=0.05, A seed 0, B seed 1."""
    return exp_decay(1024, 0.05, 0), exp_decay(1024, 0.05, 1)


def workload_alg8192(n: int = 8192) -> tuple[np.ndarray, np.ndarray]:
    """N=8192 algebraic decay 1/(1+|i-j|)^2 with random signs, A seed 0, B seed 1."""
    return algebraic_decay_signed(n, 0), algebraic_decay_signed(n, 1)


# Learned-threshold data.
MLP_SHAPES = ((128, 129), (128,), (128, 128), (128,), (128,), (1,))  # W1, b1, W2, b2, w3, b3
MLP_FAN_IN = (129, 129, 128, 128, 128, 128)


def mlp_init(seed: int) -> np.ndarray:
    """Initial network parameters, flat float32 in the order W1, b1, W2, b2, w3, b3:
    each tensor uniform in [-1/sqrt(fan_in), 1/sqrt(fan_in)) of its layer, drawn
    from (seed, tensor index, element index)."""
    parts = []
    for t, (shape, fan) in enumerate(zip(MLP_SHAPES, MLP_FAN_IN)):
        k = int(np.prod(shape))
        u = uniform01(seed, np.full(k, t, dtype=np.int64), np.arange(k, dtype=np.int64))
        parts.append((2.0 * u - 1.0) / np.sqrt(fan))
    return np.concatenate(parts).astype(np.float32)


def decay_pair_params(index: int, seed: int = 7) -> tuple[float, float, int, int]:
    """(alpha_A, alpha_B, seed_A, seed_B) of the index-th training pair: alphas
    uniform in [0.01, 0.5), matrix seeds distinct per pair."""
    i = np.array([index], dtype=np.int64)
    a1 = 0.01 + 0.49 * float(uniform01(seed, i, np.array([0]))[0])
    a2 = 0.01 + 0.49 * float(uniform01(seed, i, np.array([1]))[0])
    return a1, a2, 1000 + 2 * index, 1001 + 2 * index


def log_uniform_target(index: int, lo: float = 1e-6, hi: float = 1e-2, seed: int = 11) -> float:
    """Relative-error target of the index-th training pair, log-uniform in [lo, hi)."""
    u = float(uniform01(seed, np.array([index], dtype=np.int64), np.array([0]))[0])
    return float(10.0 ** (np.log10(lo) + u * (np.log10(hi) - np.log10(lo))))


def _uniform01_torch(seed: int, rows, cols):
    """uniform01 with torch int64 tensors (same bits as the numpy version)."""

    def wrap(v: int) -> int:  # uint64 constant as the int64 with the same bits
        return v - (1 << 64) if v >= 1 << 63 else v

    def lshr(z, s: int):  # logical right shift of int64 bit patterns
        return (z >> s) & ((1 << (64 - s)) - 1)

    key = wrap(((seed + 1) * 0x9E3779B97F4A7C15) & 0xFFFFFFFFFFFFFFFF)
    m1, m2 = wrap(0xBF58476D1CE4E5B9), wrap(0x94D049BB133111EB)
    z = ((rows << 32) | cols) + key
    z = (z ^ lshr(z, 30)) * m1
    z = (z ^ lshr(z, 27)) * m2
    z = z ^ lshr(z, 31)
    import torch

    return lshr(z, 11).to(torch.float64) * (1.0 / 9007199254740992.0)


def _build_torch(n: int, device, fn):
    import torch

    out = torch.empty((n, n), dtype=torch.float32, device=device)
    cols = torch.arange(n, dtype=torch.int64, device=device)[None, :]
    step = max(1, (1 << 22) // max(1, n))
    for r0 in range(0, n, step):
        r1 = min(n, r0 + step)
        rows = torch.arange(r0, r1, dtype=torch.int64, device=device)[:, None]
        out[r0:r1] = fn(rows, cols).to(torch.float32)
    return out


def exp_decay_torch(n: int, alpha: float, seed: int, device):
    """exp_decay(n, alpha, seed) generated with torch on `device` (same counter
    hash and formula; the integer steps are exact, exp may differ from numpy's
    in the last FP64 bit).  Returns a float32 [n, n] tensor."""
    import torch

    return _build_torch(n, device, lambda r, c: torch.exp(-alpha * (r - c).abs().to(torch.float64))
                        * (0.5 + 0.5 * _uniform01_torch(seed, r, c)))


# ReLU-like matrices: 60 % exact zeros at random positions, the other entries
# N(0, 1) (Box-Muller from two more uniforms) clipped at 0.  Three independent
# streams per element: seeds 4s (zero mask), 4s+1 and 4s+2 (Box-Muller).
RELU_ZERO_FRACTION = 0.6


def relu_like(n: int, seed: int) -> np.ndarray:
    def fn(r, c, d):
        keep = uniform01(4 * seed, r, c) >= RELU_ZERO_FRACTION
        u1 = 1.0 - uniform01(4 * seed + 1, r, c)  # (0, 1]
        u2 = uniform01(4 * seed + 2, r, c)
        z = np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)
        return np.where(keep, np.maximum(z, 0.0), 0.0)

    return _build(n, fn)


def relu_like_torch(n: int, seed: int, device):
    """relu_like on `device` (log, sqrt and cos may differ from numpy's in the
    last FP64 bit)."""
    import torch

    def fn(r, c):
        keep = _uniform01_torch(4 * seed, r, c) >= RELU_ZERO_FRACTION
        u1 = 1.0 - _uniform01_torch(4 * seed + 1, r, c)
        u2 = _uniform01_torch(4 * seed + 2, r, c)
        z = torch.sqrt(-2.0 * torch.log(u1)) * torch.cos(2.0 * np.pi * u2)
        return torch.where(keep, z.clamp_min(0.0), torch.zeros_like(z))

    return _build_torch(n, device, fn)


def batch_specs(count: int = 256, seed: int = 13, n_lo: int = 256, n_hi: int = 4096):
    """(n, alpha_A, alpha_B, seed_A, seed_B) of `count` independent products:
    n log-uniform in [n_lo, n_hi], decay rates uniform in [0.01, 0.5)."""
    out = []
    for q in range(count):
        i = np.array([q], dtype=np.int64)
        u = float(uniform01(seed, i, np.array([0]))[0])
        n = int(round(n_lo * (n_hi / n_lo) ** u))
        aa = 0.01 + 0.49 * float(uniform01(seed, i, np.array([1]))[0])
        ab = 0.01 + 0.49 * float(uniform01(seed, i, np.array([2]))[0])
        out.append((n, aa, ab, 5000 + 2 * q, 5001 + 2 * q))
    return out
