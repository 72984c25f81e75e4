"""FP64 CPU oracle for the learned threshold (test infrastructure only).

Only the test suite may import this module.  It states, in plain numpy FP64, what
the learned-threshold path computes:

* features: for A and for B, a 64-bin histogram of log10 of the positive
  leaf-tile Frobenius norms (Eq. 2) over the fixed range [-46, 3) (norms
  outside the range in the first or last bin; zero norms are not counted),
  each bin as tiles per tile row (count / bdim) capped at 4; then log10 of the
  requested relative error.  129 numbers.  Per tile row, a band of the same
  decay gives the same features at any N; the cap bounds the bins of tiny
  far-off-diagonal norms, which grow with N.
* the network: 129 -> 128 -> 128 -> 1, GELU (erf form) after both hidden
  layers, output log10(tau).  Parameters flat in this order: W1 [128, 129]
  (row = output unit), b1 [128], W2 [128, 128], b2 [128], w3 [128], b3 [1].
* the loss: mean squared error of the predicted log10(tau).
* Adam (Kingma and Ba, ICLR 2015) with bias correction.
* labels: for (A, B, leaf, target), the largest norm product tau whose SpAMM
  result has ||AB - SpAMM(A, B, tau)||_F <= target * ||AB||_F (brute force
  over every distinct leaf norm product, for small inputs).

The threshold search it learns to shortcut is the paper's (section 3.5.2, which
searches tau for a valid ratio); the relative-error target is the accuracy
measure of section 4 (Eq. 5 for the error matrix).
"""

from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

from . import leaf_norms, spamm

N_BINS = 64
LOG_LO = -46.0
LOG_HI = 3.0
HIST_CAP = 4.0
N_IN = 2 * N_BINS + 1
N_HID = 128

SHAPES = (("W1", (N_HID, N_IN)), ("b1", (N_HID,)), ("W2", (N_HID, N_HID)), ("b2", (N_HID,)),
          ("w3", (N_HID,)), ("b3", (1,)))
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(flat) -> dict:
    flat = np.asarray(flat, dtype=np.float64)
    if flat.shape != (N_PARAMS,):
        raise ValueError(f"expected {N_PARAMS} parameters")
    out, o = {}, 0
    for name, shape in SHAPES:
        k = int(np.prod(shape))
        out[name] = flat[o : o + k].reshape(shape)
        o += k
    return out


def pack(p: dict) -> np.ndarray:
    return np.concatenate([np.asarray(p[name], dtype=np.float64).ravel() for name, _ in SHAPES])


# --------------------------------------------------------------------------
# features


def histogram(norms, rows: int) -> np.ndarray:
    """64-bin histogram of log10 of the positive norms over [LOG_LO, LOG_HI),
    as counts per row of the tile grid (rows = bdim), capped at HIST_CAP."""
    x = np.asarray(norms, dtype=np.float64).ravel()
    bins = np.zeros(N_BINS, dtype=np.int64)
    pos = x > 0
    t = (np.log10(x[pos]) - LOG_LO) * (N_BINS / (LOG_HI - LOG_LO))
    idx = np.clip(np.floor(t), 0, N_BINS - 1).astype(np.int64)
    np.add.at(bins, idx, 1)
    return np.minimum(bins / float(rows), HIST_CAP)


def bin_position(norms) -> np.ndarray:
    """Continuous bin coordinate t of each positive norm (for tie checks)."""
    x = np.asarray(norms, dtype=np.float64).ravel()
    x = x[x > 0]
    return (np.log10(x) - LOG_LO) * (N_BINS / (LOG_HI - LOG_LO))


def features(a, b, leaf: int, target: float) -> np.ndarray:
    na, nb = leaf_norms(a, leaf), leaf_norms(b, leaf)
    return np.concatenate([histogram(na, na.shape[0]), histogram(nb, nb.shape[0]), [math.log10(target)]])


# --------------------------------------------------------------------------
# the network


def gelu(x):
    return 0.5 * x * (1.0 + erf(x / math.sqrt(2.0)))


def gelu_grad(x):
    return 0.5 * (1.0 + erf(x / math.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)


def forward(flat, x):
    """Predicted log10(tau) for each row of x [B, 129]; returns (y [B], cache)."""
    p = unpack(flat)
    x = np.asarray(x, dtype=np.float64)
    z1 = x @ p["W1"].T + p["b1"]
    h1 = gelu(z1)
    z2 = h1 @ p["W2"].T + p["b2"]
    h2 = gelu(z2)
    y = h2 @ p["w3"] + p["b3"][0]
    return y, (x, z1, h1, z2, h2)


def loss_and_grad(flat, x, t):
    """Mean squared error and its gradient with respect to the flat parameters."""
    p = unpack(flat)
    y, (x, z1, h1, z2, h2) = forward(flat, x)
    t = np.asarray(t, dtype=np.float64)
    nb = y.shape[0]
    r = y - t
    loss = float(np.mean(r * r))
    dy = 2.0 * r / nb
    g = {"w3": h2.T @ dy, "b3": np.array([dy.sum()])}
    dz2 = np.outer(dy, p["w3"]) * gelu_grad(z2)
    g["W2"] = dz2.T @ h1
    g["b2"] = dz2.sum(axis=0)
    dz1 = (dz2 @ p["W2"]) * gelu_grad(z1)
    g["W1"] = dz1.T @ x
    g["b1"] = dz1.sum(axis=0)
    return loss, pack(g)


def adam_step(flat, grad, m, v, step: int, lr: float, beta1: float = 0.9, beta2: float = 0.999,
              eps: float = 1e-8):
    """One Adam update (step counts from 1); returns new (params, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mh = m / (1.0 - beta1**step)
    vh = v / (1.0 - beta2**step)
    return flat - lr * mh / (np.sqrt(vh) + eps), m, v


# --------------------------------------------------------------------------
# labels


def rel_error(a, b, tau: float, leaf: int) -> float:
    """||AB - SpAMM(A, B, tau)||_F / ||AB||_F with the oracle's SpAMM (FP64)."""
    a64, b64 = np.asarray(a, np.float64), np.asarray(b, np.float64)
    ab = a64 @ b64
    c, _, _ = spamm(a, b, tau, leaf)
    den = np.linalg.norm(ab)
    return float(np.linalg.norm(ab - c) / den) if den > 0 else 0.0


def label_tau(a, b, leaf: int, target: float) -> float:
    """Largest leaf norm product tau with rel_error(tau) <= target (brute force)."""
    na, nb = leaf_norms(a, leaf), leaf_norms(b, leaf)
    prods = np.unique((na[:, :, None] * nb[None, :, :]).ravel())[::-1]  # descending
    for tau in prods:
        if rel_error(a, b, float(tau), leaf) <= target:
            return float(tau)
    raise ValueError("no threshold meets the target")
