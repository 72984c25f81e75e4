"""Threshold for a requested accuracy, learned from the plain method.

Given A, B, the leaf size and a relative-error target, the threshold wanted is
the largest leaf norm product tau with ||AB - SpAMM(A, B, tau)||_F <=
target * ||AB||_F (the paper measures accuracy by that error matrix, Eq. 5 and
section 4, and searches tau for a valid ratio in section 3.5.2).  The search
(spamm_search_tau_for_error) needs tens of SpAMM evaluations; a small network
maps cheap features (histograms of log10 leaf norms of A and B, and
log10(target)) to a predicted log10(tau), which seeds the search and so cuts
its evaluations, and which can be used on its own.

Everything on the GPU goes through libspamm.so: matrices are generated on the
device, labels come from the search, and the network is trained by the
library's forward, gradient and Adam kernels.  This module only orchestrates
(batching, shuffling order, bookkeeping).

Command line:
  python -m paper_2103_13042_amd.learned_tau --pairs 10000 --n 2048 --out DIR
generates the training set, trains, evaluates on held-out pairs and at N=8192,
and writes DIR/tau_mlp.npy (parameters) and DIR/learned_tau.json (report).
"""

from __future__ import annotations

import argparse
import json
import math
import sys
import time
from dataclasses import dataclass
from pathlib import Path

import numpy as np
import torch

from . import binding as sp
from . import inputs

PARAMS_FILE = Path(__file__).resolve().parent / "data" / "tau_mlp.npy"


@dataclass
class Problem:
    """One (A, B, leaf) problem resident on the device, with what the error
    evaluations need: pyramids, ||AB||_F^2 (from the tau = 0 product), an
    error buffer and a workspace."""

    a: torch.Tensor
    b: torch.Tensor
    leaf: int
    pyr_a: torch.Tensor
    pyr_b: torch.Tensor
    ab_sumsq: float
    e: torch.Tensor
    ws: torch.Tensor

    @property
    def n(self) -> int:
        return self.a.shape[0]

    @classmethod
    def build(cls, a: torch.Tensor, b: torch.Tensor, leaf: int, *, ws=None, e=None):
        n = a.shape[0]
        ws = sp.workspace(n, leaf, a.device) if ws is None else ws
        e = torch.empty_like(a) if e is None else e
        pa, pb = sp.pyramid(a, leaf, ws=ws), sp.pyramid(b, leaf, ws=ws)
        sp.multiply(a, b, 0.0, leaf, c=e, ws=ws, sync=False)  # exact product (every pair kept)
        ab = float(sp.sumsq(e).item())
        return cls(a, b, leaf, pa, pb, ab, e, ws)

    def features(self, target: float, out=None) -> torch.Tensor:
        return sp.tau_features(self.pyr_a, self.pyr_b, self.n, self.leaf, target, out=out)

    def search(self, target: float, guess: float = 0.0, max_evals: int = 64):
        """(tau, err, pairs, evals) of the largest norm product meeting target."""
        return sp.search_tau_for_error(self.a, self.b, self.leaf, target, self.pyr_a, self.pyr_b, self.ab_sumsq,
                                       guess=guess, max_evals=max_evals, e=self.e, ws=self.ws)

    def error(self, tau: float):
        return sp.error_for_tau(self.a, self.b, tau, self.leaf, self.pyr_a, self.pyr_b, self.ab_sumsq, e=self.e,
                                ws=self.ws)


def decay_problem(n: int, index: int, leaf: int, device, *, seed: int = 7, ws=None, e=None) -> Problem:
    """The index-th exponential-decay pair: alphas uniform in [0.01, 0.5)."""
    aa, ab, sa, sb = inputs.decay_pair_params(index, seed)
    a = inputs.exp_decay_torch(n, aa, sa, device)
    b = inputs.exp_decay_torch(n, ab, sb, device)
    return Problem.build(a, b, leaf, ws=ws, e=e)


def generate(count: int, n: int, leaf: int, device, *, first: int = 0, seed: int = 7,
             lo: float = 1e-6, hi: float = 1e-2, log=None):
    """Features X [count, 129] (device), labels log10(tau) [count] (device), and
    per-pair records (target, tau, error, evaluations)."""
    x = torch.empty((count, 129), dtype=torch.float32, device=device)
    t = torch.empty(count, dtype=torch.float32, device=device)
    ws = sp.workspace(n, leaf, device)
    e = torch.empty((n, n), dtype=torch.float32, device=device)
    recs = []
    t0 = time.perf_counter()
    for q in range(count):
        idx = first + q
        target = inputs.log_uniform_target(idx, lo, hi)
        pr = decay_problem(n, idx, leaf, device, seed=seed, ws=ws, e=e)
        pr.features(target, out=x[q])
        tau, err, pairs, evals = pr.search(target)
        if not tau > 0.0:
            raise RuntimeError(f"pair {idx}: no positive threshold")
        t[q] = math.log10(tau)
        recs.append({"index": idx, "target": target, "tau": tau, "err": err, "pairs": pairs, "evals": evals})
        if log and (q + 1) % 500 == 0:
            log(f"labels {q + 1}/{count} ({time.perf_counter() - t0:.1f}s)")
    return x, t, recs


def train(x: torch.Tensor, t: torch.Tensor, *, epochs: int = 300, batch: int = 256, lr: float = 1e-3,
          seed: int = 0, params=None, log=None):
    """Adam on the mean squared log10(tau) error; returns (params, per-epoch loss)."""
    dev = x.device
    p = torch.from_numpy(inputs.mlp_init(seed)).to(dev) if params is None else params.clone()
    m, v = torch.zeros_like(p), torch.zeros_like(p)
    acts = sp.mlp_acts(batch, dev)
    grad = torch.empty_like(p)
    loss = torch.empty(1, dtype=torch.float32, device=dev)
    count = x.shape[0]
    rng = np.random.default_rng(seed)
    hist, step = [], 0
    for ep in range(epochs):
        order = torch.from_numpy(rng.permutation(count)).to(dev)
        tot = torch.zeros(1, dtype=torch.float32, device=dev)
        nb = 0
        for s0 in range(0, count - batch + 1, batch):  # full batches only
            idx = order[s0 : s0 + batch]
            xb, tb = x.index_select(0, idx), t.index_select(0, idx)
            sp.mlp_loss_grad(p, xb, tb, acts=acts, grad=grad, loss=loss)
            step += 1
            sp.mlp_adam(p, grad, m, v, step, lr)
            tot += loss
            nb += 1
        hist.append(float(tot.item()) / max(1, nb))
        if log and (ep + 1) % 50 == 0:
            log(f"epoch {ep + 1}/{epochs}: train mse {hist[-1]:.4f}")
    return p, hist


def predict_log10_tau(params: torch.Tensor, x: torch.Tensor) -> torch.Tensor:
    return sp.mlp_forward(params, x.reshape(-1, 129))


def load_params(device, path: Path = PARAMS_FILE) -> torch.Tensor:
    arr = np.load(path, allow_pickle=False)
    if arr.dtype != np.float32 or arr.shape != (sp.mlp_param_count(),):
        raise ValueError(f"{path}: expected {sp.mlp_param_count()} float32 parameters")
    return torch.from_numpy(arr).to(device)


def compare(params: torch.Tensor, problems, targets, *, max_evals: int = 64):
    """For each (problem, target): the search from scratch against the search
    seeded with the network's prediction, and the prediction on its own."""
    rows = []
    feat = torch.empty(129, dtype=torch.float32, device=params.device)
    for pr, target in zip(problems, targets):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        tau0, err0, pairs0, ev0 = pr.search(target, max_evals=max_evals)
        t1 = time.perf_counter()
        pr.features(target, out=feat)
        guess = 10.0 ** float(predict_log10_tau(params, feat).item())
        tau1, err1, pairs1, ev1 = pr.search(target, guess=guess, max_evals=max_evals)
        t2 = time.perf_counter()
        err_g, dropped_g = pr.error(guess)
        total = sp.bdim(pr.n, pr.leaf) ** 3
        rows.append({
            "n": pr.n, "target": target, "tau": tau0, "tau_seeded": tau1, "err": err0, "err_seeded": err1,
            "evals_scratch": ev0,
            "evals_seeded": ev1, "ms_scratch": 1e3 * (t1 - t0), "ms_seeded": 1e3 * (t2 - t1),
            "tau_pred": guess, "log10_ratio_pred": math.log10(guess / tau0) if tau0 > 0 else None,
            "err_pred": err_g, "pred_meets_target": err_g <= target,
            "valid_ratio_opt": pairs0 / total, "valid_ratio_pred": (total - dropped_g) / total,
        })
    return rows


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--pairs", type=int, default=10000)
    ap.add_argument("--holdout", type=int, default=500)
    ap.add_argument("--n", type=int, default=2048)
    ap.add_argument("--leaf", type=int, default=64)
    ap.add_argument("--epochs", type=int, default=300)
    ap.add_argument("--eval-n", type=int, default=8192)
    ap.add_argument("--eval-pairs", type=int, default=32)
    ap.add_argument("--eval-target", type=float, default=1e-4)
    ap.add_argument("--out", default="learned_out", help="folder for the network, the report and the training data")
    args = ap.parse_args(argv)

    def log(msg):
        print(f"[learned_tau] {msg}", file=sys.stderr, flush=True)

    if not torch.cuda.is_available():
        log("needs a GPU")
        return 2
    dev = torch.device("cuda", 0)
    out = Path(args.out)
    out.mkdir(parents=True, exist_ok=True)
    t0 = time.perf_counter()
    x, t, recs = generate(args.pairs + args.holdout, args.n, args.leaf, dev, log=log)
    t_gen = time.perf_counter() - t0
    log(f"{len(recs)} labels in {t_gen:.1f}s; mean evaluations {np.mean([r['evals'] for r in recs]):.1f}")
    xt, tt = x[: args.pairs], t[: args.pairs]
    xh, th = x[args.pairs :], t[args.pairs :]
    t1 = time.perf_counter()
    params, hist = train(xt, tt, epochs=args.epochs, log=log)
    t_train = time.perf_counter() - t1
    np.save(out / "tau_mlp.npy", params.cpu().numpy())
    pred = predict_log10_tau(params, xh).cpu().numpy()
    resid = pred - th.cpu().numpy()
    log(f"held-out |log10 tau error|: median {np.median(np.abs(resid)):.3f}, 90% {np.quantile(np.abs(resid), 0.9):.3f}")

    # held-out problems: seeded search against search from scratch
    hold = [decay_problem(args.n, args.pairs + q, args.leaf, dev) for q in range(min(50, args.holdout))]
    rows_h = compare(params, hold, [inputs.log_uniform_target(args.pairs + q) for q in range(len(hold))])
    # the evaluation size, at the evaluation target
    evp = [decay_problem(args.eval_n, 10**6 + q, args.leaf, dev) for q in range(args.eval_pairs)]
    rows_e = compare(params, evp, [args.eval_target] * len(evp))

    def summary(rows):
        return {
            "problems": len(rows),
            "evals_scratch_mean": float(np.mean([r["evals_scratch"] for r in rows])),
            "evals_seeded_mean": float(np.mean([r["evals_seeded"] for r in rows])),
            "ms_scratch_mean": float(np.mean([r["ms_scratch"] for r in rows])),
            "ms_seeded_mean": float(np.mean([r["ms_seeded"] for r in rows])),
            "same_tau": int(sum(r["tau"] == r["tau_seeded"] for r in rows)),
            "pred_meets_target": int(sum(r["pred_meets_target"] for r in rows)),
            "median_abs_log10_pred_error": float(np.median([abs(r["log10_ratio_pred"]) for r in rows])),
        }

    report = {
        "train": {"pairs": args.pairs, "n": args.n, "leaf": args.leaf, "epochs": args.epochs,
                  "label_seconds": t_gen, "train_seconds": t_train, "final_mse": hist[-1],
                  "mse_history_every_50": hist[49::50],
                  "label_evals_mean": float(np.mean([r["evals"] for r in recs]))},
        "holdout_log10_abs_error": {"median": float(np.median(np.abs(resid))),
                                    "p90": float(np.quantile(np.abs(resid), 0.9)), "count": int(resid.size)},
        "holdout_search": summary(rows_h),
        "eval": {"n": args.eval_n, "target": args.eval_target, **summary(rows_e), "rows": rows_e},
    }
    (out / "learned_tau.json").write_text(json.dumps(report, indent=1) + "\n")
    print(json.dumps({k: v for k, v in report.items() if k != "eval"} | {"eval": summary(rows_e)}), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
