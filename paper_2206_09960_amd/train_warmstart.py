"""Training driver of the learned warm start.

Targets are fixed points s of eq. (power_psi), computed by psi_solve on
synthetic directed Chung–Lu graphs of the family the model will serve; the
loss and its gradient (psi_mpnn_loss_backward) and the Adam update
(psi_mpnn_adam_step) run in the library's kernels.  The learning rate
follows a cosine schedule.  Writes the FP32 parameter vector (.npy) and a
JSON record of the run next to it.

    python -m paper_2206_09960_amd.train_warmstart --out weights/warmstart_cl.npy
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

F0, H, MSG, LAYERS = 8, 64, 32, 3


def initial_params(seed: int) -> np.ndarray:
    """He-style initial weights, zero biases, in the order psi.h documents."""
    rng = np.random.default_rng(seed)
    parts = [rng.normal(0.0, np.sqrt(2.0 / F0), F0 * H), np.zeros(H)]
    for _ in range(LAYERS):
        parts += [rng.normal(0.0, np.sqrt(1.0 / H), H * MSG),
                  rng.normal(0.0, np.sqrt(2.0 / (H + MSG)), (H + MSG) * H), np.zeros(H)]
    parts += [rng.normal(0.0, np.sqrt(1.0 / H), H), np.zeros(1)]
    return np.concatenate(parts).astype(np.float32)


def make_graphs(n_graphs: int, n_lo: int, n_hi: int, degree: float, gamma: float, sigma: float,
                seed: int):
    import synth
    rng = np.random.default_rng(seed)
    sizes = rng.integers(n_lo, n_hi + 1, n_graphs)
    return [synth.chung_lu(int(n), degree, gamma, 10_000 * seed + k, sigma=sigma)
            for k, n in enumerate(sizes)]


def train(graphs, steps: int = 4000, lr: float = 3e-3, seed: int = 17, tol: float = 1e-9,
          log_every: int = 500, log=print):
    """Returns (params, record)."""
    import torch

    from . import api
    api.load()
    ops, targets = [], []
    t0 = time.perf_counter()
    for g in graphs:
        op = api.Operator(g.n, g.follower, g.leader, g.lam, g.mu)
        _, s, info = op.solve(tol=tol, return_s=True)
        if info["status"] != 0:
            raise RuntimeError(f"target solve failed: {info['status_name']}")
        ops.append(op)
        targets.append(s)
    t_targets = time.perf_counter() - t0
    model = api.Model(initial_params(seed))
    rng = np.random.default_rng(seed)
    order = []
    history = []
    t0 = time.perf_counter()
    for step in range(steps):
        if not order:
            order = list(rng.permutation(len(ops)))
        k = order.pop()
        loss, _ = model.loss_backward(ops[k], targets[k])
        history.append(loss)
        model.adam_step(lr=lr * 0.5 * (1.0 + np.cos(np.pi * step / steps)) + 1e-5)
        if log_every and (step + 1) % log_every == 0:
            log(f"[train] step {step + 1}/{steps} mean loss {np.mean(history[-log_every:]):.5f}")
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    final = [model.loss_backward(op, s)[0] for op, s in zip(ops, targets)]
    record = dict(steps=steps, lr=lr, seed=seed, n_graphs=len(graphs),
                  n_users=[int(g.n) for g in graphs],
                  n_edges=[int(op.stats()["n_edges"]) for op in ops],
                  target_tol=tol, seconds_targets=round(t_targets, 2),
                  seconds_train=round(t_train, 2), ms_per_step=round(1e3 * t_train / steps, 3),
                  first_losses=[round(float(x), 5) for x in history[:len(ops)]],
                  final_loss_mean=float(np.mean(final)))
    return model.params(), record


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--graphs", type=int, default=24)
    ap.add_argument("--n-lo", type=int, default=100_000)
    ap.add_argument("--n-hi", type=int, default=300_000)
    ap.add_argument("--degree", type=float, default=20.0)
    ap.add_argument("--gamma", type=float, default=2.2)
    ap.add_argument("--sigma", type=float, default=1.5)
    ap.add_argument("--steps", type=int, default=4000)
    ap.add_argument("--lr", type=float, default=3e-3)
    ap.add_argument("--seed", type=int, default=17)
    args = ap.parse_args()
    t0 = time.perf_counter()
    graphs = make_graphs(args.graphs, args.n_lo, args.n_hi, args.degree, args.gamma, args.sigma,
                         args.seed)
    print(f"[train] {len(graphs)} graphs generated in {time.perf_counter() - t0:.1f}s", flush=True)
    params, rec = train(graphs, steps=args.steps, lr=args.lr, seed=args.seed,
                        log=lambda m: print(m, flush=True))
    rec.update(family=dict(kind="directed Chung-Lu", degree=args.degree, gamma=args.gamma,
                           sigma=args.sigma, n_lo=args.n_lo, n_hi=args.n_hi,
                           graph_seed=args.seed))
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    np.save(args.out, params)
    with open(os.path.splitext(args.out)[0] + ".json", "w") as fh:
        json.dump(rec, fh, indent=1)
    print(json.dumps({k: rec[k] for k in ("steps", "ms_per_step", "seconds_train",
                                          "final_loss_mean")}), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
