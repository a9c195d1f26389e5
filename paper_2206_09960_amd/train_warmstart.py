"""Training driver of the learned warm start.

Targets are fixed points s of eq. (power_psi), computed by psi_solve on
synthetic directed Chung–Lu graphs of the family the model will serve; the
loss and its gradient (psi_mpnn_loss_backward) and the Adam update
(psi_mpnn_adam_step) run in the library's kernels.  The learning rate
follows a cosine schedule.  Writes the FP32 parameter vector (.npy) and a
JSON record of the run next to it.

Two modes: a fixed set of graphs held on the GPU and cycled (--graphs), or
(--stream) a stream of graphs, each drawn on the GPU (its N-sized host part
prepared ahead by worker threads), built, solved for its target, used for a
few steps and freed, so that thousands of graphs of up to 10^6 users fit.
A held-out set of the same family reports the loss and the iterations a
warm start saves.

    python -m paper_2206_09960_amd.train_warmstart --out weights/warmstart_cl.npy
    python -m paper_2206_09960_amd.train_warmstart --stream --graphs 2000 \
        --n-lo 100000 --n-hi 1000000 --out weights/warmstart_cl.npy
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


def stream_specs(n_graphs: int, n_lo: int, n_hi: int, degree: float, seed: int):
    """(N, edges drawn, seed) of each graph of a stream: N uniform in [n_lo, n_hi]."""
    rng = np.random.default_rng(seed)
    sizes = rng.integers(n_lo, n_hi + 1, n_graphs)
    return [(int(n), int(round(n * degree)), 10_000 * seed + k) for k, n in enumerate(sizes)]


def _host_part(spec, gamma: float, sigma: float):
    import synth
    n, m, sd = spec
    plan = synth.chung_lu_plan(n, m, gamma, sd)
    lam, mu = synth.activity(n, sd, "lognormal", sigma)
    return plan, lam, mu


def _stream(specs, gamma: float, sigma: float, workers: int):
    """Yields (spec, operator inputs on the GPU) in order; host parts are
    prepared `2·workers` graphs ahead by a thread pool."""
    from concurrent.futures import ThreadPoolExecutor

    import torch

    import synth
    with ThreadPoolExecutor(max_workers=workers) as pool:
        ahead = 2 * workers
        futs = [pool.submit(_host_part, sp, gamma, sigma) for sp in specs[:ahead]]
        for i, sp in enumerate(specs):
            plan, lam, mu = futs[i].result()
            futs[i] = None
            if i + ahead < len(specs):
                futs.append(pool.submit(_host_part, specs[i + ahead], gamma, sigma))
            n, m, sd = sp
            f, l = synth.chung_lu_edges_torch(n, m, gamma, sd, device="cuda", plan=plan)
            yield sp, (f, l, torch.from_numpy(lam).cuda(), torch.from_numpy(mu).cuda())


def evaluate(model, specs, gamma: float, sigma: float, tol: float = 1e-9,
             solve_tol: float = 1e-8, workers: int = 8):
    """Loss on held-out graphs and the iterations a warm start saves there
    (cold solve from c against the solve from the model's s_0, to solve_tol)."""
    from . import api
    out = []
    for (n, m, sd), (f, l, lam, mu) in _stream(specs, gamma, sigma, workers):
        op = api.Operator(n, f, l, lam, mu)
        del f, l
        _, s, _ = op.solve(tol=tol, return_s=True)
        loss, _ = model.loss_backward(op, s)
        _, cold = op.solve(tol=solve_tol)
        _, warm = op.solve(tol=solve_tol, s0=model.warmstart(op))
        out.append(dict(n=n, loss=round(float(loss), 6), iterations_cold=cold["iterations"],
                        iterations_warm=warm["iterations"], used_s0=warm["used_s0"]))
        op.close()
    return out


def train_stream(specs, gamma: float, sigma: float, steps_per_graph: int = 2, lr: float = 3e-3,
                 seed: int = 17, tol: float = 1e-9, workers: int = 8, max_seconds: float = 0.0,
                 log=print):
    """One pass over a stream of graphs, `steps_per_graph` Adam steps on each;
    returns (params, record)."""
    import torch

    from . import api
    api.load()
    model = api.Model(initial_params(seed))
    total = len(specs) * steps_per_graph
    step, used, history, sizes, edges = 0, 0, [], [], 0
    t0 = last = time.perf_counter()
    for (n, m, sd), (f, l, lam, mu) in _stream(specs, gamma, sigma, workers):
        op = api.Operator(n, f, l, lam, mu)
        del f, l
        _, s, info = op.solve(tol=tol, return_s=True)
        if info["status"] != 0:
            raise RuntimeError(f"target solve failed: {info['status_name']}")
        for _ in range(steps_per_graph):
            loss, _ = model.loss_backward(op, s)
            history.append(loss)
            model.adam_step(lr=lr * 0.5 * (1.0 + np.cos(np.pi * step / total)) + 1e-5)
            step += 1
        edges += int(op.stats()["n_edges"])
        sizes.append(n)
        op.close()
        del s
        used += 1
        now = time.perf_counter()
        if now - last >= 30.0:
            log(f"[train] graph {used}/{len(specs)} step {step} mean loss "
                f"{np.mean(history[-200:]):.5f} ({now - t0:.0f}s)")
            last = now
        if max_seconds and now - t0 >= max_seconds:
            log(f"[train] stopping at {max_seconds:.0f}s after {used} graphs")
            break
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    record = dict(mode="stream", steps=step, steps_per_graph=steps_per_graph, lr=lr, seed=seed,
                  n_graphs=used, n_graphs_planned=len(specs), n_users_min=int(min(sizes)),
                  n_users_max=int(max(sizes)), n_users_mean=float(np.mean(sizes)),
                  n_edges_total=edges, target_tol=tol, seconds_train=round(t_train, 2),
                  ms_per_graph=round(1e3 * t_train / max(used, 1), 2),
                  first_losses=[round(float(x), 5) for x in history[:20]],
                  last_losses_mean=float(np.mean(history[-200:])))
    return model, record


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
    ap.add_argument("--stream", action="store_true",
                    help="one pass over a stream of graphs drawn on the GPU")
    ap.add_argument("--steps-per-graph", type=int, default=2)
    ap.add_argument("--max-seconds", type=float, default=0.0)
    ap.add_argument("--workers", type=int, default=8)
    ap.add_argument("--holdout", type=int, default=8)
    args = ap.parse_args()
    if args.stream:
        specs = stream_specs(args.graphs, args.n_lo, args.n_hi, args.degree, args.seed)
        model, rec = train_stream(specs, args.gamma, args.sigma, args.steps_per_graph, args.lr,
                                  args.seed, workers=args.workers, max_seconds=args.max_seconds,
                                  log=lambda m: print(m, flush=True))
        held = stream_specs(args.holdout, args.n_lo, args.n_hi, args.degree, args.seed + 1000)
        rec["holdout"] = evaluate(model, held, args.gamma, args.sigma, workers=args.workers)
        print(f"[train] held-out: {rec['holdout']}", flush=True)
        rec.update(family=dict(kind="directed Chung-Lu", degree=args.degree, gamma=args.gamma,
                               sigma=args.sigma, n_lo=args.n_lo, n_hi=args.n_hi,
                               graph_seed=args.seed, holdout_seed=args.seed + 1000))
        params = model.params()
        os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
        np.save(args.out, params)
        with open(os.path.splitext(args.out)[0] + ".json", "w") as fh:
            json.dump(rec, fh, indent=1)
        print(json.dumps({k: rec[k] for k in ("n_graphs", "steps", "seconds_train",
                                              "last_losses_mean")}), flush=True)
        return 0
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
