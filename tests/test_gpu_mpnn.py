"""GPU parity of the learned warm start against the CPU oracle of the network.

The oracle runs the same network in FP64 and, with bf16_storage=True, rounds
exactly the values the GPU stores in bfloat16.  What remains is FP32 versus
FP64 arithmetic and the rare bf16 rounding that this flips; on these graphs
the bf16 rounding itself moves t̂ by 1.5e-3 to 5e-3 (relative L1) and the
gradient by ≈9e-3 (relative L2).  FP32 sums of a few hundred terms per
value are good to ~1e-6, so the bounds below (5e-5, 2e-4) sit far under the
bf16 effect: a GPU pass that skipped a rounding, or rounded a value the
oracle keeps, fails.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from oracle import mpnn_oracle as mo

pytestmark = pytest.mark.gpu

T_HAT_REL_L1 = 5e-5
GRAD_REL_L2 = 2e-4


def graphs():
    a = synth.chung_lu(20000, 10, 2.1, 61, sigma=1.5)  # hubs up to ~9000 followers
    b = synth.star(3001, 62)                            # one 3000-follower hub
    c = synth.random_small(37, 0.2, 63)                 # fewer users than one tile
    return {"chung_lu": a, "star": b, "small": c}


def rel_l1(a, b):
    return float(np.abs(a - b).sum() / max(np.abs(b).sum(), 1e-300))


def fixed_point(g):
    A, B, c, d = oracle.operator(g.n, g.follower, g.leader, g.lam, g.mu)
    return oracle.power_psi(A, B, c, d, 1e-13)["s"], c


@pytest.mark.parametrize("name", ["chung_lu", "star", "small"])
def test_forward_matches_oracle(gpu_lib, name):
    api = gpu_lib
    g = graphs()[name]
    theta = mo.init_params(5)
    op = api.Operator(g.n, g.follower, g.leader, g.lam, g.mu)
    model = api.Model(theta)
    t_hat, s0 = model.forward(op)
    t_gpu = t_hat.cpu().numpy().astype(np.float64)
    ga = mo.graph_arrays(g.n, g.follower, g.leader, g.lam, g.mu)
    t_ref, _ = mo.forward(theta, ga, bf16_storage=True)
    t_fp64, _ = mo.forward(theta, ga, bf16_storage=False)
    err = rel_l1(t_gpu, t_ref)
    print(f"\n[{name}] t_hat rel L1 vs oracle {err:.2e}, bf16 effect {rel_l1(t_fp64, t_ref):.2e}")
    assert err <= T_HAT_REL_L1, err
    if name != "small":
        assert err <= 0.2 * rel_l1(t_fp64, t_ref)  # the bf16 network is what matches
    np.testing.assert_allclose(s0.cpu().numpy(), ga["c"] * np.exp(t_gpu), rtol=1e-12)
    t2, s2 = model.forward(op)
    assert torch.equal(t_hat, t2) and torch.equal(s0, s2)


@pytest.mark.parametrize("name", ["chung_lu", "star"])
def test_loss_and_gradient_match_oracle(gpu_lib, name):
    api = gpu_lib
    g = graphs()[name]
    theta = mo.init_params(7)
    s, c = fixed_point(g)
    op = api.Operator(g.n, g.follower, g.leader, g.lam, g.mu)
    model = api.Model(theta)
    loss, _ = model.loss_backward(op, torch.tensor(s))
    grad = model.grad().astype(np.float64)
    ga = mo.graph_arrays(g.n, g.follower, g.leader, g.lam, g.mu)
    t, mask = mo.target(s, c)
    loss_ref, grad_ref = mo.loss_and_grad(theta, ga, t, mask, bf16_storage=True)
    assert abs(loss - loss_ref) <= 1e-4 * loss_ref
    err = np.linalg.norm(grad - grad_ref) / np.linalg.norm(grad_ref)
    print(f"\n[{name}] loss {loss:.6f} vs {loss_ref:.6f}, gradient rel L2 {err:.2e}")
    assert err <= GRAD_REL_L2, err
    # every parameter block, not only the large ones
    ref_p, got_p = mo.unpack(grad_ref), mo.unpack(grad)
    for k in ref_p:
        nr = np.linalg.norm(ref_p[k])
        if nr > 0:
            assert np.linalg.norm(got_p[k] - ref_p[k]) <= max(10 * GRAD_REL_L2 * nr, 1e-7), k
    loss2, _ = model.loss_backward(op, torch.tensor(s))
    assert loss2 == loss
    assert np.array_equal(model.grad(), grad.astype(np.float32))


def test_adam_step_matches_oracle(gpu_lib):
    api = gpu_lib
    g = graphs()["chung_lu"]
    theta = mo.init_params(9)
    s, _ = fixed_point(g)
    op = api.Operator(g.n, g.follower, g.leader, g.lam, g.mu)
    model = api.Model(theta)
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    p = theta.copy()
    for step in (1, 2):
        model.loss_backward(op, torch.tensor(s))
        grad = model.grad().astype(np.float64)
        model.adam_step(lr=1e-3)
        p, m, v = mo.adam(p, grad, m, v, step, lr=1e-3)
        got = model.params().astype(np.float64)
        np.testing.assert_allclose(got, p, rtol=0, atol=1e-6)


def test_multi_graph_forward_equals_lone_graphs(gpu_lib):
    """Block-diagonal operator: each graph's t̂ is bitwise its lone forward."""
    api = gpu_lib
    g = synth.multi_graph(5, 300, 2500, 8, 2.2, seed=64, sigma=1.5)
    theta = mo.init_params(11)
    model = api.Model(theta)
    op = api.Operator(g.n, g.follower, g.leader, g.lam, g.mu, node_offsets=g.node_offsets)
    t_all, _ = model.forward(op, want_s0=False)
    t_all = t_all.cpu().numpy()
    for k in range(5):
        lo, hi = int(g.node_offsets[k]), int(g.node_offsets[k + 1])
        sel = (g.follower >= lo) & (g.follower < hi)
        lone = api.Operator(hi - lo, g.follower[sel] - lo, g.leader[sel] - lo, g.lam[lo:hi],
                            g.mu[lo:hi])
        t1, _ = model.forward(lone, want_s0=False)
        assert np.array_equal(t1.cpu().numpy(), t_all[lo:hi]), k


def test_edgeless_graph(gpu_lib):
    api = gpu_lib
    n = 130
    lam = np.linspace(0.5, 2.0, n)
    mu = np.linspace(1.5, 0.0, n)  # one user with μ = 0 (c = 0)
    e = np.zeros(0, dtype=np.int32)
    theta = mo.init_params(13)
    op = api.Operator(n, e, e, lam, mu)
    model = api.Model(theta)
    t_hat, s0 = model.forward(op)
    ga = mo.graph_arrays(n, e, e, lam, mu)
    t_ref, _ = mo.forward(theta, ga, bf16_storage=True)
    assert rel_l1(t_hat.cpu().numpy().astype(np.float64), t_ref) <= T_HAT_REL_L1
    assert s0.cpu().numpy()[-1] == 0.0


def test_invalid_calls(gpu_lib):
    api = gpu_lib
    with pytest.raises(ValueError):
        api.Model(np.zeros(10, dtype=np.float32))
    g = graphs()["small"]
    model = api.Model(mo.init_params(1))
    op = api.Operator(g.n, g.follower, g.leader, g.lam, g.mu)
    lib = api.load()
    ws = torch.empty(16, dtype=torch.uint8, device="cuda")
    s0 = torch.empty(g.n, dtype=torch.float64, device="cuda")
    st = api._stream_handle(None)
    assert lib.psi_warmstart(model._h, op.handle, s0.data_ptr(), ws.data_ptr(), 16, st) == 6
    assert lib.psi_mpnn_adam_step(model._h, -1.0, 0.9, 0.999, 1e-8, st) == 1


def test_trained_warm_start_saves_iterations(gpu_lib):
    """Train on solver targets of a few graphs, then warm-start a held-out one."""
    api = gpu_lib
    train = [synth.chung_lu(20000, 12, 2.2, 70 + k, sigma=1.5) for k in range(6)]
    ops, targets = [], []
    for g in train:
        op = api.Operator(g.n, g.follower, g.leader, g.lam, g.mu)
        _, s, _ = op.solve(tol=1e-12, return_s=True)
        ops.append(op)
        targets.append(s)
    model = api.Model(mo.init_params(17))
    first = None
    steps = 3000
    for step in range(steps):
        k = step % len(ops)
        loss, _ = model.loss_backward(ops[k], targets[k])
        if step < len(ops):
            first = loss if first is None else max(first, loss)
        model.adam_step(lr=3e-3 * 0.5 * (1 + np.cos(np.pi * step / steps)) + 1e-5)
    last = np.mean([model.loss_backward(op, t)[0] for op, t in zip(ops, targets)])
    assert last < 0.2 * first, (first, last)

    h = synth.chung_lu(30000, 12, 2.2, 99, sigma=1.5)
    op = api.Operator(h.n, h.follower, h.leader, h.lam, h.mu)
    cold_psi, cold = op.solve(tol=1e-10)
    s0 = model.warmstart(op)
    warm_psi, warm = op.solve(tol=1e-10, s0=s0)
    print(f"warm start: {warm['iterations']} iterations vs {cold['iterations']} cold; "
          f"training loss {first:.4f} -> {last:.4f}")
    assert warm["used_s0"] == 1
    assert warm["iterations"] <= cold["iterations"] - 2, (warm, cold)
    assert rel_l1(warm_psi.cpu().numpy(), cold_psi.cpu().numpy()) <= 1e-9
