"""Parity at the full sizes of the benchmark configurations.

Where the whole oracle fits (the 64-scenario batch's first scenario, the
graphs of the 256-graph batch) it runs in full and the bar is 1e-9 relative
L1.  Where it does not (40M users / 1.4G edges, 10M users / 200M edges), the
oracle evaluates the definitions at sampled users one by one
(oracle.sampled_rows): the fixed-point residual of the GPU's s must be
within the solve's tolerance at every sampled user (a converged solve has
‖Aᵀs + c − s‖₁ ≲ tol over all users), and the GPU's ψ must be the last line
of Algorithm 2 applied to that s.  Invariants that hold at any size (s ≥ c,
ψ ≥ d/N, Σψ ≤ 1) are checked on every user.  Inputs are drawn on the GPU by
the torch twin of the generator (the same values as the NumPy generator).
"""
import os

import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

WEIGHTS = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                       "paper_2206_09960_amd", "weights", "warmstart_cl.npy")


def say(msg):
    print(f"\n[fullsize] {msg}", flush=True)


def sample(row_len, k, seed, n_hubs=1):
    rng = np.random.default_rng(seed)
    rows = rng.choice(row_len.size, k, replace=False)
    top = np.argsort(row_len)[-n_hubs:]
    return np.unique(np.concatenate([rows, top]))


def check_invariants(psi, s, lam, mu):
    c = mu / (lam + mu)
    d = lam / (lam + mu)
    n = psi.size
    assert np.all(s >= c * (1 - 1e-15))
    assert np.all(psi >= d / n * (1 - 1e-15))
    assert psi.sum() <= 1 + 1e-9


def check_sampled(n, f, l, lam, mu, s, psi, rows, tol):
    res, psi_rows = oracle.sampled_rows(n, f, l, lam, mu, s, rows)
    slack = tol + 1e-13 * np.abs(s[rows])
    bad = np.abs(res) > slack
    assert not bad.any(), (rows[bad], res[bad])
    np.testing.assert_allclose(psi[rows], psi_rows, rtol=1e-12, atol=0)
    return float(np.abs(res).max())


@pytest.mark.timeout(600)
def test_c5_warm_start_10m_users(gpu_lib):
    api = gpu_lib
    tol = synth.WORKLOADS["cl_10m"]["tol"]
    say("C5: drawing 10M users / 200M edges")
    g = synth.workload("cl_10m", device="cuda")
    op = api.Operator(g.n, g.follower, g.leader, torch.from_numpy(g.lam).cuda(),
                      torch.from_numpy(g.mu).cuda())
    f = g.follower.cpu().numpy()
    l = g.leader.cpu().numpy()
    g.follower = g.leader = None
    op.autotune("fp64")  # the schedule the benchmark times
    psi_c, s_c, cold = op.solve(tol=tol, return_s=True)
    model = api.Model(np.load(WEIGHTS))
    s0 = model.warmstart(op)
    psi_w, s_w, warm = op.solve(tol=tol, s0=s0, return_s=True)
    assert cold["status"] == 0 and warm["status"] == 0
    say(f"C5: warm start {warm['iterations']} iterations (used_s0={warm['used_s0']}) vs cold "
        f"{cold['iterations']}")
    psi_c, s_c, psi_w, s_w = (t.cpu().numpy() for t in (psi_c, s_c, psi_w, s_w))
    assert oracle.rel_l1(psi_c, psi_w) <= 1e-9  # one fixed point, whatever the start
    check_invariants(psi_w, s_w, g.lam, g.mu)
    row_len = np.diff(op.views()["row_ptr"].cpu().numpy())
    rows = sample(row_len, 48, 5, n_hubs=1)
    check_sampled(g.n, f, l, g.lam, g.mu, s_w, psi_w, rows, tol)


@pytest.mark.timeout(900)
def test_c4a_64_scenarios_full_oracle_on_one(gpu_lib):
    api = gpu_lib
    wl = synth.WORKLOADS["cl_4m_k64"]
    tol, k = wl["tol"], wl["scenarios"]
    say("C4a: drawing N=4M / 80M edges and 64 scenarios")
    g = synth.workload("cl_4m_k64", device="cuda")
    lam = np.empty((g.n, k))
    mu = np.empty((g.n, k))
    for j in range(k):
        lam[:, j], mu[:, j] = synth.activity(g.n, wl["seed"], "lognormal", wl["sigma"], scenario=j)
    op = api.Operator(g.n, g.follower, g.leader, g.lam, g.mu)
    lam_d, mu_d = torch.from_numpy(lam).cuda(), torch.from_numpy(mu).cuda()
    psi, infos = op.solve_batched(lam_d, mu_d, tol=tol)
    psi = psi.cpu().numpy()
    assert all(i["status"] == 0 for i in infos)
    say(f"C4a: passes per scenario {min(i['spmv_passes'] for i in infos)}.."
        f"{max(i['spmv_passes'] for i in infos)}")
    # mixed precision: every scenario meets its FP64 gap and matches the FP64 batch
    psi_m, infos_m = op.solve_batched(lam_d, mu_d, tol=tol, precision="mixed")
    del lam_d, mu_d
    assert all(i["status"] == 0 and i["final_gap"] <= tol for i in infos_m)
    err_m = oracle.rel_l1(psi, psi_m.cpu().numpy())
    say(f"C4a: mixed vs FP64 batch rel L1 {err_m:.2e}, FP32 passes "
        f"{max(i['fp32_passes'] for i in infos_m)}, FP64 passes "
        f"{max(i['iterations'] for i in infos_m)}")
    assert err_m <= 1e-9
    del psi_m
    # the last scenario against its lone single-graph solve
    lone = api.Operator(g.n, g.follower, g.leader, lam[:, k - 1], mu[:, k - 1])
    p1, i1 = lone.solve(tol=tol)
    assert oracle.rel_l1(p1.cpu().numpy(), psi[:, k - 1]) <= 1e-12
    del lone
    f = g.follower.cpu().numpy()
    l = g.leader.cpu().numpy()
    g.follower = g.leader = None
    A, B, c, d = oracle.operator(g.n, f, l, lam[:, 0], mu[:, 0])
    r = oracle.power_psi(A, B, c, d, tol)
    err = oracle.rel_l1(r["psi"], psi[:, 0])
    say(f"C4a: scenario 0 vs full oracle rel L1 {err:.2e}")
    assert err <= 1e-9
    assert abs(r["iterations"] - infos[0]["iterations"]) <= 1


@pytest.mark.timeout(600)
def test_c4b_256_graphs_full_oracle_on_samples(gpu_lib):
    api = gpu_lib
    wl = synth.WORKLOADS["graphs256"]
    say("C4b: drawing 256 graphs")
    g = synth.workload("graphs256", device="cuda")
    op = api.Operator(g.n, g.follower, g.leader, g.lam, g.mu, node_offsets=g.node_offsets)
    g.follower = g.leader = None
    psi, infos = op.solve_graphs(tol=wl["tol"])
    psi = psi.cpu().numpy()
    assert len(infos) == 256 and all(i["status"] == 0 for i in infos)
    sizes = np.diff(g.node_offsets)
    picks = sorted({0, 128, 255, int(np.argmax(sizes)), int(np.argmin(sizes))})
    for k in picks:
        lo, hi = int(g.node_offsets[k]), int(g.node_offsets[k + 1])
        sub = synth.chung_lu(hi - lo, wl["mean_degree"], wl["gamma"], 1000 * wl["seed"] + k,
                             wl["sigma"])
        A, B, c, d = oracle.operator(sub.n, sub.follower, sub.leader, sub.lam, sub.mu)
        r = oracle.power_psi(A, B, c, d, wl["tol"])
        err = oracle.rel_l1(r["psi"], psi[lo:hi])
        assert err <= 1e-9, (k, err)
        assert abs(r["iterations"] - infos[k]["iterations"]) <= 1, k
    say(f"C4b: graphs {picks} match the full oracle")


@pytest.mark.timeout(900)
def test_c3_40m_users_hub_rows(gpu_lib):
    api = gpu_lib
    tol = synth.WORKLOADS["cl_40m"]["tol"]
    say("C3: drawing 40M users / 1.4G edges")
    g = synth.workload("cl_40m", device="cuda")
    op = api.Operator(g.n, g.follower, g.leader, torch.from_numpy(g.lam).cuda(),
                      torch.from_numpy(g.mu).cuda())
    f = g.follower.cpu().numpy()
    l = g.leader.cpu().numpy()
    g.follower = g.leader = None
    torch.cuda.empty_cache()
    st = op.stats()
    say(f"C3: built M={st['n_edges']} max_followers={st['max_followers']}")
    assert 1_000_000 < st["max_followers"] <= 3_000_000
    for prec in ("fp64", "mixed"):  # the schedules the benchmark times
        op.autotune(prec)
    psi64, s64, i64 = op.solve(tol=tol, return_s=True)
    psim, sm, im = op.solve(tol=tol, precision="mixed", return_s=True)
    assert i64["status"] == 0 and im["status"] == 0, (i64, im)
    say(f"C3: fp64 {i64['iterations']} iterations, mixed {im['spmv_passes']} passes")
    psi64, s64, psim, sm = (t.cpu().numpy() for t in (psi64, s64, psim, sm))
    assert oracle.rel_l1(psi64, psim) <= 1e-6
    check_invariants(psi64, s64, g.lam, g.mu)
    row_len = np.diff(op.views()["row_ptr"].cpu().numpy())
    rows = sample(row_len, 48, 3, n_hubs=1)
    r64 = check_sampled(g.n, f, l, g.lam, g.mu, s64, psi64, rows, tol)
    rm = check_sampled(g.n, f, l, g.lam, g.mu, sm, psim, rows, tol)
    say(f"C3: max sampled |residual| fp64 {r64:.2e}, mixed {rm:.2e}")
