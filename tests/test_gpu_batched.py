"""GPU parity of the batched solves against the CPU oracle and single solves.

Scenario mode: K activity scenarios on one graph; column k must match the
oracle's Algorithm 2 for scenario k (1e-9 relative L1) and the single-graph
solve of that scenario.
"""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu


def scenarios(n, k, seed, sigma=1.5):
    lam = np.empty((n, k))
    mu = np.empty((n, k))
    for s in range(k):
        lam[:, s], mu[:, s] = synth.activity(n, seed, "lognormal", sigma, scenario=s)
    return lam, mu


@pytest.mark.parametrize("n,k,gamma", [(20000, 5, 2.2), (3000, 70, 2.1), (50000, 64, 2.2)])
def test_scenarios_match_oracle(gpu_lib, n, k, gamma):
    api = gpu_lib
    g = synth.chung_lu(n, 15, gamma, 41, sigma=1.5)
    lam, mu = scenarios(n, k, 42)
    op = api.Operator(g.n, g.follower, g.leader, g.lam, g.mu)
    psi, infos = op.solve_batched(torch.tensor(lam), torch.tensor(mu), tol=1e-9)
    psi = psi.cpu().numpy()
    for s in sorted({0, 1, k // 2, k - 1}):
        A, B, c, d = oracle.operator(g.n, g.follower, g.leader, lam[:, s], mu[:, s])
        r = oracle.power_psi(A, B, c, d, 1e-9)
        assert infos[s]["status"] == 0
        assert abs(infos[s]["iterations"] - r["iterations"]) <= 1
        assert oracle.rel_l1(r["psi"], psi[:, s]) <= 1e-9, s


def test_scenarios_equal_single_solves_and_repeat(gpu_lib):
    api = gpu_lib
    g = synth.chung_lu(30000, 20, 2.2, 43, sigma=1.0)
    k = 6
    lam, mu = scenarios(g.n, k, 44, sigma=2.0)
    op = api.Operator(g.n, g.follower, g.leader, g.lam, g.mu)
    psi, infos = op.solve_batched(torch.tensor(lam), torch.tensor(mu), tol=1e-10)
    again, _ = op.solve_batched(torch.tensor(lam), torch.tensor(mu), tol=1e-10)
    assert torch.equal(psi, again)
    for s in range(k):
        single = api.Operator(g.n, g.follower, g.leader, lam[:, s], mu[:, s])
        p1, info = single.solve(tol=1e-10)
        assert abs(info["iterations"] - infos[s]["iterations"]) <= 1
        assert oracle.rel_l1(p1.cpu().numpy(), psi[:, s].cpu().numpy()) <= 1e-12


def test_scenarios_star_hub_closed_form(gpu_lib):
    """A 200k-follower hub (chunked rows) in every scenario."""
    api = gpu_lib
    n = 200_001
    g = synth.star(n, 45)
    lam, mu = scenarios(n, 3, 46)
    op = api.Operator(g.n, g.follower, g.leader, g.lam, g.mu)
    psi, infos = op.solve_batched(torch.tensor(lam), torch.tensor(mu), tol=1e-11)
    psi = psi.cpu().numpy()
    for s in range(3):
        c = mu[:, s] / (lam[:, s] + mu[:, s])
        d = lam[:, s] / (lam[:, s] + mu[:, s])
        expect = d / n
        expect[0] = d[0] * (1.0 + np.sort(c[1:]).sum()) / n
        np.testing.assert_allclose(psi[:, s], expect, rtol=1e-12, atol=0)


@pytest.mark.parametrize("prec,tile", [("fp64", 0), ("mixed", 0), ("fp64", 8), ("mixed", 3)])
def test_scenarios_row_length_boundaries(gpu_lib, prec, tile):
    """Rows whose follower counts sit on the batched kernels' boundaries: 16
    gathers in flight, 64 indices per register load, 256 staged indices and
    the 256-follower hub limit (rows above it are chunked)."""
    api = gpu_lib
    n = 6000
    lengths = [0, 1, 2, 15, 16, 17, 31, 32, 33, 63, 64, 65, 127, 128, 129, 255, 256, 257, 300,
               1024, 1025, 3000]
    rng = np.random.default_rng(49)
    follower, leader = [], []
    for i in range(400):
        cnt = lengths[i % len(lengths)]
        fol = rng.choice(n - 1, cnt, replace=False)
        fol[fol >= i] += 1  # no self-loops
        follower.append(fol)
        leader.append(np.full(cnt, i))
    # a sparse background so every user has some leader
    bg_f = rng.integers(0, n, 20000)
    bg_l = rng.integers(400, n, 20000)
    keep = bg_f != bg_l
    follower = np.concatenate(follower + [bg_f[keep]]).astype(np.int32)
    leader = np.concatenate(leader + [bg_l[keep]]).astype(np.int32)
    lam, mu = scenarios(n, 3, 50)
    op = api.Operator(n, follower, leader, lam[:, 0], mu[:, 0])
    psi, infos = op.solve_batched(torch.tensor(lam), torch.tensor(mu), tol=1e-11, precision=prec,
                                  batch_tile=tile)
    assert all(i["batch_tile"] == (tile or 64) for i in infos)
    psi = psi.cpu().numpy()
    for s in range(3):
        A, B, c, d = oracle.operator(n, follower, leader, lam[:, s], mu[:, s])
        r = oracle.power_psi(A, B, c, d, 1e-11)
        assert infos[s]["status"] == 0
        if prec == "fp64":
            assert abs(infos[s]["iterations"] - r["iterations"]) <= 1
        else:  # FP64 residual passes, the last of which met tol
            assert infos[s]["final_gap"] <= 1e-11 and infos[s]["fp32_passes"] > 0
        assert oracle.rel_l1(r["psi"], psi[:, s]) <= 1e-9, s


@pytest.mark.parametrize("n,k,gamma", [(20000, 5, 2.2), (3000, 70, 2.1), (50000, 64, 2.2)])
def test_scenarios_mixed_match_oracle(gpu_lib, n, k, gamma):
    """Mixed precision: FP32 corrections refined by FP64 residual passes; each
    scenario stops on its FP64 gap, so it must match the oracle's Algorithm 2
    at the same tolerance and the FP64 batch."""
    api = gpu_lib
    g = synth.chung_lu(n, 15, gamma, 41, sigma=1.5)
    lam, mu = scenarios(n, k, 42)
    op = api.Operator(g.n, g.follower, g.leader, g.lam, g.mu)
    psi, infos = op.solve_batched(torch.tensor(lam), torch.tensor(mu), tol=1e-9,
                                  precision="mixed")
    psi64, _ = op.solve_batched(torch.tensor(lam), torch.tensor(mu), tol=1e-9)
    again, _ = op.solve_batched(torch.tensor(lam), torch.tensor(mu), tol=1e-9, precision="mixed")
    assert torch.equal(psi, again)
    psi = psi.cpu().numpy()
    assert oracle.rel_l1(psi64.cpu().numpy(), psi) <= 1e-9
    for s in sorted({0, 1, k // 2, k - 1}):
        A, B, c, d = oracle.operator(g.n, g.follower, g.leader, lam[:, s], mu[:, s])
        r = oracle.power_psi(A, B, c, d, 1e-9)
        i = infos[s]
        assert i["status"] == 0 and i["final_gap"] <= 1e-9, i
        assert i["fp32_passes"] > 0 and i["refinements"] >= 1, i
        assert i["spmv_passes"] == i["iterations"] + i["fp32_passes"] + 1
        assert oracle.rel_l1(r["psi"], psi[:, s]) <= 1e-9, s


def test_scenario_schedules_give_the_same_sums(gpu_lib):
    """Scenarios per tile (lane groups of a wave: 64/Kc rows at a time), items
    per wave tile and hub chunk sizes change only the schedule: each row's sum
    keeps its order for a given chunk size, so a scenario that stops at the
    same step has the same bits; every schedule matches the oracle."""
    api = gpu_lib
    g = synth.chung_lu(40_000, 14, 2.05, 61, sigma=1.5)  # hubs of thousands of followers
    k = 20
    lam, mu = scenarios(g.n, k, 62)
    op = api.Operator(g.n, g.follower, g.leader, g.lam, g.mu)
    assert op.stats()["max_followers"] > 2048
    ref, i_ref = op.solve_batched(torch.tensor(lam), torch.tensor(mu), tol=1e-11)
    for tile, items, chunk in [(8, 256, 1024), (16, 128, 1024), (5, 1024, 1024), (20, 512, 1024),
                               (64, 256, 512), (7, 256, 4096)]:
        psi, infos = op.solve_batched(torch.tensor(lam), torch.tensor(mu), tol=1e-11,
                                      batch_tile=tile, batch_items=items, hub_chunk=chunk)
        assert all((i["batch_tile"], i["tile_items"], i["hub_chunk"]) == (tile, items, chunk)
                   for i in infos)
        for s in range(k):
            same_step = infos[s]["iterations"] == i_ref[s]["iterations"]
            if chunk == 1024 and same_step:
                assert torch.equal(psi[:, s], ref[:, s]), (tile, items, s)
            assert abs(infos[s]["iterations"] - i_ref[s]["iterations"]) <= 1
        for s in (0, k - 1):
            A, B, c, d = oracle.operator(g.n, g.follower, g.leader, lam[:, s], mu[:, s])
            r = oracle.power_psi(A, B, c, d, 1e-11)
            assert oracle.rel_l1(r["psi"], psi[:, s].cpu().numpy()) <= 1e-9, (tile, s)
    with pytest.raises(api.PsiError, match="batch_tile"):
        op.solve_batched(torch.tensor(lam), torch.tensor(mu), batch_tile=65)
    with pytest.raises(api.PsiError, match="hub_chunk"):
        op.solve_batched(torch.tensor(lam), torch.tensor(mu), hub_chunk=100)
    with pytest.raises(api.PsiError, match="batch_items"):
        op.solve_batched(torch.tensor(lam), torch.tensor(mu), batch_items=64)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_autotune_batched_schedule_is_used(gpu_lib, prec):
    api = gpu_lib
    g = synth.chung_lu(30_000, 12, 2.1, 63, sigma=1.5)
    k = 24
    lam, mu = scenarios(g.n, k, 64)
    op = api.Operator(g.n, g.follower, g.leader, g.lam, g.mu)
    t = op.autotune_batched(k, prec)
    assert t["batch_tile"] in (8, 16, 24) and t["pass_ms"] > 0
    assert t["batch_items"] in (128, 256, 512, 1024)
    assert t["hub_chunk"] in (512, 1024, 2048, 4096)
    psi, infos = op.solve_batched(torch.tensor(lam), torch.tensor(mu), tol=1e-10, precision=prec)
    assert all((i["batch_tile"], i["tile_items"], i["hub_chunk"]) ==
               (t["batch_tile"], t["batch_items"], t["hub_chunk"]) for i in infos)
    for s in (0, k - 1):
        A, B, c, d = oracle.operator(g.n, g.follower, g.leader, lam[:, s], mu[:, s])
        r = oracle.power_psi(A, B, c, d, 1e-10)
        assert infos[s]["status"] == 0
        assert oracle.rel_l1(r["psi"], psi[:, s].cpu().numpy()) <= 1e-9
    # an explicit schedule still wins over the tuned one
    _, i2 = op.solve_batched(torch.tensor(lam), torch.tensor(mu), tol=1e-10, precision=prec,
                             batch_tile=64)
    assert i2[0]["batch_tile"] == 64


def test_scenarios_mixed_statuses(gpu_lib):
    api = gpu_lib
    g = synth.chung_lu(5000, 10, 2.2, 47)
    lam, mu = scenarios(g.n, 4, 48)
    op = api.Operator(g.n, g.follower, g.leader, g.lam, g.mu)
    bad = lam.copy()
    bad[10, 2] = -1.0
    with pytest.raises(api.PsiError, match="activity"):
        op.solve_batched(torch.tensor(bad), torch.tensor(mu), precision="mixed")
    psi, infos = op.solve_batched(torch.tensor(lam), torch.tensor(mu), tol=1e-14, max_iter=3,
                                  precision="mixed")
    assert all(i["status_name"] == "PSI_ENOTCONV" and i["iterations"] == 3 for i in infos), infos
    with pytest.raises(api.PsiError, match="PSI_PREC"):
        op.solve_batched(torch.tensor(lam), torch.tensor(mu), precision="fp32")


def test_scenarios_invalid_and_statuses(gpu_lib):
    api = gpu_lib
    g = synth.chung_lu(5000, 10, 2.2, 47)
    lam, mu = scenarios(g.n, 4, 48)
    op = api.Operator(g.n, g.follower, g.leader, g.lam, g.mu)
    bad = lam.copy()
    bad[10, 2] = -1.0
    with pytest.raises(api.PsiError, match="activity"):
        op.solve_batched(torch.tensor(bad), torch.tensor(mu))
    psi, infos = op.solve_batched(torch.tensor(lam), torch.tensor(mu), tol=1e-12, max_iter=3)
    assert all(i["status_name"] == "PSI_ENOTCONV" and i["iterations"] == 3 for i in infos)
    with pytest.raises(ValueError):
        op.solve_batched(torch.tensor(lam[:-1]), torch.tensor(mu[:-1]))


# ---------------------------------------------------------------- graph mode
def subgraph(g, k):
    lo, hi = int(g.node_offsets[k]), int(g.node_offsets[k + 1])
    sel = (g.follower >= lo) & (g.follower < hi)
    return synth.Graph(hi - lo, g.follower[sel] - lo, g.leader[sel] - lo, g.lam[lo:hi], g.mu[lo:hi])


@pytest.mark.parametrize("n_graphs,lo,hi", [(7, 500, 3000), (256, 100, 400), (3, 20, 40),
                                             (4, 20000, 40000)])
def test_graphs_match_oracle_and_lone_solves(gpu_lib, n_graphs, lo, hi):
    api = gpu_lib
    g = synth.multi_graph(n_graphs, lo, hi, 8, 2.2, seed=51, sigma=1.5)
    op = api.Operator(g.n, g.follower, g.leader, g.lam, g.mu, node_offsets=g.node_offsets)
    psi, infos = op.solve_graphs(tol=1e-10)
    psi = psi.cpu().numpy()
    assert len(infos) == n_graphs
    again, _ = op.solve_graphs(tol=1e-10)
    assert np.array_equal(again.cpu().numpy(), psi)
    for k in sorted({0, 1, n_graphs // 2, n_graphs - 1}):
        sub = subgraph(g, k)
        A, B, c, d = oracle.operator(sub.n, sub.follower, sub.leader, sub.lam, sub.mu)
        r = oracle.power_psi(A, B, c, d, 1e-10)
        part = psi[g.node_offsets[k]:g.node_offsets[k + 1]]
        assert infos[k]["status"] == 0
        assert abs(infos[k]["iterations"] - r["iterations"]) <= 1
        assert oracle.rel_l1(r["psi"], part) <= 1e-9
        lone = api.Operator(sub.n, sub.follower, sub.leader, sub.lam, sub.mu)
        p1, i1 = lone.solve(tol=1e-10)
        assert abs(i1["iterations"] - infos[k]["iterations"]) <= 1
        assert oracle.rel_l1(p1.cpu().numpy(), part) <= 1e-12


@pytest.mark.parametrize("S,form", [(2, "tiles"), (2, "slices"), (4, "slices"), (8, "tiles")])
def test_graphs_column_segmented_passes(gpu_lib, S, form):
    """Graph batches through a column-segmented pass (partial kernel in either
    form, then the combine with the per-graph epilogue): the same results as
    the fused pass, and the oracle's on a sampled graph."""
    api = gpu_lib
    g = synth.multi_graph(5, 20000, 40000, 10, 2.1, seed=53, sigma=1.5)
    op = api.Operator(g.n, g.follower, g.leader, g.lam, g.mu, node_offsets=g.node_offsets)
    fused, i_f = op.solve_graphs(tol=1e-10, col_segments=1)
    seg, i_s = op.solve_graphs(tol=1e-10, col_segments=S, seg_form=form)
    assert all(i["col_segments"] == S for i in i_s)
    assert oracle.rel_l1(fused.cpu().numpy(), seg.cpu().numpy()) <= 1e-12
    assert all(abs(a["iterations"] - b["iterations"]) <= 1 for a, b in zip(i_f, i_s))
    k = 3
    sub = subgraph(g, k)
    A, B, c, d = oracle.operator(sub.n, sub.follower, sub.leader, sub.lam, sub.mu)
    r = oracle.power_psi(A, B, c, d, 1e-10)
    part = seg.cpu().numpy()[g.node_offsets[k]:g.node_offsets[k + 1]]
    assert i_s[k]["status"] == 0 and abs(i_s[k]["iterations"] - r["iterations"]) <= 1
    assert oracle.rel_l1(r["psi"], part) <= 1e-9


@pytest.mark.parametrize("n_graphs,lo,hi,S,form", [(7, 500, 3000, 1, "auto"),
                                                   (4, 20000, 40000, 1, "auto"),
                                                   (5, 20000, 40000, 2, "tiles"),
                                                   (5, 20000, 40000, 4, "slices")])
def test_graphs_mixed_match_oracle(gpu_lib, n_graphs, lo, hi, S, form):
    """Graph batches in mixed precision: per graph, FP32 correction solves
    refined by FP64 residual passes, stopping on the FP64 gap: each graph
    matches the oracle's Algorithm 2 at the same tolerance and the FP64 batch;
    repeat solves are bitwise equal."""
    api = gpu_lib
    g = synth.multi_graph(n_graphs, lo, hi, 10, 2.1, seed=54, sigma=1.5)
    op = api.Operator(g.n, g.follower, g.leader, g.lam, g.mu, node_offsets=g.node_offsets)
    psi, infos = op.solve_graphs(tol=1e-10, precision="mixed", col_segments=S, seg_form=form)
    again, _ = op.solve_graphs(tol=1e-10, precision="mixed", col_segments=S, seg_form=form)
    assert torch.equal(psi, again)
    psi64, _ = op.solve_graphs(tol=1e-10)
    psi = psi.cpu().numpy()
    assert oracle.rel_l1(psi64.cpu().numpy(), psi) <= 1e-9
    assert sum(i["fp32_passes"] for i in infos) > 0
    for k in sorted({0, n_graphs // 2, n_graphs - 1}):
        i = infos[k]
        assert i["status"] == 0 and i["final_gap"] <= 1e-10, i
        assert i["spmv_passes"] == i["iterations"] + i["fp32_passes"] + 1
        assert i["col_segments"] == S
        sub = subgraph(g, k)
        A, B, c, d = oracle.operator(sub.n, sub.follower, sub.leader, sub.lam, sub.mu)
        r = oracle.power_psi(A, B, c, d, 1e-10)
        part = psi[g.node_offsets[k]:g.node_offsets[k + 1]]
        assert oracle.rel_l1(r["psi"], part) <= 1e-9
        assert oracle.max_rel(r["psi"], part) <= 1e-7


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_autotune_graphs_schedule_is_used(gpu_lib, prec):
    api = gpu_lib
    g = synth.multi_graph(6, 20000, 40000, 10, 2.1, seed=55, sigma=1.5)
    op = api.Operator(g.n, g.follower, g.leader, g.lam, g.mu, node_offsets=g.node_offsets)
    t = op.autotune_graphs(prec)
    assert t["col_segments"] in ((1, 2, 4) if prec == "mixed" else (1, 2, 4, 8))
    assert t["tile_items"] in (1024, 2048, 3072, 4096) and t["solve_ms"] > 0
    psi, infos = op.solve_graphs(tol=1e-10, precision=prec)
    for i in infos:
        assert (i["tile_items"], i["col_segments"]) == (t["tile_items"], t["col_segments"])
        assert i["status"] == 0
    k = 2
    sub = subgraph(g, k)
    A, B, c, d = oracle.operator(sub.n, sub.follower, sub.leader, sub.lam, sub.mu)
    r = oracle.power_psi(A, B, c, d, 1e-10)
    part = psi.cpu().numpy()[g.node_offsets[k]:g.node_offsets[k + 1]]
    assert oracle.rel_l1(r["psi"], part) <= 1e-9


def test_graphs_with_an_edgeless_graph(gpu_lib):
    api = gpu_lib
    a = synth.chung_lu(2000, 6, 2.2, 52)
    n_iso = 50
    b_lam = np.linspace(0.2, 3.0, n_iso)
    b_mu = np.linspace(1.5, 0.1, n_iso)
    n = a.n + n_iso
    offs = np.array([0, a.n, n], dtype=np.int64)
    op = api.Operator(n, a.follower, a.leader, np.concatenate([a.lam, b_lam]),
                      np.concatenate([a.mu, b_mu]), node_offsets=offs)
    psi, infos = op.solve_graphs(tol=1e-11)
    psi = psi.cpu().numpy()
    np.testing.assert_allclose(psi[a.n:], b_lam / (b_lam + b_mu) / n_iso, rtol=1e-15)
    A, B, c, d = oracle.operator(a.n, a.follower, a.leader, a.lam, a.mu)
    r = oracle.power_psi(A, B, c, d, 1e-11)
    assert oracle.rel_l1(r["psi"], psi[:a.n]) <= 1e-9
    bad_f = np.array([0, a.n + 1], dtype=np.int32)  # an edge joining the two graphs
    bad_l = np.array([1, 3], dtype=np.int32)
    with pytest.raises(api.PsiError, match="joins two graphs"):
        api.Operator(n, bad_f, bad_l, np.ones(n), np.ones(n), node_offsets=offs)


# ---------------------------------------------------------------- origin mode
def test_origins_match_power_nf_and_power_psi(gpu_lib):
    """Algorithm 1 (Power-NF) for 70 origins at once (two tiles of lanes)."""
    api = gpu_lib
    g = synth.chung_lu(4000, 8, 2.1, 81, sigma=1.5)
    op = api.Operator(g.n, g.follower, g.leader, g.lam, g.mu)
    A, B, c, d = oracle.operator(g.n, g.follower, g.leader, g.lam, g.mu)
    n_followers = np.asarray((B > 0).sum(axis=0)).ravel()  # column i of B: followers of i
    hub = int(np.argmax(n_followers))
    lonely = int(np.flatnonzero(n_followers == 0)[0])
    rng = np.random.default_rng(5)
    origins = np.concatenate([[hub, lonely, hub], rng.choice(g.n, 67, replace=False)])
    psi_o, P, infos = op.solve_origins(origins, tol=1e-12)
    psi_o, P = psi_o.cpu().numpy(), P.cpu().numpy()
    psi_all = oracle.power_psi(A, B, c, d, 1e-13)["psi"]
    for k, i in enumerate(origins):
        b = B[:, i].toarray().ravel()
        p_ref, t_ref = oracle.power_nf(A, b, 1e-12)
        assert infos[k]["status"] == 0 and abs(infos[k]["iterations"] - t_ref) <= 1, (k, i)
        assert np.abs(P[:, k] - p_ref).sum() <= 1e-10 * max(np.abs(p_ref).sum(), 1e-300) + 1e-300
        psi_ref = (c @ p_ref + d[i]) / g.n  # eqs. wall and psiscore
        assert abs(psi_o[k] - psi_ref) <= 1e-12 * psi_ref
        assert abs(psi_o[k] - psi_all[i]) <= 1e-9 * psi_all[i]  # the same ψ_i as Power-ψ
    assert np.array_equal(P[:, 0], P[:, 2])  # a repeated origin gives the same column
    assert not P[:, 1].any()                 # nobody follows `lonely`: p = 0, ψ = d/N
    assert psi_o[1] == d[lonely] / g.n


def test_origins_invalid(gpu_lib):
    api = gpu_lib
    g = synth.chung_lu(500, 5, 2.2, 82)
    op = api.Operator(g.n, g.follower, g.leader, g.lam, g.mu)
    with pytest.raises(api.PsiError, match="origin"):
        op.solve_origins([0, g.n])
    with pytest.raises(ValueError):
        op.solve_origins([])


def test_origins_with_a_user_who_follows_everyone(gpu_lib):
    """One follower with 3000 leaders: a chunked row of CSR(A) in origin mode."""
    api = gpu_lib
    n = 3001
    base = synth.chung_lu(n, 4, 2.2, 83, sigma=1.0)
    f = np.concatenate([base.follower, np.zeros(n - 1, dtype=np.int32)])
    l = np.concatenate([base.leader, np.arange(1, n, dtype=np.int32)])
    op = api.Operator(n, f, l, base.lam, base.mu)
    A, B, c, d = oracle.operator(n, f, l, base.lam, base.mu)
    origins = np.array([1, 17, 2500, 0])
    psi_o, P, infos = op.solve_origins(origins, tol=1e-13)
    psi_o, P = psi_o.cpu().numpy(), P.cpu().numpy()
    for k, i in enumerate(origins):
        p_ref, t_ref = oracle.power_nf(A, B[:, i].toarray().ravel(), 1e-13)
        assert abs(infos[k]["iterations"] - t_ref) <= 1
        assert np.abs(P[:, k] - p_ref).sum() <= 1e-10 * max(np.abs(p_ref).sum(), 1e-300) + 1e-300
        assert abs(psi_o[k] - (c @ p_ref + d[i]) / n) <= 1e-12 * psi_o[k]
