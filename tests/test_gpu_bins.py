"""The binned two-launch pass (propagation blocking) against the oracle.

Rows of every kind the layout has to handle: a hub row cut into pieces over
several follower blocks, rows at and one past a bin's edge budget, a row in
the last follower block, the last user, users with no followers; one and
many follower blocks of 20,480 users, bins whose chunks hold the same row in
two runs (the adds go run by run), and degenerate operators.  One pass is
compared element by element (rtol 1e-13) and bit for bit between repeats;
solves to the oracle's Algorithm 2 at the same tolerance (1e-9 relative L1,
and element by element).
"""
import numpy as np
import pytest
import torch

import oracle
import oracle.psi_oracle_c as oc
import synth

pytestmark = pytest.mark.gpu


def graph_with_rows(n, rows, m_background, seed):
    """Leader r gets the followers [lo, lo + k) for each (r, lo, k), plus
    m_background random edges (none from the listed leaders)."""
    rng = np.random.default_rng(seed)
    bf = rng.integers(0, n, m_background)
    bl = rng.integers(0, n, m_background)
    keep = ~np.isin(bl, [r for r, _, _ in rows])
    f = [np.arange(lo, lo + k) for _, lo, k in rows] + [bf[keep]]
    l = [np.full(k, r) for r, _, k in rows] + [bl[keep]]
    lam = np.exp(rng.normal(0.0, 1.5, n))
    mu = np.exp(rng.normal(0.0, 1.5, n))
    return synth.Graph(n, np.concatenate(f).astype(np.int32), np.concatenate(l).astype(np.int32),
                       lam, mu)


def special_graph():
    # N = 300,000: 15 follower blocks; about 4 edges a user, so a bin's edge
    # budget is max(4096, 2.5 · 1280 · M/N) ≈ 11,900
    n = 300_000
    rows = [(5, 0, 150_000),          # hub over ten follower blocks: about twelve pieces
            (9, 20_000, 11_000),      # just under the budget, across a follower-block edge
            (12, 100_000, 40_000),    # a few pieces
            (15, 290_000, 9_999),     # into the last follower block
            (n - 1, 10, 5_000),       # the last user
            (77, 20_479, 2)]          # the two users around the first follower-block edge
    return graph_with_rows(n, rows, 3 * n, 11)


@pytest.fixture(scope="module")
def special(gpu_lib):
    g = special_graph()
    A, B, c, d = oracle.operator(g.n, g.follower, g.leader, g.lam, g.mu)
    return g, A, B, c, d


def test_bins_step_and_final_match_oracle(gpu_lib, special):
    api = gpu_lib
    g, A, B, c, d = special
    op = api.Operator(g.n, g.follower, g.leader, g.lam, g.mu)
    s_in = np.random.default_rng(4).uniform(0.5, 3.0, g.n)
    expect = A.T @ s_in + c
    out, gap = op.step(torch.tensor(s_in, device="cuda"), seg_form="bins")
    torch.cuda.synchronize()
    np.testing.assert_allclose(out.cpu().numpy(), expect, rtol=1e-13, atol=0)
    assert abs(gap.item() - np.abs(expect - s_in).sum()) <= 1e-12 * np.abs(expect - s_in).sum()
    for _ in range(3):  # bitwise repeatable
        again, gap2 = op.step(torch.tensor(s_in, device="cuda"), seg_form="bins")
        torch.cuda.synchronize()
        assert torch.equal(again, out) and torch.equal(gap2, gap)
    bi = op.bins_info()
    assert bi["block_users"] == 20480 and bi["rows"] == 1280, bi
    assert bi["col_blocks"] == -(-g.n // 20480) and bi["split_rows"] >= 2, bi
    assert bi["bins"] >= -(-g.n // 1280) and 0 < bi["runs"] <= bi["bins"] * bi["col_blocks"], bi
    r = oracle.power_psi(A, B, c, d, 1e-9)
    psi, info = op.solve(tol=1e-9, seg_form="bins")
    assert info["status"] == 0 and info["seg_form"] == api.SEG_FORMS["bins"], info
    assert oracle.rel_l1(r["psi"], psi.cpu().numpy()) <= 1e-9
    assert oracle.max_rel(r["psi"], psi.cpu().numpy()) <= (
        1e-9 if info["iterations"] == r["iterations"] else 1e-6)
    psi2, info2 = op.solve(tol=1e-9, seg_form="bins")
    assert torch.equal(psi2, psi) and info2["iterations"] == info["iterations"]


@pytest.mark.parametrize("prec,tol,bar,elem", [("fp64", 1e-9, 1e-9, 1e-6), ("mixed", 1e-9, 1e-9, 1e-6),
                                               ("fp32", 1e-5, 1e-6, 1e-4)])
def test_bins_solves_every_precision(gpu_lib, prec, tol, bar, elem):
    api = gpu_lib
    g = synth.chung_lu(300_000, 20, 2.1, 15, sigma=2.0)
    A, B, c, d = oracle.operator(g.n, g.follower, g.leader, g.lam, g.mu)
    r = oracle.power_psi(A, B, c, d, tol)
    op = api.Operator(g.n, g.follower, g.leader, g.lam, g.mu)
    psi, info = op.solve(tol=tol, precision=prec, seg_form="bins")
    assert info["status"] == 0 and info["seg_form"] == api.SEG_FORMS["bins"], info
    got = psi.cpu().numpy()
    assert oracle.rel_l1(r["psi"], got) <= bar
    assert oracle.max_rel(r["psi"], got) <= elem
    if prec == "fp64":
        fin = op.final(torch.tensor(r["s"], device="cuda")).cpu().numpy()
        np.testing.assert_allclose(fin, (B.T @ r["s"] + d) / g.n, rtol=1e-13, atol=0)


def test_bins_many_blocks_against_the_c_oracle(gpu_lib):
    """5·10⁶ users: 245 follower blocks and thousands of bins; every user
    against the C oracle, and one pass element by element."""
    api = gpu_lib
    g = synth.chung_lu(5_000_000, 4, 2.1, 16, sigma=2.0)
    G = oc.Graph(g.n, g.follower, g.leader, g.lam, g.mu)
    op = api.Operator(g.n, g.follower, g.leader, g.lam, g.mu)
    ref = G.power_psi(1e-8)
    psi, s, info = op.solve(tol=1e-8, seg_form="bins", return_s=True)
    assert info["status"] == 0 and info["seg_form"] == api.SEG_FORMS["bins"], info
    assert oracle.rel_l1(ref["psi"], psi.cpu().numpy()) <= 1e-9
    assert oracle.max_rel(ref["psi"], psi.cpu().numpy()) <= (
        1e-9 if info["iterations"] == ref["iterations"] else 1e-6)
    s_in = np.random.default_rng(5).uniform(0.5, 3.0, g.n)
    res, _ = G.residual(s_in)
    out, _ = op.step(torch.tensor(s_in, device="cuda"), seg_form="bins")
    torch.cuda.synchronize()
    # the oracle's residual r = (Aᵀs + c) − s gives back Aᵀs + c only to an
    # ulp of s (the cancellation in r): allow that beside rtol 1e-13
    np.testing.assert_allclose(out.cpu().numpy(), res + s_in, rtol=1e-13, atol=1e-15)


def test_bins_degenerate_operators(gpu_lib):
    """Five users (one follower block, mostly empty), no edges at all, and one
    user: the binned pass gives the oracle's step and ψ."""
    api = gpu_lib
    f = np.array([1, 2, 3, 4, 0, 0], dtype=np.int32)
    l = np.array([0, 0, 0, 0, 4, 3], dtype=np.int32)
    lam = np.array([0.5, 1.0, 2.0, 0.7, 1.3])
    mu = np.array([1.0, 0.5, 0.2, 0.9, 0.4])
    s_in = np.array([1.0, 2.0, 3.0, 4.0, 5.0])
    for n, ff, ll in ((5, f, l), (5, f[:0], l[:0])):
        A, B, c, d = oracle.operator(n, ff, ll, lam, mu)
        op = api.Operator(n, ff, ll, lam, mu)
        out, _ = op.step(torch.tensor(s_in, device="cuda"), seg_form="bins")
        torch.cuda.synchronize()
        np.testing.assert_allclose(out.cpu().numpy(), A.T @ s_in + c, rtol=1e-15, atol=0)
        r = oracle.power_psi(A, B, c, d, 1e-12)
        psi, info = op.solve(tol=1e-12, seg_form="bins")
        assert info["status"] == 0
        np.testing.assert_allclose(psi.cpu().numpy(), r["psi"], rtol=1e-13, atol=0)
    op = api.Operator(1, np.zeros(0, np.int32), np.zeros(0, np.int32), [2.0], [1.0])
    psi, info = op.solve(tol=1e-12, seg_form="bins")
    assert info["status"] == 0 and abs(psi.item() - 2.0 / 3.0) <= 1e-15


def test_bins_refused_where_it_does_not_apply(gpu_lib):
    api = gpu_lib
    g = synth.chung_lu(2000, 5, 2.2, 3)
    op = api.Operator(g.n, g.follower, g.leader, g.lam, g.mu, flags=api.PSI_WEIGHTED_FP64)
    with pytest.raises(api.PsiError):
        op.solve(tol=1e-8, precision="fp64_weighted", seg_form="bins")
    with pytest.raises(api.PsiError):
        op.pass_time("part64", reps=1, seg_form="bins")


def test_bins_tables_that_do_not_fit_are_refused_and_skipped(gpu_lib):
    """10⁷ users and a few hundred edges: the layout's count tables (bins ×
    follower blocks) outgrow the value array they are built in, so the binned
    layout is refused with an error, and the autotuner goes on without it."""
    api = gpu_lib
    n = 10_000_000
    rng = np.random.default_rng(21)
    f = rng.integers(0, n, 300).astype(np.int32)
    l = rng.integers(0, n, 300).astype(np.int32)
    lam = np.full(n, 1.0)
    mu = np.full(n, 0.5)
    op = api.Operator(n, f, l, lam, mu)
    with pytest.raises(api.PsiError, match="count tables"):
        op.solve(tol=1e-8, seg_form="bins")
    t = op.autotune("fp64", reps=2)
    assert t["seg_form"] != "bins", t
    psi, info = op.solve(tol=1e-8)
    assert info["status"] == 0
    A, B, c, d = oracle.operator(n, f, l, lam, mu)
    r = oracle.power_psi(A, B, c, d, 1e-8)
    assert oracle.rel_l1(r["psi"], psi.cpu().numpy()) <= 1e-9
