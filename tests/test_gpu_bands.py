"""The band (column-blocked) layout of the pass against the oracle.

Rows of every kind the layout has to handle: rows inside one column block
and rows spread over all of them, rows exactly at a row block's edge budget
and one past it (cut into two pieces), hub rows cut into hundreds of pieces,
the last user's row, users with no followers; one and several column blocks
(2^17 and 2^18 users), one band and several bands (more row blocks than a
launch has waves), and degenerate operators.  One pass is compared element
by element (rtol 1e-13) and bit for bit between repeats; solves to the
oracle's Algorithm 2 at the same tolerance (1e-9 relative L1, and element
by element).
"""
import numpy as np
import pytest
import torch

import oracle
import oracle.psi_oracle_c as oc
import synth

pytestmark = pytest.mark.gpu

PARAMS = [(17, 1024), (17, 1280), (17, 1536), (17, 2048), (18, 1024), (18, 2048)]


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
    n = 600_000
    rows = [(5, 0, 300_000),          # hub over three column blocks, cut into pieces
            (9, 131_000, 2_048),      # exactly a minimal row block's budget, across a block edge
            (12, 262_100, 2_049),     # one past it: two pieces
            (15, 500_000, 99_999),    # into the last column block
            (n - 1, 10, 5_000),       # the last user
            (77, 131_071, 2)]         # the two users around the first column-block edge
    return graph_with_rows(n, rows, 3 * n, 7)


@pytest.fixture(scope="module")
def special(gpu_lib):
    g = special_graph()
    A, B, c, d = oracle.operator(g.n, g.follower, g.leader, g.lam, g.mu)
    return g, A, B, c, d


@pytest.mark.parametrize("col_log,rows", PARAMS)
def test_band_step_and_final_match_oracle(gpu_lib, special, col_log, rows):
    api = gpu_lib
    g, A, B, c, d = special
    op = api.Operator(g.n, g.follower, g.leader, g.lam, g.mu)
    r = oracle.power_psi(A, B, c, d, 1e-9)
    psi, info = op.solve(tol=1e-9, seg_form="bands", band_col_log=col_log, band_rows=rows)
    assert info["status"] == 0 and info["seg_form"] == api.SEG_FORMS["bands"], info
    bi = op.band_info()
    assert bi["col_log"] == col_log and bi["rows"] == rows
    assert bi["col_blocks"] == -(-g.n // (1 << col_log)) and bi["split_rows"] >= 2, bi
    assert oracle.rel_l1(r["psi"], psi.cpu().numpy()) <= 1e-9
    assert oracle.max_rel(r["psi"], psi.cpu().numpy()) <= (
        1e-9 if info["iterations"] == r["iterations"] else 1e-6)
    s_in = np.random.default_rng(4).uniform(0.5, 3.0, g.n)
    expect = A.T @ s_in + c
    out, gap = op.step(torch.tensor(s_in, device="cuda"), seg_form="bands")
    torch.cuda.synchronize()
    np.testing.assert_allclose(out.cpu().numpy(), expect, rtol=1e-13, atol=0)
    assert abs(gap.item() - np.abs(expect - s_in).sum()) <= 1e-12 * np.abs(expect - s_in).sum()
    for _ in range(3):  # bitwise repeatable
        again, gap2 = op.step(torch.tensor(s_in, device="cuda"), seg_form="bands")
        torch.cuda.synchronize()
        assert torch.equal(again, out) and torch.equal(gap2, gap)
    assert op.band_info() == bi  # the step kept the layout the solve built
    fin = op.final(torch.tensor(s_in, device="cuda")).cpu().numpy()
    np.testing.assert_allclose(fin, (B.T @ s_in + d) / g.n, rtol=1e-13, atol=0)


@pytest.mark.parametrize("prec,tol,bar,elem", [("fp64", 1e-9, 1e-9, 1e-6), ("mixed", 1e-9, 1e-9, 1e-6),
                                               ("fp32", 1e-5, 1e-6, 1e-4)])
def test_band_solves_every_precision(gpu_lib, prec, tol, bar, elem):
    api = gpu_lib
    g = synth.chung_lu(300_000, 20, 2.1, 15, sigma=2.0)
    A, B, c, d = oracle.operator(g.n, g.follower, g.leader, g.lam, g.mu)
    r = oracle.power_psi(A, B, c, d, tol)
    op = api.Operator(g.n, g.follower, g.leader, g.lam, g.mu)
    psi, info = op.solve(tol=tol, precision=prec, seg_form="bands", band_col_log=17,
                         band_rows=1024)
    assert info["status"] == 0, info
    got = psi.cpu().numpy()
    assert oracle.rel_l1(r["psi"], got) <= bar
    assert oracle.max_rel(r["psi"], got) <= elem
    if prec == "fp64":
        psi_a, info_a = op.solve_anderson(tol=tol, depth=4, seg_form="bands")
        assert info_a["status"] == 0 and oracle.rel_l1(r["psi"], psi_a.cpu().numpy()) <= 1e-9


def test_band_several_bands_against_the_c_oracle(gpu_lib):
    """5·10⁶ users: more row blocks than one launch has waves, so a pass runs
    several band launches; every user against the C oracle."""
    api = gpu_lib
    g = synth.chung_lu(5_000_000, 4, 2.1, 16, sigma=2.0)
    G = oc.Graph(g.n, g.follower, g.leader, g.lam, g.mu)
    op = api.Operator(g.n, g.follower, g.leader, g.lam, g.mu)
    s_in = np.random.default_rng(5).uniform(0.5, 3.0, g.n)
    ref = G.power_psi(1e-8)
    for col_log, rows in ((17, 2048), (18, 1024), (17, 1280), (18, 1536)):
        psi, s, info = op.solve(tol=1e-8, seg_form="bands", band_col_log=col_log,
                                band_rows=rows, return_s=True)
        assert info["status"] == 0, info
        assert op.band_info()["bands"] >= 2, op.band_info()
        assert oracle.rel_l1(ref["psi"], psi.cpu().numpy()) <= 1e-9
        assert oracle.max_rel(ref["psi"], psi.cpu().numpy()) <= (
            1e-9 if info["iterations"] == ref["iterations"] else 1e-6)
        res, _ = G.residual(s_in)
        out, _ = op.step(torch.tensor(s_in, device="cuda"), seg_form="bands")
        torch.cuda.synchronize()
        # the oracle's residual r = (Aᵀs + c) − s gives back Aᵀs + c only to an
        # ulp of s (the cancellation in r): allow that beside rtol 1e-13
        np.testing.assert_allclose(out.cpu().numpy(), res + s_in, rtol=1e-13, atol=1e-15)


def test_band_degenerate_operators(gpu_lib):
    """Five users (one column block, mostly empty), no edges at all, and one
    user: the band layout gives the oracle's step and ψ."""
    api = gpu_lib
    f = np.array([1, 2, 3, 4, 0, 0], dtype=np.int32)
    l = np.array([0, 0, 0, 0, 4, 3], dtype=np.int32)
    lam = np.array([0.5, 1.0, 2.0, 0.7, 1.3])
    mu = np.array([1.0, 0.5, 0.2, 0.9, 0.4])
    s_in = np.array([1.0, 2.0, 3.0, 4.0, 5.0])
    for n, ff, ll in ((5, f, l), (5, f[:0], l[:0])):
        A, B, c, d = oracle.operator(n, ff, ll, lam, mu)
        op = api.Operator(n, ff, ll, lam, mu)
        out, _ = op.step(torch.tensor(s_in, device="cuda"), seg_form="bands")
        torch.cuda.synchronize()
        np.testing.assert_allclose(out.cpu().numpy(), A.T @ s_in + c, rtol=1e-15, atol=0)
        r = oracle.power_psi(A, B, c, d, 1e-12)
        psi, info = op.solve(tol=1e-12, seg_form="bands")
        assert info["status"] == 0
        np.testing.assert_allclose(psi.cpu().numpy(), r["psi"], rtol=1e-13, atol=0)
    op = api.Operator(1, np.zeros(0, np.int32), np.zeros(0, np.int32), [2.0], [1.0])
    psi, info = op.solve(tol=1e-12, seg_form="bands")
    assert info["status"] == 0 and abs(psi.item() - 2.0 / 3.0) <= 1e-15


U = 2.0 ** -53  # unit roundoff of FP64


def residual_within_rounding(A, c, s, tol):
    """‖Aᵀs + c − s‖₁ ≤ tol up to the rounding of two summation orders: the
    oracle evaluates each row in its own order, which moves s_i' by at most
    (|F(i)| + 3) ulps of its terms' magnitude on each side."""
    deg = np.diff(A.T.tocsr().indptr)
    res = np.abs(A.T @ s + c - s)
    slack = 2 * U * (deg + 3) * (np.abs(s) + c)
    assert np.all(res <= tol + slack), int(np.argmax(res - slack))
    return res.sum()


@pytest.mark.parametrize("col_log,rows", [(17, 1024), (18, 2048)])
def test_async_sweeps_match_the_oracle(gpu_lib, special, col_log, rows):
    """Block Gauss–Seidel sweeps over the bands: the oracle's Algorithm 2 result
    at the same tolerance, bitwise repeatable, and a fixed point whose residual
    the oracle confirms (this graph fits one band, so a sweep is a Power-ψ
    step; several bands are tested below)."""
    api = gpu_lib
    g, A, B, c, d = special
    r = oracle.power_psi(A, B, c, d, 1e-10)
    op = api.Operator(g.n, g.follower, g.leader, g.lam, g.mu)
    psi, s, info = op.solve_async(tol=1e-10, band_col_log=col_log, band_rows=rows,
                                  return_s=True)
    assert info["status"] == 0 and info["seg_form"] == api.SEG_FORMS["bands"], info
    got = psi.cpu().numpy()
    assert oracle.rel_l1(r["psi"], got) <= 1e-9
    assert oracle.max_rel(r["psi"], got) <= 1e-6
    residual_within_rounding(A, c, s.cpu().numpy(), 1e-10)
    assert info["iterations"] <= r["iterations"] + 1
    psi2, info2 = op.solve_async(tol=1e-10, band_col_log=col_log, band_rows=rows)
    assert torch.equal(psi2, psi) and info2["iterations"] == info["iterations"]


def test_async_sweeps_several_bands_and_a_start(gpu_lib):
    """Several bands per sweep (5·10⁶ users) against the C oracle, and a start
    vector used as given."""
    api = gpu_lib
    g = synth.chung_lu(5_000_000, 4, 2.1, 17, sigma=2.0)
    G = oc.Graph(g.n, g.follower, g.leader, g.lam, g.mu)
    ref = G.power_psi(1e-8)
    op = api.Operator(g.n, g.follower, g.leader, g.lam, g.mu)
    psi, s, info = op.solve_async(tol=1e-8, band_col_log=17, band_rows=1024, return_s=True)
    assert info["status"] == 0, info
    assert op.band_info()["bands"] >= 2
    assert oracle.rel_l1(ref["psi"], psi.cpu().numpy()) <= 1e-9
    assert oracle.max_rel(ref["psi"], psi.cpu().numpy()) <= 1e-6
    assert info["iterations"] < ref["iterations"], (info["iterations"], ref["iterations"])
    _, l1 = G.residual(s.cpu().numpy())
    _, l1_ref = G.residual(ref["s"])
    assert l1 <= 1e-8 + 2 * l1_ref  # the sweep's change bounds the residual (κ ≤ 1)
    psi_w, info_w = op.solve_async(tol=1e-8, s0=s)  # from the fixed point: one sweep
    assert info_w["status"] == 0 and info_w["iterations"] <= 2 and info_w["used_s0"] == 1
    assert oracle.rel_l1(ref["psi"], psi_w.cpu().numpy()) <= 1e-9
    with pytest.raises(api.PsiError):
        op.solve_async(tol=0.0)
