"""Pins for the CPU oracle: every check compares it with something other than
itself — the hand-derived two-user example, closed forms, a textbook PageRank
routine, the paper's error bound, invariants of the model, and the ψ
definition solved as N separate systems.  CPU only."""
import json
import os

import networkx as nx
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def two_user():
    with open(os.path.join(GOLDEN, "two_user.json")) as fh:
        return json.load(fh)


def three_user():
    with open(os.path.join(GOLDEN, "three_user.json")) as fh:
        return json.load(fh)


def op_of(g):
    return oracle.operator(g.n, g.follower, g.leader, g.lam, g.mu)


# ---------------------------------------------------------------- worked example
def test_two_user_closed_form():
    gd = two_user()
    A, B, c, d = oracle.operator(gd["n"], gd["follower"], gd["leader"], gd["lambda"], gd["mu"])
    assert np.array_equal(c, gd["c"]) and np.array_equal(d, gd["d"])
    r = oracle.power_psi(A, B, c, d, 1e-15)
    np.testing.assert_allclose(r["s"], gd["s_fixed_point"], rtol=0, atol=1e-14)
    np.testing.assert_allclose(r["psi"], gd["psi"], rtol=0, atol=1e-14)
    psi_def, _, _ = oracle.psi_by_definition(gd["n"], gd["follower"], gd["leader"],
                                             gd["lambda"], gd["mu"])
    np.testing.assert_allclose(psi_def, gd["psi"], rtol=0, atol=1e-15)
    assert oracle.b_norm(B) == gd["b_norm"]
    assert oracle.kappa(A) == gd["kappa"]


def test_two_user_iterates_bit_exact():
    """The iterates are dyadic, so FP64 reproduces them exactly."""
    gd = two_user()
    A, B, c, d = oracle.operator(gd["n"], gd["follower"], gd["leader"], gd["lambda"], gd["mu"])
    for t in range(1, len(gd["iterates"])):
        s_prev = np.array(gd["iterates"][t - 1])
        r = oracle.power_psi(A, B, c, d, tol=1.0 - 1e-12, s0=s_prev)  # exactly one step
        assert r["iterations"] == 1
        assert np.array_equal(r["s"], gd["iterates"][t])
        assert r["gap"] == gd["gaps"][t - 1]
    r = oracle.power_psi(A, B, c, d, tol=0.3, record=True)
    assert r["gaps"] == gd["gaps"][:3] and r["iterations"] == 3


def test_three_user_norms_are_row_sums():
    """‖B‖ and κ are the largest row sums (row-vector L1 norm); in this
    hand-derived case the largest column sums differ, so a transposed
    reading fails here."""
    gd = three_user()
    A, B, c, d = oracle.operator(gd["n"], gd["follower"], gd["leader"], gd["lambda"], gd["mu"])
    assert oracle.b_norm(B) == pytest.approx(gd["b_norm"], rel=1e-15)
    assert oracle.kappa(A) == pytest.approx(gd["kappa"], rel=1e-15)
    assert gd["b_norm"] != gd["b_norm_columns"] and gd["kappa"] != gd["kappa_columns"]
    assert oracle.b_norm(B.T.tocsr()) == pytest.approx(gd["b_norm_columns"], rel=1e-15)
    assert oracle.kappa(A.T.tocsr()) == pytest.approx(gd["kappa_columns"], rel=1e-15)
    assert np.array_equal(c, gd["c"]) and np.array_equal(d, gd["d"])
    r = oracle.power_psi(A, B, c, d, 1e-15)
    np.testing.assert_allclose(r["s"], gd["s_fixed_point"], rtol=1e-15, atol=0)
    np.testing.assert_allclose(r["psi"], gd["psi"], rtol=1e-15, atol=0)
    assert r["psi"].sum() == pytest.approx(gd["psi_sum"], rel=1e-15)
    psi_def, _, _ = oracle.psi_by_definition(gd["n"], gd["follower"], gd["leader"],
                                             gd["lambda"], gd["mu"])
    np.testing.assert_allclose(psi_def, gd["psi"], rtol=1e-15, atol=0)
    # the bnorm stopping mode uses the row-sum norm: first gap = ‖B‖·‖s_1 − c‖₁
    rb = oracle.power_psi(A, B, c, d, tol=1e-3, tol_mode="bnorm", record=True)
    s1 = A.T @ c + c
    assert rb["gaps"][0] == pytest.approx(gd["b_norm"] * np.abs(s1 - c).sum(), rel=1e-15)


# ---------------------------------------------------------------- definition (N solves)
@pytest.mark.parametrize("n,p,seed,dangling", [(30, 0.15, 11, True), (60, 0.08, 12, False),
                                               (120, 0.04, 13, True), (200, 0.03, 14, False)])
def test_power_psi_matches_n_separate_solves(n, p, seed, dangling):
    g = synth.random_small(n, p, seed, dangling=dangling, extra_self_loops=3, extra_duplicates=5)
    psi_def, P, Q = oracle.psi_by_definition(g.n, g.follower, g.leader, g.lam, g.mu)
    A, B, c, d = op_of(g)
    r = oracle.power_psi(A, B, c, d, 1e-14)
    assert oracle.rel_l1(psi_def, r["psi"]) < 1e-12
    cf, _ = oracle.psi_closed_form(A, B, c, d)
    assert oracle.rel_l1(psi_def, cf) < 1e-12
    # matrix form of the same systems: P = (I − A)⁻¹ B, Q = C P + D (eqs. nf_solution, wall)
    I = np.eye(n)
    P2 = np.linalg.solve(I - A.toarray(), B.toarray())
    np.testing.assert_allclose(P2, P, rtol=0, atol=1e-12)
    np.testing.assert_allclose(np.diag(c) @ P2 + np.diag(d), Q, rtol=0, atol=1e-12)


def test_power_nf_matches_definition():
    g = synth.random_small(40, 0.1, 21, dangling=True)
    psi_def, P, Q = oracle.psi_by_definition(g.n, g.follower, g.leader, g.lam, g.mu)
    A, B, c, d = op_of(g)
    Bd = B.toarray()
    for i in (0, 7, 39):
        p, t = oracle.power_nf(A, Bd[:, i], 1e-14)
        np.testing.assert_allclose(p, P[:, i], rtol=0, atol=1e-12)


# ---------------------------------------------------------------- closed forms
def test_star_closed_form():
    g = synth.star(7, seed=3)
    A, B, c, d = op_of(g)
    r = oracle.power_psi(A, B, c, d, 1e-15)
    h = 0
    expect = d / g.n
    expect[h] = d[h] * (1.0 + c[1:].sum()) / g.n
    np.testing.assert_allclose(r["psi"], expect, rtol=1e-15, atol=0)
    assert r["psi"].sum() < 1.0  # the hub has no leader


@pytest.mark.parametrize("maker", [synth.cycle, synth.complete])
@pytest.mark.parametrize("n", [5, 17])
def test_symmetric_graphs_uniform(maker, n):
    g = maker(n)
    A, B, c, d = op_of(g)
    r = oracle.power_psi(A, B, c, d, 1e-14)
    np.testing.assert_allclose(r["psi"], np.full(n, 1.0 / n), rtol=1e-12, atol=0)


# ---------------------------------------------------------------- PageRank reduction
@pytest.mark.parametrize("n,p,seed", [(50, 0.1, 31), (200, 0.03, 32)])
def test_homogeneous_equals_textbook_pagerank(n, p, seed):
    g = synth.random_small(n, p, seed, dangling=False, activity_kind="homogeneous")
    A, B, c, d = op_of(g)
    r = oracle.power_psi(A, B, c, d, 1e-15)
    G = nx.DiGraph()
    G.add_nodes_from(range(n))
    G.add_edges_from(zip(g.follower.tolist(), g.leader.tolist()))
    pr = nx.pagerank(G, alpha=0.85, tol=1e-15, max_iter=10_000)
    pr = np.array([pr[i] for i in range(n)])
    assert np.abs(pr - r["psi"]).max() < 1e-13
    W = oracle.transition_matrix(g.n, g.follower, g.leader)
    pi, _ = oracle.pagerank_power(W, 0.85, 1e-15)
    assert np.abs(pi - r["psi"]).max() < 1e-14


def test_homogeneous_with_dangling_is_leaking_pagerank():
    g = synth.random_small(80, 0.03, 33, dangling=True, activity_kind="homogeneous")
    A, B, c, d = op_of(g)
    r = oracle.power_psi(A, B, c, d, 1e-15)
    W = oracle.transition_matrix(g.n, g.follower, g.leader)
    n = g.n
    pi = np.linalg.solve(np.eye(n) - 0.85 * W.toarray().T, np.full(n, 0.15 / n))
    assert np.abs(pi - r["psi"]).max() < 1e-14
    assert r["psi"].sum() < 1.0


# ---------------------------------------------------------------- invariants and bounds
def test_psi_sums_to_one_without_dangling_users():
    g = synth.random_small(150, 0.05, 41, dangling=False)
    A, B, c, d = op_of(g)
    r = oracle.power_psi(A, B, c, d, 1e-15)
    assert abs(r["psi"].sum() - 1.0) < 1e-13
    g2 = synth.random_small(150, 0.01, 42, dangling=True)
    A, B, c, d = op_of(g2)
    assert oracle.power_psi(A, B, c, d, 1e-15)["psi"].sum() < 1.0 - 1e-6


def test_monotone_iterates_and_lower_bounds():
    g = synth.chung_lu(2000, 10, 2.2, 5, sigma=1.5)
    A, B, c, d = op_of(g)
    s = c.copy()
    AT = A.T.tocsr()
    for _ in range(30):
        s_new = AT @ s + c
        assert np.all(s_new >= s)
        s = s_new
    r = oracle.power_psi(A, B, c, d, 1e-12)
    assert np.all(r["s"] >= c)
    assert np.all(r["psi"] >= d / g.n)
    assert oracle.fixed_point_residual(A, c, r["s"]) <= 1e-12 * 1.0001


def test_psi_gap_bound():
    """‖ψ_t − ψ_{t−1}‖₁ ≤ ε_t ‖B‖ / N (eq. psi_diff and the bound after it)."""
    g = synth.chung_lu(3000, 10, 2.2, 6, sigma=2.0)
    A, B, c, d = op_of(g)
    n = g.n
    prev = oracle.power_psi(A, B, c, d, 1e-8, steps=0)
    assert prev["iterations"] == 0
    for t in range(1, 25):
        cur = oracle.power_psi(A, B, c, d, 1e-8, steps=t)
        delta = np.abs(cur["psi"] - prev["psi"]).sum()
        assert delta <= cur["gap"] * cur["bnorm"] / n * (1 + 1e-12)
        prev = cur
    assert 0 < cur["bnorm"] <= 1.0


def test_error_bound_kappa():
    """‖s − s_t‖₁ ≤ κ/(1−κ) ε_t when every row sum of A is at most κ < 1."""
    g = synth.chung_lu(3000, 10, 2.2, 7, sigma=1.0)
    A, B, c, d = op_of(g)
    k = oracle.kappa(A)
    assert k < 1
    _, s_star = oracle.psi_closed_form(A, B, c, d)
    r = oracle.power_psi(A, B, c, d, 1e-6)
    err = np.abs(r["s"] - s_star).sum()
    assert err <= k / (1 - k) * r["gap"] * (1 + 1e-9)


def test_tol_modes_and_zero_iterations():
    gd = two_user()
    A, B, c, d = oracle.operator(gd["n"], gd["follower"], gd["leader"], gd["lambda"], gd["mu"])
    r = oracle.power_psi(A, B, c, d, tol=2.0)  # initial gap 1 ≤ ε: no step
    assert r["iterations"] == 0
    np.testing.assert_array_equal(r["s"], c)
    rb = oracle.power_psi(A, B, c, d, tol=0.2, tol_mode="bnorm", record=True)
    assert rb["gaps"][0] == 0.5 * 0.75
    with pytest.raises(ValueError):
        oracle.power_psi(A, B, c, d, tol=0.0)


def test_clean_edges_counts():
    f = np.array([0, 1, 1, 2, 2, 2, 3], dtype=np.int32)
    l = np.array([1, 0, 0, 2, 0, 1, 3], dtype=np.int32)
    ff, ll, loops, dups = oracle.clean_edges(4, f, l)
    assert loops == 2 and dups == 1
    assert list(zip(ff.tolist(), ll.tolist())) == [(0, 1), (1, 0), (2, 0), (2, 1)]
    with pytest.raises(ValueError):
        oracle.clean_edges(4, [0], [4])


# ---------------------------------------------------------------- the pins catch planted mistakes
def _mutants():
    def transposed(n, f, l, lam, mu):
        A, B, c, d = oracle.operator(n, f, l, lam, mu)
        return A.T.tocsr(), B, c, d

    def den_lambda_only(n, f, l, lam, mu):
        return _den_variant(n, f, l, lam, mu)

    def swapped_cd(n, f, l, lam, mu):
        A, B, c, d = oracle.operator(n, f, l, lam, mu)
        return A, B, d, c

    def swapped_ab(n, f, l, lam, mu):
        A, B, c, d = oracle.operator(n, f, l, lam, mu)
        return B, A, c, d

    def dropped_d(n, f, l, lam, mu):
        A, B, c, d = oracle.operator(n, f, l, lam, mu)
        return A, B, c, np.zeros_like(d)

    def reversed_edges(n, f, l, lam, mu):
        return oracle.operator(n, l, f, lam, mu)

    return [transposed, den_lambda_only, swapped_cd, swapped_ab, dropped_d, reversed_edges]


def _den_variant(n, f, l, lam, mu):
    """den_j with only the posting rates of the leaders (a dropped term)."""
    lam = np.asarray(lam, dtype=np.float64)
    mu = np.asarray(mu, dtype=np.float64)
    ff, ll, _, _ = oracle.clean_edges(n, f, l)
    den = np.zeros(n)
    np.add.at(den, ff, lam[ll])
    A = sp.csr_matrix((mu[ll] / den[ff], (ff, ll)), shape=(n, n))
    B = sp.csr_matrix((lam[ll] / den[ff], (ff, ll)), shape=(n, n))
    return A, B, mu / (lam + mu), lam / (lam + mu)


@pytest.mark.parametrize("mutant", _mutants(), ids=lambda m: m.__name__)
def test_pins_reject_planted_mistakes(mutant):
    g = synth.random_small(40, 0.12, 51, dangling=True)
    psi_def, _, _ = oracle.psi_by_definition(g.n, g.follower, g.leader, g.lam, g.mu)
    A, B, c, d = mutant(g.n, g.follower, g.leader, g.lam, g.mu)
    try:
        r = oracle.power_psi(A, B, c, d, 1e-13, max_iter=5000)
        bad = r["psi"]
    except (RuntimeError, FloatingPointError):
        return  # diverged: caught
    assert oracle.rel_l1(psi_def, bad) > 1e-6


def test_non_finite_gap_raises():
    """A dropped term in den makes the row sums of A exceed 1: the iterates
    overflow, and the loop must raise rather than stop on a NaN gap."""
    g = synth.random_small(40, 0.12, 51, dangling=True)
    A, B, c, d = _den_variant(g.n, g.follower, g.leader, g.lam, g.mu)
    assert oracle.kappa(A) > 1
    with pytest.raises(FloatingPointError):
        oracle.power_psi(A, B, c, d, 1e-13, max_iter=100_000)
    with pytest.raises(FloatingPointError):
        oracle.power_nf(A, B[:, 0].toarray().ravel(), 1e-13, max_iter=100_000)
    W = sp.csr_matrix(np.full((3, 3), 1.0))
    with pytest.raises(FloatingPointError):
        oracle.pagerank_power(W, 2.0, 1e-13, max_iter=100_000)


def test_sampled_rows_agree_with_the_full_operator():
    """The one-by-one row evaluation (raw edges, duplicates and self-loops
    present) against the full operator's Aᵀs + c − s and (Bᵀs + d)/N."""
    g = synth.random_small(300, 0.03, 21, extra_self_loops=20, extra_duplicates=40)
    A, B, c, d = oracle.operator(g.n, g.follower, g.leader, g.lam, g.mu)
    s = oracle.power_psi(A, B, c, d, 1e-6)["s"] * 1.01  # any vector, not the fixed point
    rows = np.array([0, 5, 17, 123, 299])
    res, psi = oracle.sampled_rows(g.n, g.follower, g.leader, g.lam, g.mu, s, rows, chunk=97)
    np.testing.assert_allclose(res, (A.T @ s + c - s)[rows], rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(psi, ((B.T @ s + d) / g.n)[rows], rtol=1e-13, atol=0)
