"""Pins of the C/OpenMP oracle: the same checks that pin the NumPy oracle
(hand-derived examples bit for bit, the ψ definition solved as N separate
systems, the star closed form, the clean-up counts), plus agreement with the
NumPy oracle on a power-law graph and the same bits for any thread count.
CPU only."""
import json
import os

import numpy as np
import pytest

import oracle
import oracle.psi_oracle_c as oc
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def golden(name):
    with open(os.path.join(GOLDEN, name)) as fh:
        return json.load(fh)


def graph_of(gd):
    return oc.Graph(gd["n"], gd["follower"], gd["leader"], gd["lambda"], gd["mu"])


def test_two_user_iterates_bit_exact():
    gd = golden("two_user.json")
    g = graph_of(gd)
    c, d, _ = g.vectors()
    assert np.array_equal(c, gd["c"]) and np.array_equal(d, gd["d"])
    for t in range(1, len(gd["iterates"])):
        r = g.power_psi(1e-3, steps=1, s0=np.array(gd["iterates"][t - 1]))
        assert r["iterations"] == 1
        assert np.array_equal(r["s"], gd["iterates"][t])
        assert r["gap"] == gd["gaps"][t - 1]
    r = g.power_psi(0.3)
    assert r["iterations"] == 3 and r["gap"] == gd["gaps"][2]
    r = g.power_psi(1e-15)
    np.testing.assert_allclose(r["s"], gd["s_fixed_point"], rtol=0, atol=1e-14)
    np.testing.assert_allclose(r["psi"], gd["psi"], rtol=0, atol=1e-14)
    assert g.b_norm() == gd["b_norm"] and g.kappa() == gd["kappa"]


def test_three_user_row_sum_norms_and_fixed_point():
    gd = golden("three_user.json")
    g = graph_of(gd)
    assert g.b_norm() == pytest.approx(gd["b_norm"], rel=1e-15)
    assert g.kappa() == pytest.approx(gd["kappa"], rel=1e-15)
    assert g.n_no_leaders == 1
    r = g.power_psi(1e-15)
    np.testing.assert_allclose(r["s"], gd["s_fixed_point"], rtol=1e-15, atol=0)
    np.testing.assert_allclose(r["psi"], gd["psi"], rtol=1e-15, atol=0)
    # Algorithm 2 as printed: the gap is ‖B‖ times the step size
    rb = g.power_psi(1e-3, tol_mode="bnorm", steps=1)
    assert rb["gap"] == pytest.approx(gd["b_norm"] * rb["l1_step"], rel=1e-15)
    assert g.power_psi(2.0)["iterations"] == 0  # initial gap 1 ≤ ε


@pytest.mark.parametrize("n,p,seed,dangling", [(30, 0.15, 11, True), (60, 0.08, 12, False),
                                               (120, 0.04, 13, True), (200, 0.03, 14, False)])
def test_matches_n_separate_solves(n, p, seed, dangling):
    gs = synth.random_small(n, p, seed, dangling=dangling, extra_self_loops=5,
                            extra_duplicates=9)
    psi_def, _, _ = oracle.psi_by_definition(gs.n, gs.follower, gs.leader, gs.lam, gs.mu)
    g = oc.Graph(gs.n, gs.follower, gs.leader, gs.lam, gs.mu)
    r = g.power_psi(1e-13)
    assert oracle.rel_l1(psi_def, r["psi"]) <= 1e-11
    assert np.max(np.abs(r["psi"] - psi_def) / psi_def) <= 1e-10


def test_clean_up_counts_match_the_numpy_oracle():
    gs = synth.random_small(150, 0.05, 23, extra_self_loops=17, extra_duplicates=31)
    _, _, loops, dups = oracle.clean_edges(gs.n, gs.follower, gs.leader)
    g = oc.Graph(gs.n, gs.follower, gs.leader, gs.lam, gs.mu)
    assert (g.n_self_loops, g.n_duplicates) == (loops, dups)
    assert g.m + loops + dups == gs.m_raw
    row, fol = g.rows()
    assert np.array_equal(g.row_lengths(), np.diff(row))
    ff, ll, _, _ = oracle.clean_edges(gs.n, gs.follower, gs.leader)
    order = np.lexsort((ff, ll))  # by leader, then follower
    assert np.array_equal(np.repeat(np.arange(gs.n), np.diff(row)), ll[order])
    assert np.array_equal(fol, ff[order])


def test_star_closed_form():
    gs = synth.star(5001, 31, sigma=1.5)
    g = oc.Graph(gs.n, gs.follower, gs.leader, gs.lam, gs.mu)
    c, d, _ = g.vectors()
    r = g.power_psi(1e-14)
    hub = d[0] * (1 + c[1:].sum()) / gs.n
    assert r["psi"][0] == pytest.approx(hub, rel=1e-14)
    np.testing.assert_allclose(r["psi"][1:], d[1:] / gs.n, rtol=1e-15, atol=0)
    assert g.max_followers == gs.n - 1


def test_agrees_with_the_numpy_oracle_on_a_power_law_graph():
    gs = synth.chung_lu(20000, 12, 2.1, 41, sigma=2.0)
    A, B, c, d = oracle.operator(gs.n, gs.follower, gs.leader, gs.lam, gs.mu)
    ref = oracle.power_psi(A, B, c, d, 1e-10)
    g = oc.Graph(gs.n, gs.follower, gs.leader, gs.lam, gs.mu)
    r = g.power_psi(1e-10)
    assert r["iterations"] == ref["iterations"]
    assert np.max(np.abs(r["psi"] - ref["psi"]) / ref["psi"]) <= 1e-14
    assert np.max(np.abs(r["s"] - ref["s"]) / ref["s"]) <= 1e-14
    s = ref["s"] * 1.001
    res, l1 = g.residual(s)
    np.testing.assert_allclose(res, A.T @ s + c - s, rtol=1e-13, atol=1e-15)
    assert l1 == pytest.approx(np.abs(A.T @ s + c - s).sum(), rel=1e-13)
    np.testing.assert_allclose(g.final(s), (B.T @ s + d) / gs.n, rtol=1e-14, atol=0)
    assert g.b_norm() == pytest.approx(oracle.b_norm(B), rel=1e-14)
    assert g.kappa() == pytest.approx(oracle.kappa(A), rel=1e-14)


def test_same_bits_for_any_thread_count():
    gs = synth.chung_lu(30000, 15, 2.2, 42, sigma=1.5)
    out = []
    for k in (1, 3, 8):
        oc.set_threads(k)
        g = oc.Graph(gs.n, gs.follower, gs.leader, gs.lam, gs.mu)
        r = g.power_psi(1e-9)
        out.append((r["iterations"], r["gap"], r["psi"].tobytes(), g.rows()[1].tobytes()))
    oc.set_threads(os.cpu_count() or 1)
    assert out[0] == out[1] == out[2]


def test_errors():
    gs = synth.random_small(20, 0.2, 3)
    lam = gs.lam.copy()
    lam[4] = 0.0
    with pytest.raises(ValueError):
        oc.Graph(gs.n, gs.follower, gs.leader, lam, gs.mu)
    with pytest.raises(ValueError):
        oc.Graph(gs.n, np.array([0, 20], np.int32), np.array([1, 2], np.int32), gs.lam, gs.mu)
    g = oc.Graph(gs.n, gs.follower, gs.leader, gs.lam, gs.mu)
    with pytest.raises(ValueError):
        g.power_psi(0.0)
    s0 = np.full(gs.n, np.inf)
    with pytest.raises(FloatingPointError):
        g.power_psi(1e-9, s0=s0)
