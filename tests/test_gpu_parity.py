"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Tolerances: FP64 solves match the oracle's Algorithm 2 at the same tolerance
within 1e-9 relative L1; mixed precision (FP32 corrections + FP64 residual)
within 1e-9; FP32-only within 1e-6.  Element by element (ψ_i ≥ d_i/N > 0, so
the relative error of every user is defined): 1e-9 when the GPU and the
oracle stop at the same step, 1e-6 when their stopping steps differ by one
(allowed: rounding can move the last gap across tol) or the solve is mixed,
1e-4 for FP32-only.  Index work (CSR structure, clean-up counts) is compared
exactly.
"""
import ctypes
import json
import os

import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def oracle_run(g, tol, tol_mode="abs_l1"):
    A, B, c, d = oracle.operator(g.n, g.follower, g.leader, g.lam, g.mu)
    r = oracle.power_psi(A, B, c, d, tol, tol_mode=tol_mode)
    return A, B, c, d, r


def assert_psi(ref, got, bar, elem_bar):
    """ψ (or s) against the oracle: relative L1 ≤ bar and the largest
    element-wise relative error ≤ elem_bar; returns the latter."""
    got = got if isinstance(got, np.ndarray) else got.cpu().numpy()
    assert oracle.rel_l1(ref, got) <= bar
    mr = oracle.max_rel(ref, got)
    print(f"max element-wise relative error {mr:.2e}")
    assert mr <= elem_bar, mr
    return mr


def elem_bar_fp64(info, r):
    """1e-9 when both stopped at the same step, else 1e-6."""
    return 1e-9 if info["iterations"] == r["iterations"] else 1e-6


def gpu_op(api, g, flags=0):
    return api.Operator(g.n, g.follower, g.leader, g.lam, g.mu, flags=flags)


# ---------------------------------------------------------------- worked example
def test_two_user_bit_exact(gpu_lib):
    api = gpu_lib
    with open(os.path.join(GOLDEN, "two_user.json")) as fh:
        gd = json.load(fh)
    f = np.array(gd["follower"], dtype=np.int32)
    l = np.array(gd["leader"], dtype=np.int32)
    op = api.Operator(2, f, l, np.array(gd["lambda"]), np.array(gd["mu"]))
    st = op.stats()
    assert st["b_norm"] == gd["b_norm"] and st["kappa"] == gd["kappa"]
    v = op.views()
    assert v["c"].cpu().tolist() == gd["c"] and v["d"].cpu().tolist() == gd["d"]
    for t in range(1, len(gd["iterates"])):
        s_in = torch.tensor(gd["iterates"][t - 1], dtype=torch.float64, device="cuda")
        s_out, gap = op.step(s_in)
        torch.cuda.synchronize()
        assert s_out.cpu().tolist() == gd["iterates"][t]
        assert gap.item() == gd["gaps"][t - 1]
    psi, s, info = op.solve(tol=1e-15, return_s=True)
    np.testing.assert_allclose(psi.cpu().numpy(), gd["psi"], rtol=0, atol=1e-15)
    np.testing.assert_allclose(s.cpu().numpy(), gd["s_fixed_point"], rtol=0, atol=1e-14)
    assert info["status"] == 0
    psi3, info3 = op.solve(tol=0.3)  # three steps, dyadic iterate
    assert info3["iterations"] == 3
    s3 = np.array(gd["iterates"][3])
    B = np.array([[0, 0.25], [0.5, 0]])
    expect = (s3 @ B + np.array(gd["d"])) / 2
    assert psi3.cpu().tolist() == expect.tolist()


# ---------------------------------------------------------------- operator build
@pytest.mark.parametrize("case", ["random_small", "chung_lu_20k", "star", "cycle"])
def test_operator_structure(gpu_lib, case):
    api = gpu_lib
    if case == "random_small":
        g = synth.random_small(150, 0.05, 3, dangling=True, extra_self_loops=7, extra_duplicates=11)
    elif case == "chung_lu_20k":
        g = synth.chung_lu(20000, 12, 2.2, 9, sigma=1.5)
    elif case == "star":
        g = synth.star(5000, 2)
    else:
        g = synth.cycle(777)
    op = gpu_op(api, g)
    st = op.stats()
    f, l, loops, dups = oracle.clean_edges(g.n, g.follower, g.leader)
    assert st["n_edges"] == f.size and st["n_self_loops"] == loops and st["n_duplicates"] == dups
    A, B, c, d = oracle.operator(g.n, g.follower, g.leader, g.lam, g.mu)
    AT = A.T.tocsr()
    AT.sort_indices()
    v = op.views()
    assert np.array_equal(v["row_ptr"].cpu().numpy(), AT.indptr)
    assert np.array_equal(v["col"].cpu().numpy(), AT.indices)
    assert np.array_equal(v["c"].cpu().numpy(), c)
    assert np.array_equal(v["d"].cpu().numpy(), d)
    den = np.zeros(g.n)
    np.add.at(den, f, g.lam[l] + g.mu[l])
    inv = np.where(den > 0, 1.0 / np.where(den > 0, den, 1.0), 0.0)
    np.testing.assert_allclose(v["inv_den"].cpu().numpy(), inv, rtol=1e-15, atol=0)
    assert abs(st["b_norm"] - oracle.b_norm(B)) <= 1e-15 * oracle.b_norm(B)
    assert abs(st["kappa"] - oracle.kappa(A)) <= 1e-15 * oracle.kappa(A)
    assert st["n_no_leaders"] == int((np.bincount(f, minlength=g.n) == 0).sum())
    assert st["max_followers"] == int(np.diff(AT.indptr).max())


@pytest.mark.parametrize("case", ["random_small", "chung_lu_20k"])
def test_host_and_device_inputs_build_the_same_operator(gpu_lib, case):
    """Edge lists and activities passed as device memory (no PSI_INPUT_HOST)
    build the operator of the same inputs passed from the host, bit for bit,
    and its solve returns the same ψ bit for bit."""
    api = gpu_lib
    if case == "random_small":
        g = synth.random_small(300, 0.03, 4, dangling=True, extra_self_loops=5, extra_duplicates=9)
    else:
        g = synth.chung_lu(20000, 12, 2.2, 10, sigma=1.5)
    op_h = gpu_op(api, g)
    op_d = api.Operator(g.n, torch.from_numpy(g.follower).cuda(), torch.from_numpy(g.leader).cuda(),
                        torch.from_numpy(g.lam).cuda(), torch.from_numpy(g.mu).cuda())
    sh, sd = op_h.stats(), op_d.stats()
    assert sh.pop("flags") == api.PSI_INPUT_HOST and sd.pop("flags") == 0
    assert sd == sh
    vh, vd = op_h.views(), op_d.views()
    for key in vh:
        assert torch.equal(vh[key], vd[key]), key
    psi_h, _ = op_h.solve(tol=1e-10)
    psi_d, _ = op_d.solve(tol=1e-10)
    assert torch.equal(psi_h, psi_d)


def test_strict_and_invalid_inputs(gpu_lib):
    api = gpu_lib
    g = synth.random_small(40, 0.1, 5, extra_self_loops=2)
    with pytest.raises(api.PsiError, match="PSI_EINVAL"):
        api.Operator(g.n, g.follower, g.leader, g.lam, g.mu, flags=api.PSI_STRICT)
    bad = g.leader.copy()
    bad[3] = g.n
    with pytest.raises(api.PsiError, match="outside"):
        api.Operator(g.n, g.follower, bad, g.lam, g.mu)
    lam = g.lam.copy()
    lam[7] = 0.0
    with pytest.raises(api.PsiError, match="activity"):
        api.Operator(g.n, g.follower, g.leader, lam, g.mu)
    mu = g.mu.copy()
    mu[1] = np.nan
    with pytest.raises(api.PsiError, match="activity"):
        api.Operator(g.n, g.follower, g.leader, g.lam, mu)
    op = gpu_op(api, g)
    with pytest.raises(api.PsiError, match="tol"):
        op.solve(tol=0.0)
    with pytest.raises(api.PsiError, match="tile"):
        op.solve(tile_items=1000)
    # the binding refuses buffers the kernels would read or write past
    short = torch.ones(g.n - 1, dtype=torch.float64, device="cuda")
    with pytest.raises(ValueError, match="s0"):
        op.solve(s0=short)
    with pytest.raises(ValueError, match="s_in"):
        op.step(short)
    with pytest.raises(ValueError, match="must hold"):
        op.final(short)
    with pytest.raises(ValueError, match="psi_out"):
        op.solve(psi_out=torch.empty(g.n, dtype=torch.float32, device="cuda"))
    with pytest.raises(ValueError, match="psi_out"):
        op.solve(psi_out=torch.empty(2 * g.n, dtype=torch.float64, device="cuda")[::2])
    psi_buf = torch.empty(g.n, dtype=torch.float64, device="cuda")
    psi, info = op.solve(psi_out=psi_buf)
    assert info["status"] == 0 and psi.data_ptr() == psi_buf.data_ptr()


# ---------------------------------------------------------------- one step
@pytest.mark.parametrize("tile", [1024, 1536, 2048, 3072, 4096])
def test_step_matches_oracle(gpu_lib, tile):
    api = gpu_lib
    g = synth.chung_lu(30000, 15, 2.1, 11, sigma=2.0)
    op = gpu_op(api, g, flags=api.PSI_WEIGHTED_FP64)
    A, B, c, d = oracle.operator(g.n, g.follower, g.leader, g.lam, g.mu)
    s_in = np.random.default_rng(1).uniform(0.5, 3.0, g.n)
    expect = A.T @ s_in + c
    for prec in ("fp64", "fp64_weighted"):
        out, gap = op.step(torch.tensor(s_in, device="cuda"), precision=prec, tile_items=tile)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        np.testing.assert_allclose(got, expect, rtol=1e-13, atol=0)
        assert abs(gap.item() - np.abs(expect - s_in).sum()) <= 1e-12 * np.abs(expect - s_in).sum()
    psi = op.final(torch.tensor(s_in, device="cuda")).cpu().numpy()
    np.testing.assert_allclose(psi, (B.T @ s_in + d) / g.n, rtol=1e-13, atol=0)


@pytest.mark.parametrize("segs", [2, 4, 8])
@pytest.mark.parametrize("form,tile", [("tiles", 1024), ("tiles", 2048), ("tiles", 4096),
                                       ("slices", 0)])
def test_segmented_step_matches_oracle(gpu_lib, segs, form, tile):
    """Column-segmented pass (per-XCD-group partials + combine) vs the oracle,
    with the partial pass over merge-path tiles or over slices."""
    api = gpu_lib
    g = synth.chung_lu(40000, 15, 2.1, 13, sigma=2.0)
    op = gpu_op(api, g)
    A, B, c, d = oracle.operator(g.n, g.follower, g.leader, g.lam, g.mu)
    s_in = np.random.default_rng(2).uniform(0.5, 3.0, g.n)
    expect = A.T @ s_in + c
    out, gap = op.step(torch.tensor(s_in, device="cuda"), tile_items=tile, col_segments=segs,
                       seg_form=form)
    torch.cuda.synchronize()
    np.testing.assert_allclose(out.cpu().numpy(), expect, rtol=1e-13, atol=0)
    assert abs(gap.item() - np.abs(expect - s_in).sum()) <= 1e-12 * np.abs(expect - s_in).sum()
    for _ in range(3):  # bitwise repeatable
        again, gap2 = op.step(torch.tensor(s_in, device="cuda"), tile_items=tile, col_segments=segs,
                              seg_form=form)
        torch.cuda.synchronize()
        assert torch.equal(again, out) and torch.equal(gap2, gap)


@pytest.mark.parametrize("prec,tol,bar", [("fp64", 1e-9, 1e-9), ("mixed", 1e-9, 1e-9),
                                          ("fp32", 1e-5, 1e-6)])
@pytest.mark.parametrize("segs,form", [(1, "auto"), (2, "tiles"), (2, "slices"), (4, "tiles"),
                                       (4, "slices"), (8, "tiles"), (8, "slices"), (0, "bands")])
def test_segmented_solve(gpu_lib, prec, tol, bar, segs, form):
    api = gpu_lib
    g = synth.chung_lu(60000, 20, 2.2, 14, sigma=1.5)
    A, B, c, d, r = oracle_run(g, tol)
    op = gpu_op(api, g)
    psi, info = op.solve(tol=tol, precision=prec, col_segments=segs, seg_form=form)
    assert info["status"] == 0, info
    assert info["seg_form"] == (0 if segs == 1 else api.SEG_FORMS[form])
    elem = {"fp64": elem_bar_fp64(info, r), "mixed": 1e-6, "fp32": 1e-4}[prec]
    assert_psi(r["psi"], psi, bar, elem)


def _graph_with_rows(n, rows, m_background, seed):
    """Leader r gets the followers [lo, lo + k) for each (r, lo, k) in rows,
    plus m_background random edges."""
    rng = np.random.default_rng(seed)
    bf = rng.integers(0, n, m_background)
    bl = rng.integers(0, n, m_background)
    keep = ~np.isin(bl, [r for r, _, _ in rows])  # the listed rows keep their exact lengths
    f = [np.arange(lo, lo + k) for _, lo, k in rows] + [bf[keep]]
    l = [np.full(k, r) for r, _, k in rows] + [bl[keep]]
    lam = np.exp(rng.normal(0.0, 1.0, n))
    mu = np.exp(rng.normal(0.0, 1.0, n))
    return synth.Graph(n, np.concatenate(f).astype(np.int32), np.concatenate(l).astype(np.int32),
                       lam, mu)


@pytest.mark.parametrize("segs", [2, 4, 8])
def test_sliced_layout_row_lengths(gpu_lib, segs):
    """Rows at every boundary of the sliced layout: 31/32/33 followers in one
    segment (short row or chunk), one chunk of 2048 and two of 2049, exactly
    64 chunks, 66 chunks (the last chunk to finish sums more than 64
    partials), a row that straddles segment boundaries, and a last window of
    fewer than 4096 rows (N = 1.1e6)."""
    api = gpu_lib
    n = 1_100_000
    rows = [(7, 100, 135_001), (11, 100, 131_072), (13, 1000, 2048), (17, 5000, 2049),
            (19, 9000, 32), (23, 9100, 33), (29, 9200, 31), (31, 9300, 1),
            (4095, 20_000, 40), (4096, 21_000, 40), (n - 1, 30_000, 2050),
            (37, 130_000, 300_000)]
    g = _graph_with_rows(n, rows, 3 * n, 41)
    op = gpu_op(api, g)
    A, B, c, d = oracle.operator(g.n, g.follower, g.leader, g.lam, g.mu)
    s_in = np.random.default_rng(3).uniform(0.5, 3.0, g.n)
    expect = A.T @ s_in + c
    out, gap = op.step(torch.tensor(s_in, device="cuda"), col_segments=segs, seg_form="slices")
    torch.cuda.synchronize()
    np.testing.assert_allclose(out.cpu().numpy(), expect, rtol=1e-13, atol=0)
    for _ in range(2):  # bitwise repeatable, chunk partials summed in chunk order
        again, _ = op.step(torch.tensor(s_in, device="cuda"), col_segments=segs,
                           seg_form="slices")
        torch.cuda.synchronize()
        assert torch.equal(again, out)
    tiled, _ = op.step(torch.tensor(s_in, device="cuda"), col_segments=segs, seg_form="tiles")
    torch.cuda.synchronize()
    np.testing.assert_allclose(tiled.cpu().numpy(), expect, rtol=1e-13, atol=0)
    psi, info = op.solve(tol=1e-10, col_segments=segs, seg_form="slices")
    _, _, _, _, r = oracle_run(g, 1e-10)
    assert info["status"] == 0 and oracle.rel_l1(r["psi"], psi.cpu().numpy()) <= 1e-9


def test_sliced_layout_degenerate(gpu_lib):
    """N = 5 with 8 segments (three of them hold no column), and an operator
    with no edges, in every segment count."""
    api = gpu_lib
    f = np.array([1, 2, 3, 4, 0, 0], dtype=np.int32)
    l = np.array([0, 0, 0, 0, 4, 3], dtype=np.int32)
    lam = np.array([0.5, 1.0, 2.0, 0.7, 1.3])
    mu = np.array([1.0, 0.5, 0.2, 0.9, 0.4])
    s_in = np.array([1.0, 2.0, 3.0, 4.0, 5.0])
    for n, ff, ll in ((5, f, l), (5, f[:0], l[:0])):
        A, B, c, d = oracle.operator(n, ff, ll, lam, mu)
        op = api.Operator(n, ff, ll, lam, mu)
        for segs in (2, 4, 8):
            for form in ("slices", "tiles"):
                out, _ = op.step(torch.tensor(s_in, device="cuda"), col_segments=segs,
                                 seg_form=form)
                torch.cuda.synchronize()
                np.testing.assert_allclose(out.cpu().numpy(), A.T @ s_in + c, rtol=1e-15,
                                           atol=0)


def test_step_bitwise_repeatable(gpu_lib):
    api = gpu_lib
    g = synth.chung_lu(200000, 20, 2.1, 12, sigma=2.0)
    op = gpu_op(api, g)
    s_in = torch.rand(g.n, dtype=torch.float64, device="cuda") + 0.5
    ref, gref = op.step(s_in)
    for _ in range(5):
        out, gap = op.step(s_in)
        torch.cuda.synchronize()
        assert torch.equal(out, ref) and torch.equal(gap, gref)


# ---------------------------------------------------------------- full solves
SOLVE_CASES = [
    ("random_dangling", lambda: synth.random_small(200, 0.02, 21, dangling=True), 1e-12),
    ("random_closed", lambda: synth.random_small(180, 0.03, 22, dangling=False), 1e-12),
    ("cl_1k", lambda: synth.workload("cl_1k"), 1e-10),
    ("cl_50k_g2.1", lambda: synth.chung_lu(50000, 20, 2.1, 23, sigma=2.0), 1e-8),
    ("star_300k", lambda: synth.star(300001, 24), 1e-10),
    ("uniform_act", lambda: synth.chung_lu(20000, 8, 2.5, 25, activity_kind="uniform"), 1e-9),
]


@pytest.mark.parametrize("name,make,tol", SOLVE_CASES, ids=[c[0] for c in SOLVE_CASES])
def test_solve_fp64_matches_oracle(gpu_lib, name, make, tol):
    api = gpu_lib
    g = make()
    A, B, c, d, r = oracle_run(g, tol)
    op = gpu_op(api, g)
    psi, s, info = op.solve(tol=tol, return_s=True)
    psi = psi.cpu().numpy()
    assert info["status"] == 0, info
    assert abs(info["iterations"] - r["iterations"]) <= 1
    assert_psi(r["psi"], psi, 1e-9, elem_bar_fp64(info, r))
    assert_psi(r["s"], s, 1e-9, elem_bar_fp64(info, r))
    s_np = s.cpu().numpy()
    # the CPU's own evaluation of the residual rounds at about eps·Σ|s|
    assert oracle.fixed_point_residual(A, c, s_np) <= tol * 1.5 + 1e-15 * np.abs(s_np).sum()


@pytest.mark.parametrize("segs,form", [(1, "auto"), (4, "slices"), (1, "bands"), (1, "bins")])
def test_resume_from_a_checkpointed_iterate_is_bitwise_equal(gpu_lib, segs, form):
    """A solve stopped by max_iter (PSI_ENOTCONV) returns its iterate s_k;
    restarting from it (used as given) runs the remaining steps of eq.
    (power_psi) and ends on the same s and ψ, bit for bit, as an
    uninterrupted solve."""
    api = gpu_lib
    g = synth.chung_lu(60_000, 12, 2.2, 62, sigma=1.5)
    op = gpu_op(api, g)
    tol = 1e-10
    kw = dict(tile_items=2048, col_segments=segs, seg_form=form)
    psi, s, info = op.solve(tol=tol, return_s=True, **kw)
    assert info["status"] == 0
    t = info["iterations"]
    k = t // 2
    _, s_k, info_k = op.solve(tol=tol, max_iter=k, return_s=True, **kw)
    assert info_k["status_name"] == "PSI_ENOTCONV" and info_k["iterations"] == k
    psi2, s2, info2 = op.solve(tol=tol, s0=s_k, no_fallback=True, return_s=True, **kw)
    assert info2["status"] == 0 and info2["iterations"] == t - k, (info2, t, k)
    assert torch.equal(s2, s) and torch.equal(psi2, psi)


@pytest.mark.parametrize("segs,form", [(1, "auto"), (4, "slices"), (4, "tiles"), (1, "bins")])
def test_deferred_decision_stops_at_the_first_step_under_tol(gpu_lib, segs, form):
    """The solve loop decides each pass's gap in the next pass (deferred);
    single psi_step calls reduce it inside the pass.  Both run the same
    kernels, so the solve must stop exactly at the first step whose gap is
    at most tol, with that step's iterate bit for bit — one pass later would
    overshoot, a missed decision would run on."""
    api = gpu_lib
    g = synth.chung_lu(50_000, 12, 2.2, 61, sigma=1.5)
    op = gpu_op(api, g)
    A, B, c, d = oracle.operator(g.n, g.follower, g.leader, g.lam, g.mu)
    tol = 1e-9
    s = torch.tensor(c, device="cuda")
    t = 0
    while True:
        s_next, gap = op.step(s, tile_items=2048, col_segments=segs, seg_form=form)
        torch.cuda.synchronize()
        t += 1
        s = s_next
        if gap.item() <= tol:
            break
        assert t < 500
    psi, s_solve, info = op.solve(tol=tol, tile_items=2048, col_segments=segs, seg_form=form,
                                  return_s=True)
    assert info["status"] == 0, info
    assert info["iterations"] == t and info["spmv_passes"] == t + 1
    assert torch.equal(s_solve, s)
    for check_every in (1, 3, 64):  # batch ends at every step, mid-run, or past convergence
        _, s2, info2 = op.solve(tol=tol, tile_items=2048, col_segments=segs, seg_form=form,
                                check_every=check_every, return_s=True)
        assert info2["iterations"] == t and torch.equal(s2, s), (check_every, info2)


@pytest.mark.parametrize("form", ["auto", "bins"])
def test_star_hub_closed_form(gpu_lib, form):
    """One 3M-long row: ψ_h = d_h(1 + Σ_{j≠h} c_j)/N, ψ_j = d_j/N (in the
    binned layout the row is cut into hundreds of pieces over all follower
    blocks)."""
    api = gpu_lib
    g = synth.star(3_000_001, 26)
    op = gpu_op(api, g)
    psi, info = op.solve(tol=1e-10, seg_form=form)
    assert info["status"] == 0, info
    if form == "bins":
        assert op.bins_info()["split_rows"] == 1 and op.bins_info()["bins"] > 500
    psi = psi.cpu().numpy()
    c = g.mu / (g.lam + g.mu)
    d = g.lam / (g.lam + g.mu)
    expect = d / g.n
    expect[0] = d[0] * (1.0 + np.sort(c[1:]).sum()) / g.n
    np.testing.assert_allclose(psi, expect, rtol=1e-12, atol=0)


def test_solve_repeatable_and_tile_independent(gpu_lib):
    api = gpu_lib
    g = synth.chung_lu(100000, 20, 2.2, 27, sigma=1.5)
    op = gpu_op(api, g)
    ref, info = op.solve(tol=1e-8)
    for _ in range(3):
        again, info2 = op.solve(tol=1e-8)
        assert torch.equal(again, ref) and info2["iterations"] == info["iterations"]
    for tile in (1024, 3072, 4096):
        other, _ = op.solve(tol=1e-8, tile_items=tile)
        assert oracle.rel_l1(ref.cpu().numpy(), other.cpu().numpy()) <= 1e-12


@pytest.mark.parametrize("mode", ["bnorm", "rel_l1"])
def test_tol_modes(gpu_lib, mode):
    api = gpu_lib
    g = synth.chung_lu(5000, 10, 2.2, 28, sigma=1.0)
    tol = 1e-9 if mode == "bnorm" else 1e-13
    A, B, c, d, r = oracle_run(g, tol, tol_mode=mode)
    op = gpu_op(api, g)
    psi, info = op.solve(tol=tol, tol_mode=mode)
    assert abs(info["iterations"] - r["iterations"]) <= 1
    assert oracle.rel_l1(r["psi"], psi.cpu().numpy()) <= 1e-9


def test_weighted_form(gpu_lib):
    api = gpu_lib
    g = synth.chung_lu(40000, 15, 2.2, 29, sigma=1.5)
    A, B, c, d, r = oracle_run(g, 1e-9)
    op = gpu_op(api, g, flags=api.PSI_WEIGHTED_FP64)
    psi, info = op.solve(tol=1e-9, precision="fp64_weighted")
    assert info["status"] == 0
    assert_psi(r["psi"], psi, 1e-9, elem_bar_fp64(info, r))


def test_mixed_and_fp32(gpu_lib):
    api = gpu_lib
    g = synth.chung_lu(100000, 20, 2.2, 30, sigma=1.5)
    A, B, c, d, r = oracle_run(g, 1e-8)
    op = gpu_op(api, g)
    psi_m, s_m, info_m = op.solve(tol=1e-8, precision="mixed", return_s=True)
    assert info_m["status"] == 0, info_m
    assert info_m["fp32_passes"] > 0 and info_m["refinements"] >= 1
    assert_psi(r["psi"], psi_m, 1e-9, 1e-6)
    s_np = s_m.cpu().numpy()
    assert oracle.fixed_point_residual(A, c, s_np) <= 1.5e-8 + 1e-15 * np.abs(s_np).sum()
    psi_f, info_f = op.solve(tol=1e-4, precision="fp32")
    assert_psi(r["psi"], psi_f, 1e-6, 1e-4)


def test_edge_cases(gpu_lib):
    api = gpu_lib
    # no edges at all: s = c, ψ = d/N
    n = 7
    lam = np.linspace(0.5, 2.0, n)
    mu = np.linspace(1.0, 0.2, n)
    e = np.zeros(0, dtype=np.int32)
    op = api.Operator(n, e, e, lam, mu)
    psi, info = op.solve(tol=1e-12)
    np.testing.assert_allclose(psi.cpu().numpy(), lam / (lam + mu) / n, rtol=1e-15)
    # only self-loops and repeats
    f = np.array([0, 1, 1, 1, 2], dtype=np.int32)
    l = np.array([0, 2, 2, 2, 2], dtype=np.int32)
    op = api.Operator(3, f, l, lam[:3], mu[:3])
    st = op.stats()
    assert (st["n_edges"], st["n_self_loops"], st["n_duplicates"]) == (1, 2, 2)
    A, B, c, d = oracle.operator(3, f, l, lam[:3], mu[:3])
    psi, info = op.solve(tol=1e-14)
    np.testing.assert_allclose(psi.cpu().numpy(), oracle.psi_closed_form(A, B, c, d)[0],
                               rtol=1e-14)
    # μ = 0 for some users is allowed
    g = synth.chung_lu(3000, 10, 2.2, 31)
    mu0 = g.mu.copy()
    mu0[::3] = 0.0
    g0 = synth.Graph(g.n, g.follower, g.leader, g.lam, mu0)
    A, B, c, d, r = oracle_run(g0, 1e-10)
    psi, info = gpu_op(api, g0).solve(tol=1e-10)
    assert oracle.rel_l1(r["psi"], psi.cpu().numpy()) <= 1e-9


def test_termination_statuses(gpu_lib):
    api = gpu_lib
    g = synth.chung_lu(20000, 10, 2.2, 32)
    op = gpu_op(api, g)
    psi, info = op.solve(tol=1e-12, max_iter=3)
    assert info["status_name"] == "PSI_ENOTCONV" and info["iterations"] == 3
    with pytest.raises(api.PsiError, match="ENOTCONV"):
        op.solve(tol=1e-12, max_iter=2, raise_on_status=True)
    # the deterministic FP32 map either lands on an exact FP32 fixed point (gap 0)
    # or stops improving; both keep ψ within the FP32 bound
    A, B, c, d, r = oracle_run(g, 1e-12)
    psi, info = op.solve(tol=1e-14, precision="fp32")
    assert info["status_name"] in ("PSI_OK", "PSI_ESTAGNATED")
    assert oracle.rel_l1(r["psi"], psi.cpu().numpy()) <= 1e-6


def test_warm_start_and_fallback(gpu_lib):
    api = gpu_lib
    g = synth.chung_lu(50000, 20, 2.2, 33, sigma=1.5)
    op = gpu_op(api, g)
    ref, s_ref, info_cold = op.solve(tol=1e-8, return_s=True)
    # start from a nearly converged iterate: few iterations, same ψ
    # (the error contracts geometrically, so the saving is the log of the start's error)
    for rel, most in ((1e-6, 0.75 * info_cold["iterations"]), (1e-12, 6)):
        psi, info = op.solve(tol=1e-8, s0=s_ref * (1 + rel))
        assert info["used_s0"] == 1 and info["iterations"] <= most, (rel, info)
        assert oracle.rel_l1(ref.cpu().numpy(), psi.cpu().numpy()) <= 1e-9
    # a garbage start is rejected for c
    bad = torch.full_like(s_ref, 1e6)
    psi, info = op.solve(tol=1e-8, s0=bad)
    assert info["used_s0"] == 0
    assert oracle.rel_l1(ref.cpu().numpy(), psi.cpu().numpy()) <= 1e-9
    # unless asked to keep it: still converges to the same fixed point
    psi, info = op.solve(tol=1e-8, s0=bad, no_fallback=True)
    assert info["used_s0"] == 1
    assert oracle.rel_l1(ref.cpu().numpy(), psi.cpu().numpy()) <= 1e-9
    # the residual of c is kept by the operator and the step from a kept s0 is the
    # first iteration: a warm FP64 solve runs no pass beyond its iterations and ψ
    psi, info = op.solve(tol=1e-8, s0=s_ref * (1 + 1e-6))
    assert info["used_s0"] == 1 and info["spmv_passes"] == info["iterations"] + 1
    psi, info = op.solve(tol=1e-8, s0=bad)
    assert info["used_s0"] == 0 and info["spmv_passes"] == info["iterations"] + 2
    assert oracle.rel_l1(ref.cpu().numpy(), psi.cpu().numpy()) <= 1e-9
    # the other precisions compare residuals the same way
    psi, info = op.solve(tol=1e-8, precision="mixed", s0=s_ref * (1 + 1e-6))
    assert info["status"] == 0 and info["used_s0"] == 1
    assert oracle.rel_l1(ref.cpu().numpy(), psi.cpu().numpy()) <= 1e-9


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_full_size_1m(gpu_lib, prec):
    """The measured workload (N = 1,000,000, mean degree 20, γ = 2.2, σ = 1.5,
    tol 1e-8), element by element against the oracle, in the schedule the
    autotuner picks (the launch configuration the benchmark times)."""
    api = gpu_lib
    g = synth.workload("cl_1m")
    A, B, c, d, r = oracle_run(g, 1e-8)
    op = gpu_op(api, g)
    tuned = op.autotune(prec)
    psi, s, info = op.solve(tol=1e-8, precision=prec, return_s=True)
    assert info["status"] == 0, info
    assert info["col_segments"] == tuned["col_segments"], (info, tuned)
    assert_psi(r["psi"], psi, 1e-9, elem_bar_fp64(info, r) if prec == "fp64" else 1e-6)
    assert oracle.rel_l2(r["psi"], psi.cpu().numpy()) <= 1e-9
    s_np = s.cpu().numpy()
    assert oracle.fixed_point_residual(A, c, s_np) <= 1.5e-8 + 1e-15 * np.abs(s_np).sum()


def test_autotune_picks_a_supported_schedule_that_solves_use(gpu_lib):
    api = gpu_lib
    g = synth.chung_lu(200_000, 12, 2.2, 31, sigma=1.5)
    op = api.Operator(g.n, g.follower, g.leader, g.lam, g.mu)
    ref, _ = op.solve(tol=1e-10)
    ref = ref.cpu().numpy()
    for prec, bar in (("fp64", 1e-12), ("mixed", 1e-9)):
        t = op.autotune(prec, reps=3)
        assert t["tile_items"] in (1024, 1536, 2048, 3072, 4096)
        assert t["col_segments"] in (1, 2, 4, 8) and t["pass_ms"] > 0
        assert t["seg_form"] in ("none", "tiles", "slices", "bands", "bins")
        if t["seg_form"] not in ("bands", "bins"):
            assert t["seg_form"] == ("none" if t["col_segments"] == 1 else t["seg_form"])
        psi, info = op.solve(tol=1e-10, precision=prec)
        assert info["status"] == 0
        assert (info["tile_items"], info["col_segments"]) == (t["tile_items"], t["col_segments"])
        assert api.SEG_FORM_NAMES[info["seg_form"]] == t["seg_form"]
        assert oracle.rel_l1(ref, psi.cpu().numpy()) <= bar
        # an explicit choice still wins over the tuned one
        _, info2 = op.solve(tol=1e-10, precision=prec, tile_items=1024, col_segments=1)
        assert (info2["tile_items"], info2["col_segments"]) == (1024, 1)
    with pytest.raises(api.PsiError, match="WEIGHTED"):
        op.autotune("fp64_weighted")


@pytest.mark.parametrize("power_method", [True, False])
def test_pagerank_mode_matches_the_power_method(gpu_lib, power_method):
    """Homogeneous activity on the same kernels gives the PageRank vector; with
    the power method's start and π-tolerance, its iterates and count too."""
    api = gpu_lib
    g = synth.chung_lu(30_000, 8, 2.2, 57)  # some users follow nobody: leaking PageRank
    W = oracle.transition_matrix(g.n, g.follower, g.leader)
    pi_ref, t_ref = oracle.pagerank_power(W, 0.85, 1e-10)
    pi, info, _ = api.pagerank(g.n, g.follower, g.leader, alpha=0.85, tol=1e-10,
                               power_method=power_method)
    assert info["status"] == 0
    pi = pi.cpu().numpy()
    if power_method:
        # the same stopping step; ψ from s_t is π_{t+1}, one step past the oracle's π_t
        assert abs(info["iterations"] - t_ref) <= 1
        assert oracle.rel_l1(pi_ref, pi) <= 1e-9
    else:
        exact, _ = oracle.pagerank_power(W, 0.85, 1e-15)
        assert oracle.rel_l1(exact, pi) <= 1e-8


def test_pagerank_entry_point_checks_the_activity_and_maps_the_tolerance(gpu_lib):
    """psi_pagerank refuses an operator whose activity is not λ = 1 − α,
    μ = α; in the power-method form the relative tolerance is scale-free, so
    it stops at the oracle's step for the same relative π-tolerance."""
    import ctypes
    from paper_2206_09960_amd import _ffi
    api = gpu_lib
    g = synth.chung_lu(20_000, 8, 2.2, 58)
    op = api.Operator(g.n, g.follower, g.leader, g.lam, g.mu)  # heterogeneous activity
    with pytest.raises(api.PsiError, match="lambda = 1 - alpha"):
        api.pagerank(g.n, g.follower, g.leader, alpha=0.85, op=op)
    W = oracle.transition_matrix(g.n, g.follower, g.leader)
    op = api.Operator(g.n, g.follower, g.leader, np.full(g.n, 0.15), np.full(g.n, 0.85))
    p = op._params(1e-9, "rel_l1", 10_000, "fp64", 0)
    pi = torch.empty(g.n, dtype=torch.float64, device="cuda")
    start = torch.empty(g.n, dtype=torch.float64, device="cuda")
    info = _ffi.Info()
    st = op._lib.psi_pagerank(op._h, 0.85, ctypes.byref(p), 1, start.data_ptr(), pi.data_ptr(),
                              ctypes.byref(info), None)
    assert st == 0
    # s_0 = K/N with K = αN/(1 − α)
    assert torch.all(start == 0.85 * g.n / (1.0 - 0.85) / g.n)
    # the oracle's relative step test: ‖π_t − π_{t−1}‖₁ / ‖π_t‖₁ ≤ tol
    x = np.full(g.n, 1.0 / g.n)
    t = 0
    while True:
        x_new = 0.85 * (W.T @ x) + 0.15 / g.n
        t += 1
        if np.abs(x_new - x).sum() / np.abs(x_new).sum() <= 1e-9:
            break
        x = x_new
    assert abs(info.iterations - t) <= 1
    assert oracle.rel_l1(x_new, pi.cpu().numpy()) <= 1e-8
    with pytest.raises(api.PsiError, match="alpha"):
        api.pagerank(g.n, g.follower, g.leader, alpha=1.0, op=op)


def test_exact_fixed_point_equals_the_closed_form(gpu_lib):
    """The reference ψ of the experiments (FP64 map run until its step stops
    shrinking) against eq. (ultimsol) solved exactly by the oracle."""
    api = gpu_lib
    g = synth.chung_lu(12_591, 49_743 / 12_591, 2.2, 21, activity_kind="uniform")
    op = api.Operator(g.n, g.follower, g.leader, g.lam, g.mu)
    psi, info = op.solve(tol=1e-300, max_iter=2000)
    assert info["status_name"] in ("PSI_OK", "PSI_ESTAGNATED")
    A, B, c, d = oracle.operator(g.n, g.follower, g.leader, g.lam, g.mu)
    exact, _ = oracle.psi_closed_form(A, B, c, d)
    assert oracle.rel_l1(exact, psi.cpu().numpy()) <= 1e-12


@pytest.mark.parametrize("n,deg,gamma,sigma,tol,depth", [
    (50_000, 12, 2.2, 1.5, 1e-10, 4),
    (200_000, 20, 2.1, 2.0, 1e-8, 1),
    (200_000, 20, 2.1, 2.0, 1e-8, 8),
])
def test_anderson_matches_oracle_in_fewer_passes(gpu_lib, n, deg, gamma, sigma, tol, depth):
    api = gpu_lib
    g = synth.chung_lu(n, deg, gamma, 91, sigma=sigma)
    op = api.Operator(g.n, g.follower, g.leader, g.lam, g.mu)
    A, B, c, d = oracle.operator(g.n, g.follower, g.leader, g.lam, g.mu)
    r = oracle.power_psi(A, B, c, d, tol)
    psi, s, info = op.solve_anderson(tol=tol, depth=depth, return_s=True)
    assert info["status"] == 0, info
    psi, s = psi.cpu().numpy(), s.cpu().numpy()
    assert oracle.rel_l1(r["psi"], psi) <= 1e-9
    # the returned s is a Power-ψ step of size <= tol: its own residual is below tol too
    res = oracle.fixed_point_residual(A, c, s)
    assert res <= 1.5 * tol + 1e-15 * np.abs(s).sum(), res
    if depth > 1:
        assert info["iterations"] < r["iterations"], (info["iterations"], r["iterations"])
    again, _ = op.solve_anderson(tol=tol, depth=depth)
    assert np.array_equal(again.cpu().numpy(), psi)
    # a start far from the fixed point converges to the same ψ
    s0 = torch.tensor(np.full(g.n, 3.0))
    psi2, info2 = op.solve_anderson(tol=tol, depth=depth, s0=s0)
    assert info2["status"] == 0 and info2["used_s0"] == 1
    assert oracle.rel_l1(r["psi"], psi2.cpu().numpy()) <= 1e-9


@pytest.mark.parametrize("seg_form", [0, "bins"])
def test_anderson_mixed_matches_oracle_in_fewer_passes(gpu_lib, seg_form):
    """Accelerated FP32 corrections between FP64 residual passes: the oracle's
    ψ at the same tolerance, s a Power-ψ step of size <= tol, and fewer passes
    than the plain mixed refinement."""
    api = gpu_lib
    tol = 1e-9
    g = synth.chung_lu(300_000, 20, 2.1, 15, sigma=2.0)
    A, B, c, d = oracle.operator(g.n, g.follower, g.leader, g.lam, g.mu)
    r = oracle.power_psi(A, B, c, d, tol)
    op = api.Operator(g.n, g.follower, g.leader, g.lam, g.mu)
    psi, s, info = op.solve_anderson(tol=tol, depth=4, precision="mixed", seg_form=seg_form,
                                     return_s=True)
    assert info["status"] == 0, info
    assert info["refinements"] >= 1 and info["fp32_passes"] > 0, info
    got = psi.cpu().numpy()
    assert oracle.rel_l1(r["psi"], got) <= 1e-9
    assert oracle.max_rel(r["psi"], got) <= 1e-6
    res = oracle.fixed_point_residual(A, c, s.cpu().numpy())
    assert res <= 1.5 * tol + 1e-15 * np.abs(r["s"]).sum(), res
    _, plain = op.solve(tol=tol, precision="mixed", seg_form=seg_form)
    assert info["spmv_passes"] < plain["spmv_passes"], (info["spmv_passes"],
                                                        plain["spmv_passes"])
    again, _ = op.solve_anderson(tol=tol, depth=4, precision="mixed", seg_form=seg_form)
    assert torch.equal(again, psi)


def test_anderson_invalid(gpu_lib):
    api = gpu_lib
    g = synth.chung_lu(2000, 5, 2.2, 92)
    op = api.Operator(g.n, g.follower, g.leader, g.lam, g.mu)
    with pytest.raises(api.PsiError, match="depth"):
        op.solve_anderson(depth=9)
    with pytest.raises(api.PsiError, match="PSI_PREC_FP64 or PSI_PREC_MIXED"):
        op.solve_anderson(precision="fp32")
    psi, info = op.solve_anderson(tol=1e-14, max_iter=3)
    assert info["status_name"] == "PSI_ENOTCONV" and info["iterations"] == 3


def test_gather_probe_runs_and_clamps(gpu_lib):
    api = gpu_lib
    r = api.gather_probe(100_000, 1_000_000, col_segments=4, reps=2)
    assert r["ms"] > 0 and r["gathers_per_s"] > 1e9
    # indices outside the segment are clamped, not read out of bounds
    x = torch.arange(16, dtype=torch.float64, device="cuda")
    idx = torch.tensor([0, 3, 100, -5], dtype=torch.int32, device="cuda")
    out = torch.zeros(8, dtype=torch.float64, device="cuda")
    ms = ctypes.c_double()
    assert api.load().psi_gather_probe(x.data_ptr(), 16, 2, idx.data_ptr(), 4, out.data_ptr(), 8,
                                       1, ctypes.byref(ms), api._stream_handle(None)) == 0
    # workgroup 0 gathers segment 0 (entries 0..7): 0 + 3 + 7 + 7
    assert out[0].item() == 17.0


@pytest.mark.parametrize("segs,form", [(1, "auto"), (4, "tiles"), (4, "slices")])
def test_a_wait_that_gives_up_fails_the_call_and_is_recovered(gpu_lib, segs, form):
    """The host forces every bounded wait of the passes to give up at once (no
    wait runs long; every kernel ends normally): the solve must fail with
    PSI_EDEVICE instead of returning a ψ built from missing partials, and the
    next solve, with normal waits, must be exact again (the partials left in
    their slots were emptied)."""
    api = gpu_lib
    g = synth.star(300001, 24)  # one 300k-follower hub: its row spans many tiles and chunks
    A, B, c, d, r = oracle_run(g, 1e-10)
    op = gpu_op(api, g)
    op.debug_force_slot_timeout(True)
    with pytest.raises(api.PsiError) as e:
        op.solve(tol=1e-10, col_segments=segs, seg_form=form)
    assert e.value.status == 5  # PSI_EDEVICE
    with pytest.raises(api.PsiError):
        op.solve(tol=1e-10, precision="mixed", col_segments=segs, seg_form=form)
    op.debug_force_slot_timeout(False)
    for prec in ("fp64", "mixed"):
        psi, info = op.solve(tol=1e-10, precision=prec, col_segments=segs, seg_form=form)
        assert info["status"] == 0, info
        assert_psi(r["psi"], psi, 1e-9, 1e-6)
