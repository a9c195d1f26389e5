"""The entry point for callers that cannot allocate device memory
(psi_solve_anderson_noalloc, through the C ABI) against the workspace entry
point it mirrors (psi_solve_anderson): the same kernels on the same inputs,
so the same bits, in FP64 and in mixed precision; two calls in a row, the
second on a smaller graph (the fixed scratch keeps the first call's
contents), and the size limit."""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu


def test_no_alloc_anderson_equals_the_workspace_entry_point(gpu_lib):
    api = gpu_lib
    for n, seed in ((300_000, 71), (40_000, 72)):  # the second call on a smaller input
        g = synth.chung_lu(n, 12, 2.2, seed, sigma=1.5)
        op = api.Operator(g.n, g.follower, g.leader, g.lam, g.mu)
        psi_ws, s_ws, info_ws = op.solve_anderson(tol=1e-10, depth=4, return_s=True)
        psi_na, s_na, info_na = op.solve_anderson_noalloc(tol=1e-10, depth=4, return_s=True)
        assert info_na["status"] == 0, info_na
        assert torch.equal(psi_na, psi_ws) and torch.equal(s_na, s_ws)
        assert info_na["iterations"] == info_ws["iterations"]
        A, B, c, d = oracle.operator(g.n, g.follower, g.leader, g.lam, g.mu)
        r = oracle.power_psi(A, B, c, d, 1e-10)
        assert oracle.rel_l1(r["psi"], psi_na.cpu().numpy()) <= 1e-9
        # mixed precision: the FP32 window in the same scratch, after the FP64 call
        psi_wm, info_wm = op.solve_anderson(tol=1e-10, depth=4, precision="mixed")
        psi_nm, info_nm = op.solve_anderson_noalloc(tol=1e-10, depth=4, precision="mixed")
        assert info_nm["status"] == 0, info_nm
        assert torch.equal(psi_nm, psi_wm)
        assert (info_nm["iterations"], info_nm["fp32_passes"]) == (info_wm["iterations"],
                                                                   info_wm["fp32_passes"])
        assert oracle.rel_l1(r["psi"], psi_nm.cpu().numpy()) <= 1e-9


def test_no_alloc_anderson_refuses_more_than_its_scratch(gpu_lib):
    api = gpu_lib
    n = 900_000  # 80 bytes per user at depth 4: 72 MB, above the fixed 64 MiB
    rng = np.random.default_rng(3)
    f = rng.integers(0, n, 2 * n).astype(np.int32)
    l = rng.integers(0, n, 2 * n).astype(np.int32)
    op = api.Operator(n, f, l, np.ones(n), np.ones(n))
    with pytest.raises(api.PsiError, match="fixed"):
        op.solve_anderson_noalloc(tol=1e-8, depth=4)
    psi, info = op.solve_anderson_noalloc(tol=1e-8, depth=1)  # 32 bytes per user fit
    assert info["status"] == 0
    ref, _ = op.solve_anderson(tol=1e-8, depth=1)
    assert torch.equal(psi, ref)
