"""The smallest inputs through every entry point: a single user (a self-loop
is the only edge it can have, and the build drops it, so s = c and ψ = d,
Sec. II), and block-diagonal batches whose graphs hold one or two users."""
import numpy as np
import pytest
import torch

import oracle
from oracle import mpnn_oracle as mo

pytestmark = pytest.mark.gpu

LAM1 = np.array([0.8])
MU1 = np.array([0.6])
D1 = LAM1 / (LAM1 + MU1)
C1 = MU1 / (LAM1 + MU1)


def one_user(api):
    loop = np.array([0], dtype=np.int32)
    op = api.Operator(1, loop, loop, LAM1, MU1)
    st = op.stats()
    assert (st["n_edges"], st["n_self_loops"], st["n_no_leaders"]) == (0, 1, 1)
    return op


def test_one_user_every_solver(gpu_lib):
    api = gpu_lib
    op = one_user(api)
    ref = oracle.power_psi(*oracle.operator(1, np.zeros(0, np.int32), np.zeros(0, np.int32),
                                            LAM1, MU1), 1e-12)
    np.testing.assert_array_equal(ref["psi"], D1)
    for prec in ("fp64", "mixed", "fp32"):
        psi, info = op.solve(tol=1e-12, precision=prec)
        assert info["status"] == 0, (prec, info["status_name"])
        np.testing.assert_allclose(psi.cpu().numpy(), D1, rtol=1e-15, err_msg=prec)
    psi, s, info = op.solve(tol=1e-12, return_s=True)
    assert info["iterations"] == ref["iterations"]
    np.testing.assert_allclose(s.cpu().numpy(), C1, rtol=1e-15)
    for segs in (1, 2):
        out, gap = op.step(torch.tensor([5.0], device="cuda"), col_segments=segs)
        torch.cuda.synchronize()
        np.testing.assert_allclose(out.cpu().numpy(), C1, rtol=1e-15)  # no leader: y = 0
        assert abs(gap.item() - abs(C1[0] - 5.0)) <= 1e-15
    np.testing.assert_allclose(op.final(torch.tensor([3.0], device="cuda")).cpu().numpy(), D1,
                               rtol=1e-15)
    psi, info = op.solve_anderson(tol=1e-12, depth=2)
    assert info["status"] == 0
    np.testing.assert_allclose(psi.cpu().numpy(), D1, rtol=1e-15)
    # the band layout (one column block, one row block) and its sweeps
    psi, info = op.solve(tol=1e-12, seg_form="bands", band_col_log=17, band_rows=1280)
    assert info["status"] == 0
    np.testing.assert_allclose(psi.cpu().numpy(), D1, rtol=1e-15)
    assert op.band_info()["bands"] == 1
    psi, info = op.solve_async(tol=1e-12)
    assert info["status"] == 0
    np.testing.assert_allclose(psi.cpu().numpy(), D1, rtol=1e-15)


def test_one_user_batches_and_warm_start(gpu_lib):
    api = gpu_lib
    op = one_user(api)
    lam = torch.tensor([[0.8, 2.0, 0.1]], dtype=torch.float64)
    mu = torch.tensor([[0.6, 0.0, 3.0]], dtype=torch.float64)
    for prec in ("fp64", "mixed"):
        psi, infos = op.solve_batched(lam, mu, tol=1e-12, precision=prec)
        assert all(i["status"] == 0 for i in infos), prec
        np.testing.assert_allclose(psi.cpu().numpy(), (lam / (lam + mu)).numpy(), rtol=1e-15)
        # one scenario per lane group (eight groups of one lane)
        psi1, infos1 = op.solve_batched(lam, mu, tol=1e-12, precision=prec, batch_tile=1)
        assert all(i["status"] == 0 and i["batch_tile"] == 1 for i in infos1), prec
        assert torch.equal(psi1, psi)
        t = op.autotune_batched(3, prec)
        assert t["batch_tile"] == 3
    psi, p, infos = op.solve_origins([0], tol=1e-12)
    assert infos[0]["status"] == 0
    # Algorithm 1 for the only origin: its newsfeed is empty, so p = 0 and ψ = d
    np.testing.assert_array_equal(p.cpu().numpy(), [[0.0]])
    np.testing.assert_allclose(psi.cpu().numpy(), D1, rtol=1e-15)
    theta = mo.init_params(3)
    model = api.Model(theta)
    t_hat, s0 = model.forward(op)
    ga = mo.graph_arrays(1, np.zeros(0, np.int32), np.zeros(0, np.int32), LAM1, MU1)
    t_ref, _ = mo.forward(theta, ga, bf16_storage=True)
    assert abs(t_hat.item() - t_ref[0]) <= 1e-2 * abs(t_ref[0]) + 1e-3
    psi, info = op.solve(tol=1e-12, s0=s0)
    assert info["status"] == 0
    np.testing.assert_allclose(psi.cpu().numpy(), D1, rtol=1e-15)


@pytest.mark.parametrize("segs,form", [(1, "tiles"), (2, "tiles"), (2, "slices")])
def test_graphs_of_one_and_two_users(gpu_lib, segs, form):
    api = gpu_lib
    # graphs {0}, {1, 2}, {3}, {4}: user 1 follows user 2, user 3 has a self-loop
    offs = np.array([0, 1, 3, 4, 5], dtype=np.int64)
    f = np.array([1, 3], dtype=np.int32)
    l = np.array([2, 3], dtype=np.int32)
    lam = np.array([0.8, 1.5, 0.4, 2.0, 0.3])
    mu = np.array([0.6, 0.5, 1.2, 0.0, 0.9])
    op = api.Operator(5, f, l, lam, mu, node_offsets=offs)
    d = lam / (lam + mu)
    A, B, c, dd = oracle.operator(2, np.array([0], np.int32), np.array([1], np.int32),
                                  lam[1:3], mu[1:3])
    ref = oracle.power_psi(A, B, c, dd, 1e-12)
    for prec in ("fp64", "mixed"):
        psi, infos = op.solve_graphs(tol=1e-12, col_segments=segs, seg_form=form, precision=prec)
        psi = psi.cpu().numpy()
        assert len(infos) == 4 and all(i["status"] == 0 for i in infos), prec
        for u in (0, 3, 4):  # one-user graphs: ψ = d
            assert abs(psi[u] - d[u]) <= 1e-15 * d[u], prec
        assert oracle.rel_l1(ref["psi"], psi[1:3]) <= 1e-14, prec
    t = op.autotune_graphs("mixed", tol=1e-12)
    assert t["col_segments"] in (1, 2, 4)
