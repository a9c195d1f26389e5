"""Seeded sweep over small random graphs: every solver mode against the
oracle's Algorithm 2 on the same graph and activity.

Each case draws a graph (Erdős–Rényi-style with users who follow nobody,
repeated edges and self-loops in the input, or a small Chung–Lu graph with
hubs) and checks the plain solve in both pass forms and segment counts, the
band and binned layouts (FP64 and mixed precision), the mixed-precision
solve, Anderson acceleration (FP64 and mixed precision), and the scenario
batch in both precisions,
each within 1e-9 relative L1 of the oracle at the same tolerance.
"""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

TOL = 1e-10
BAR = 1e-9


def draw(seed):
    if seed % 2 == 0:
        n = 60 + 37 * seed
        return synth.random_small(n, 4.0 / n, 100 + seed, dangling=seed % 4 == 0,
                                  extra_self_loops=seed, extra_duplicates=2 * seed)
    return synth.chung_lu(1500 + 700 * seed, 8 + seed, 2.1 + 0.05 * seed, 200 + seed, sigma=1.5)


@pytest.mark.parametrize("seed", range(10))
def test_all_modes_match_the_oracle(gpu_lib, seed):
    api = gpu_lib
    g = draw(seed)
    A, B, c, d = oracle.operator(g.n, g.follower, g.leader, g.lam, g.mu)
    ref = oracle.power_psi(A, B, c, d, TOL)
    op = api.Operator(g.n, g.follower, g.leader, g.lam, g.mu)

    def check(psi, info, what, exact_iters=False):
        assert info["status"] == 0, (what, info["status_name"])
        err = oracle.rel_l1(ref["psi"], psi.cpu().numpy())
        assert err <= BAR, (what, err)
        if exact_iters:
            assert abs(info["iterations"] - ref["iterations"]) <= 1, (what, info["iterations"])

    psi, info = op.solve(tol=TOL, col_segments=1)
    check(psi, info, "fp64 fused", exact_iters=True)
    segs = (2, 4, 8)[seed % 3]
    for form in ("tiles", "slices"):
        psi, info = op.solve(tol=TOL, col_segments=segs, seg_form=form)
        assert info["col_segments"] == segs
        check(psi, info, f"fp64 S={segs} {form}", exact_iters=True)
    psi, info = op.solve(tol=TOL, precision="mixed")
    check(psi, info, "mixed")
    for form in ("bands", "bins"):
        for prec in ("fp64", "mixed"):
            psi, info = op.solve(tol=TOL, precision=prec, seg_form=form)
            assert info["seg_form"] == api.SEG_FORMS[form]
            check(psi, info, f"{prec} {form}", exact_iters=prec == "fp64")
    psi, info = op.solve_anderson(tol=TOL, depth=1 + seed % 4)
    check(psi, info, "anderson")
    psi, info = op.solve_anderson(tol=TOL, depth=1 + seed % 4, precision="mixed",
                                  seg_form=("bins", 0)[seed % 2])
    check(psi, info, "mixed anderson")

    # three scenarios: the operator's own activity and two more draws
    k = 3
    lam = np.empty((g.n, k))
    mu = np.empty((g.n, k))
    lam[:, 0], mu[:, 0] = g.lam, g.mu
    for s in range(1, k):
        lam[:, s], mu[:, s] = synth.activity(g.n, 300 + seed, "lognormal", 1.0 + 0.25 * s,
                                             scenario=s)
    refs = [ref] + [oracle.power_psi(*oracle.operator(g.n, g.follower, g.leader, lam[:, s],
                                                      mu[:, s]), TOL) for s in range(1, k)]
    for prec in ("fp64", "mixed"):
        psi_b, infos = op.solve_batched(torch.tensor(lam), torch.tensor(mu), tol=TOL,
                                        precision=prec)
        psi_b = psi_b.cpu().numpy()
        for s in range(k):
            assert infos[s]["status"] == 0, (prec, s, infos[s]["status_name"])
            err = oracle.rel_l1(refs[s]["psi"], psi_b[:, s])
            assert err <= BAR, (prec, s, err)
