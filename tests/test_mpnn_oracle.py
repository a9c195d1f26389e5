"""Pins of the learned warm start's CPU oracle: central finite differences of
its loss, the bfloat16 rounding against its definition, and Adam against a
hand-computed first step."""
import numpy as np

import oracle
import oracle.mpnn_oracle as mo
import synth


def small_graph(seed=61, n=60):
    g = synth.random_small(n, 0.08, seed, dangling=True)
    ga = mo.graph_arrays(g.n, g.follower, g.leader, g.lam, g.mu)
    A, B, c, d = oracle.operator(g.n, g.follower, g.leader, g.lam, g.mu)
    s = oracle.power_psi(A, B, c, d, 1e-13)["s"]
    t, mask = mo.target(s, c)
    return g, ga, t, mask


def test_param_count():
    assert mo.param_count() == 8 * 64 + 64 + 3 * (64 * 32 + 96 * 64 + 64) + 64 + 1
    theta = mo.init_params(0)
    assert theta.size == mo.param_count()
    assert np.array_equal(mo.pack(mo.unpack(theta)), theta)


def test_gradient_matches_central_differences():
    g, ga, t, mask = small_graph()
    theta = mo.init_params(3)
    loss, grad = mo.loss_and_grad(theta, ga, t, mask)
    rng = np.random.default_rng(4)
    idx = rng.choice(theta.size, 60, replace=False)
    h = 1e-6
    for k in idx:
        tp = theta.copy(); tp[k] += h
        tm = theta.copy(); tm[k] -= h
        lp, _ = mo.loss_and_grad(tp, ga, t, mask)
        lm, _ = mo.loss_and_grad(tm, ga, t, mask)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - grad[k]) <= 1e-6 * max(1.0, abs(fd)), (k, fd, grad[k])


def test_gradient_direction_decreases_loss():
    g, ga, t, mask = small_graph(62)
    theta = mo.init_params(5)
    loss, grad = mo.loss_and_grad(theta, ga, t, mask)
    loss2, _ = mo.loss_and_grad(theta - 1e-4 * grad / np.linalg.norm(grad), ga, t, mask)
    assert loss2 < loss


def test_bf16_rounding():
    x = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 2 ** -7 + 2 ** -9, -3.1415926, 0.0, 65504.0])
    r = mo.bf16(x)
    assert r[0] == 1.0 and r[1] == 1.0  # tie rounds to even
    # 1 + 2^-7 + 2^-9 lies below the midpoint 1 + 2^-7 + 2^-8 of its two
    # neighbours 1 + 2^-7 and 1 + 2^-6: only the lower one is correct
    assert r[2] == 1.0 + 2 ** -7
    assert abs(r[3] + 3.140625) < 1e-12 and r[4] == 0.0
    # every rounded value has at most 8 significant bits
    for v in r[r != 0]:
        m, e = np.frexp(abs(v))
        assert (m * 2 ** 8) == np.floor(m * 2 ** 8)


def test_adam_first_step():
    theta = np.array([1.0, -2.0])
    grad = np.array([0.5, -0.25])
    th, m, v = mo.adam(theta, grad, np.zeros(2), np.zeros(2), 1, lr=0.1)
    # first bias-corrected step moves each weight by lr * sign(grad)
    np.testing.assert_allclose(th, theta - 0.1 * np.sign(grad), rtol=0, atol=1e-7)


def test_warm_start_is_at_least_c():
    g, ga, t, mask = small_graph(63)
    s0 = mo.warm_start(mo.init_params(7), ga)
    assert np.all(s0 >= ga["c"])
