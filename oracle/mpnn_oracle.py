"""CPU oracle of the learned warm start — TEST INFRASTRUCTURE ONLY.

The warm start is an extension of the method (the paper has no learned part): a
small message-passing network predicts t_i = log(s_i / c_i) for the fixed
point s of eq. (power_psi) (s ≥ c because A and c are non-negative), and the
solver starts from s0 = c ⊙ exp(t̂).  The network, in the order the GPU runs
it:

    x0_i  = [log λ_i, log(μ_i + 1e-12), c_i, d_i, log(1+|F(i)|),
             log(1+|L(i)|), log(1+den_i), log(λ_i + μ_i)]       (8 features)
    h     = ReLU(x0 Win + bin)                                  (64)
    3 ×:  p_j = (h_j Wm) / den_j                                (32, the
                message of user j, scaled by the column weight 1/den_j
                that A gives j's leaders, without μ)
          m_i = log(1 + ReLU((λ_i + μ_i) Σ_{j∈F(i)} p_j))        (the pull
                pattern of Aᵀ; the receiver factor and the log make one
                layer able to express log(s_i/c_i) = log(1 + (λ_i + μ_i)
                Σ_j s_j/den_j), which the fixed point satisfies exactly)
          h   = ReLU([h | m] Wl + bl)                           (96 → 64)
    out_i = h_i · w_out + b_out;   t̂_i = softplus(out_i)
    loss  = mean over users with c_i > 0 of (t̂_i − t_i)²

Parameters are one flat FP32 vector in the order Win [8×64], bin [64], then
per layer Wm [64×32], Wl [96×64], bl [64], then w_out [64], b_out [1].

Everything here is FP64.  With ``bf16_storage=True`` the values the GPU stores in
bfloat16 (Wm, Wl, and h, the scaled message p and m after each layer) are rounded the same way
(round to nearest even) so GPU and oracle differ only by FP32 summation
order; the backward pass treats the rounding as the identity, as the GPU does.

Pins: the gradient against central finite differences of the loss, a descent
step lowering the loss, the bfloat16 rounding against its definition and the
first Adam step against its closed form.  How well a trained network predicts
t has no reference value in the paper: that quality is parity unpinned, and the
solver, which keeps c whenever s0's residual is larger, alone decides ψ.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

F0, H, MSG, LAYERS = 8, 64, 32, 3


def param_count() -> int:
    return F0 * H + H + LAYERS * (H * MSG + (H + MSG) * H + H) + H + 1


def unpack(theta):
    theta = np.asarray(theta, dtype=np.float64)
    out = {}
    k = 0

    def take(name, shape):
        nonlocal k
        size = int(np.prod(shape))
        out[name] = theta[k:k + size].reshape(shape)
        k += size

    take("Win", (F0, H))
    take("bin", (H,))
    for l in range(LAYERS):
        take(f"Wm{l}", (H, MSG))
        take(f"Wl{l}", (H + MSG, H))
        take(f"bl{l}", (H,))
    take("w_out", (H,))
    take("b_out", (1,))
    assert k == theta.size
    return out


def pack(params) -> np.ndarray:
    parts = [params["Win"].ravel(), params["bin"]]
    for l in range(LAYERS):
        parts += [params[f"Wm{l}"].ravel(), params[f"Wl{l}"].ravel(), params[f"bl{l}"]]
    parts += [params["w_out"], params["b_out"]]
    return np.concatenate(parts)


def init_params(seed: int = 0) -> np.ndarray:
    """He-style initial weights (the training's starting point)."""
    rng = np.random.default_rng(seed)
    p = {"Win": rng.normal(0, np.sqrt(2 / F0), (F0, H)), "bin": np.zeros(H)}
    for l in range(LAYERS):
        p[f"Wm{l}"] = rng.normal(0, np.sqrt(1 / H), (H, MSG))
        p[f"Wl{l}"] = rng.normal(0, np.sqrt(2 / (H + MSG)), (H + MSG, H))
        p[f"bl{l}"] = np.zeros(H)
    p["w_out"] = rng.normal(0, np.sqrt(1 / H), H)
    p["b_out"] = np.zeros(1)
    return pack(p).astype(np.float32).astype(np.float64)


def bf16(x):
    """Round float64 values to bfloat16 (via float32, round to nearest even)."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    rounded = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return rounded.astype(np.uint32).view(np.float32).astype(np.float64)


def graph_arrays(n, follower, leader, lam, mu):
    """Pattern and per-user quantities the network reads (from the
    definitions of A, c, d; self-loops and repeated edges dropped)."""
    import oracle.psi_oracle as po
    f, l, _, _ = po.clean_edges(n, follower, leader)
    lam = np.asarray(lam, dtype=np.float64)
    mu = np.asarray(mu, dtype=np.float64)
    den = np.zeros(n)
    np.add.at(den, f, lam[l] + mu[l])
    invden = np.where(den > 0, 1.0 / np.where(den > 0, den, 1.0), 0.0)
    # P[i, j] = 1 for j ∈ F(i): rows = leaders, columns = followers
    P = sp.csr_matrix((np.ones(f.size), (l, f)), shape=(n, n))
    n_followers = np.bincount(l, minlength=n)
    n_leaders = np.bincount(f, minlength=n)
    c = mu / (lam + mu)
    d = lam / (lam + mu)
    x0 = np.stack([np.log(lam), np.log(mu + 1e-12), c, d, np.log1p(n_followers),
                   np.log1p(n_leaders), np.log1p(den), np.log(lam + mu)], axis=1)
    return dict(P=P, invden=invden, lm=lam + mu, c=c, d=d, x0=x0, n=n)


def forward(theta, g, bf16_storage=False):
    """Returns (t_hat, cache)."""
    q = bf16 if bf16_storage else (lambda v: v)
    p = unpack(theta)
    P, invden = g["P"], g["invden"]
    cache = {}
    h = np.maximum(g["x0"] @ p["Win"] + p["bin"], 0.0)
    h = q(h)
    cache["h0"] = h
    for l in range(LAYERS):
        Wm = q(p[f"Wm{l}"])
        W = q(p[f"Wl{l}"])
        msg = q(invden[:, None] * (h @ Wm))
        m = q(np.log1p(np.maximum(g["lm"][:, None] * (P @ msg), 0.0)))
        x = np.concatenate([h, m], axis=1)
        h = q(np.maximum(x @ W + p[f"bl{l}"], 0.0))
        cache[f"msg{l}"] = msg
        cache[f"m{l}"] = m
        cache[f"x{l}"] = x
        cache[f"h{l + 1}"] = h
        cache[f"Wm{l}"] = Wm
        cache[f"Wl{l}"] = W
    out = h @ p["w_out"] + p["b_out"][0]
    cache["out"] = out
    t_hat = np.logaddexp(0.0, out)
    return t_hat, cache


def target(s, c):
    """t = log(s/c) on users with c > 0 (mask)."""
    s = np.asarray(s, dtype=np.float64)
    c = np.asarray(c, dtype=np.float64)
    mask = c > 0
    t = np.zeros_like(s)
    t[mask] = np.log(s[mask] / c[mask])
    return t, mask


def loss_and_grad(theta, g, t, mask, bf16_storage=False):
    """Mean squared error on t̂ and its gradient (FP64 backprop)."""
    p = unpack(theta)
    t_hat, cache = forward(theta, g, bf16_storage)
    n_valid = max(int(mask.sum()), 1)
    diff = np.where(mask, t_hat - t, 0.0)
    loss = float((diff ** 2).sum() / n_valid)
    out = cache["out"]
    d_out = 2.0 * diff / n_valid * (1.0 / (1.0 + np.exp(-out)))  # softplus' = sigmoid
    grads = {"w_out": cache[f"h{LAYERS}"].T @ d_out, "b_out": np.array([d_out.sum()])}
    dh = np.outer(d_out, p["w_out"])
    P, invden = g["P"], g["invden"]
    for l in reversed(range(LAYERS)):
        h_out = cache[f"h{l + 1}"]
        dz = dh * (h_out > 0)
        x = cache[f"x{l}"]
        grads[f"Wl{l}"] = x.T @ dz
        grads[f"bl{l}"] = dz.sum(axis=0)
        dx = dz @ cache[f"Wl{l}"].T
        dh_prev = dx[:, :H]
        # m = log1p(a) for a = lm ⊙ (P msg) > 0, else 0: dm/da = exp(−m) where m > 0
        m = cache[f"m{l}"]
        da = dx[:, H:] * np.where(m > 0, np.exp(-m), 0.0) * g["lm"][:, None]
        # msg = invden ⊙ (h Wm), a = lm ⊙ P msg  ⇒  d(h Wm) = invden ⊙ (Pᵀ (da))
        dmsg = invden[:, None] * (P.T @ da)
        h_prev = cache[f"h{l}"]
        grads[f"Wm{l}"] = h_prev.T @ dmsg
        dh = dh_prev + dmsg @ cache[f"Wm{l}"].T
    dz0 = dh * (cache["h0"] > 0)
    grads["Win"] = g["x0"].T @ dz0
    grads["bin"] = dz0.sum(axis=0)
    return loss, pack(grads)


def warm_start(theta, g, bf16_storage=False):
    """s0 = c ⊙ exp(t̂)."""
    t_hat, _ = forward(theta, g, bf16_storage)
    return g["c"] * np.exp(t_hat)


def adam(theta, grad, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba, 2015), bias-corrected, FP64."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mhat = m / (1 - b1 ** step)
    vhat = v / (1 - b2 ** step)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v
