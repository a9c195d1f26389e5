"""Seeded synthetic follower graphs and activity vectors.

Directed Chung–Lu recipe (stand-in for the paper's social graphs, whose data
is not shipped): every edge picks its *leader* endpoint with probability
proportional to a power-law weight and its *follower* endpoint uniformly, so
the number of followers of a user (the row length of the pull operator) has a
power-law tail while the number of leaders of a user is about Poisson(mean
degree).

* weight of the user of rank r (r = 1..N): w_r = (N / r)^(1/(γ-1)), scaled by a
  factor s and capped at d_max so that Σ min(s·w_r, d_max) = M_target;
* edge e: leader = perm[rank], rank drawn by inverse CDF of the capped weights
  from uniform e of stream 0; follower = floor(N·u) with u uniform e of
  stream 1; ``perm`` is a random permutation (stream 4) so hubs are not
  clustered at low ids;
* raw edges may contain self-loops and duplicates: the operator build drops
  them and reports how many;
* activity: λ_n = exp(σ·Z), μ_n = exp(σ·Z') with Z, Z' standard normal
  (streams 2 and 3; scenario k uses streams 2+2k and 3+2k), or U(0,1), or the
  homogeneous pair λ = 0.15, μ = 0.85.

Edge (follower[k], leader[k]) means follower[k] follows leader[k].  The module
holds no part of the ψ-score arithmetic; both the oracle and the GPU path are
fed from it.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import rng

STREAM_LEADER = 0
STREAM_FOLLOWER = 1
STREAM_LAMBDA = 2
STREAM_MU = 3
STREAM_PERM = 4
STREAM_SIZES = 5

_CHUNK = 1 << 24


@dataclass
class Graph:
    n: int
    follower: np.ndarray  # int32 [M_raw]
    leader: np.ndarray  # int32 [M_raw]
    lam: np.ndarray  # float64 [N]
    mu: np.ndarray  # float64 [N]
    node_offsets: np.ndarray | None = None  # int64 [G+1] for multi-graph inputs
    meta: dict = field(default_factory=dict)

    @property
    def m_raw(self) -> int:
        return int(self.follower.shape[0])


def capped_weights(n: int, m_target: float, gamma: float, d_max: float) -> np.ndarray:
    r = np.arange(1, n + 1, dtype=np.float64)
    w = (n / r) ** (1.0 / (gamma - 1.0))
    scale = m_target / w.sum()
    for _ in range(100):
        capped = scale * w >= d_max
        free = w[~capped].sum()
        if free <= 0:
            break
        new_scale = (m_target - d_max * capped.sum()) / free
        if abs(new_scale - scale) <= 1e-15 * scale:
            scale = new_scale
            break
        scale = new_scale
    return np.minimum(scale * w, d_max)


def permutation(n: int, seed: int) -> np.ndarray:
    keys = rng.words(seed, STREAM_PERM, 0, n)
    return np.argsort(keys, kind="stable").astype(np.int32)


def chung_lu_edges(n: int, m_target: int, gamma: float, seed: int,
                   d_max: float | None = None) -> tuple[np.ndarray, np.ndarray]:
    if n < 2:
        raise ValueError("need at least two users")
    if d_max is None:
        d_max = n - 1
    w = capped_weights(n, float(m_target), gamma, float(d_max))
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    perm = permutation(n, seed)
    follower = np.empty(m_target, dtype=np.int32)
    leader = np.empty(m_target, dtype=np.int32)
    for start in range(0, m_target, _CHUNK):
        cnt = min(_CHUNK, m_target - start)
        u0 = rng.uniform01(seed, STREAM_LEADER, cnt, start)
        rank = np.searchsorted(cdf, u0, side="right")
        np.minimum(rank, n - 1, out=rank)
        leader[start:start + cnt] = perm[rank]
        u1 = rng.uniform01(seed, STREAM_FOLLOWER, cnt, start)
        f = (u1 * n).astype(np.int64)
        np.minimum(f, n - 1, out=f)
        follower[start:start + cnt] = f
    return follower, leader


def chung_lu_plan(n: int, m_target: int, gamma: float, seed: int,
                  d_max: float | None = None) -> tuple[np.ndarray, np.ndarray]:
    """The N-sized host part of a Chung–Lu draw: the leader CDF and the
    rank-to-user permutation (NumPy; independent of the device)."""
    if n < 2:
        raise ValueError("need at least two users")
    if d_max is None:
        d_max = n - 1
    w = capped_weights(n, float(m_target), gamma, float(d_max))
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    return cdf, permutation(n, seed)


def chung_lu_edges_torch(n: int, m_target: int, gamma: float, seed: int,
                         d_max: float | None = None, device="cpu", plan=None):
    """chung_lu_edges drawn with torch on ``device``: the same edges, bit for
    bit (the N-sized weights and permutation are still computed by NumPy, or
    passed in as ``plan`` from chung_lu_plan)."""
    import torch
    if n < 2:
        raise ValueError("need at least two users")
    cdf, perm = plan if plan is not None else chung_lu_plan(n, m_target, gamma, seed, d_max)
    cdf_t = torch.from_numpy(cdf).to(device)
    perm_t = torch.from_numpy(perm).to(device)
    follower = torch.empty(m_target, dtype=torch.int32, device=device)
    leader = torch.empty(m_target, dtype=torch.int32, device=device)
    chunk = 1 << 26
    for start in range(0, m_target, chunk):
        cnt = min(chunk, m_target - start)
        u0 = rng.uniform01_torch(seed, STREAM_LEADER, cnt, start, device)
        rank = torch.searchsorted(cdf_t, u0, right=True).clamp_(max=n - 1)
        leader[start:start + cnt] = perm_t[rank]
        del u0, rank
        u1 = rng.uniform01_torch(seed, STREAM_FOLLOWER, cnt, start, device)
        follower[start:start + cnt] = (u1 * n).to(torch.int64).clamp_(max=n - 1).to(torch.int32)
        del u1
    return follower, leader


def activity(n: int, seed: int, kind: str = "lognormal", sigma: float = 1.0,
             scenario: int = 0) -> tuple[np.ndarray, np.ndarray]:
    if kind == "lognormal":
        lam = np.exp(sigma * rng.standard_normal(seed, STREAM_LAMBDA + 2 * scenario, n))
        mu = np.exp(sigma * rng.standard_normal(seed, STREAM_MU + 2 * scenario, n))
    elif kind == "uniform":
        lam = rng.uniform01(seed, STREAM_LAMBDA + 2 * scenario, n)
        mu = rng.uniform01(seed, STREAM_MU + 2 * scenario, n)
    elif kind == "homogeneous":
        lam = np.full(n, 0.15)
        mu = np.full(n, 0.85)
    else:
        raise ValueError(f"unknown activity kind {kind!r}")
    return lam, mu


def chung_lu(n: int, mean_degree: float, gamma: float, seed: int,
             sigma: float = 1.0, d_max: float | None = None,
             activity_kind: str = "lognormal") -> Graph:
    m_target = int(round(n * mean_degree))
    follower, leader = chung_lu_edges(n, m_target, gamma, seed, d_max)
    lam, mu = activity(n, seed, activity_kind, sigma)
    return Graph(n, follower, leader, lam, mu,
                 meta=dict(kind="chung_lu", n=n, m_target=m_target, gamma=gamma,
                           seed=seed, sigma=sigma, d_max=d_max if d_max else n - 1,
                           activity=activity_kind))


def multi_graph(n_graphs: int, n_lo: int, n_hi: int, mean_degree: float, gamma: float,
                seed: int, sigma: float = 1.0, device=None) -> Graph:
    """Independent Chung–Lu graphs stacked block-diagonally.

    Graph g has N_g uniform in {n_lo..n_hi} (stream 5 of ``seed``) and is drawn
    with seed 1000*seed + g; its users are numbered from node_offsets[g].
    With ``device`` the edges are drawn there by the torch twin (same values)
    and returned as torch int32 tensors.
    """
    u = rng.uniform01(seed, STREAM_SIZES, n_graphs)
    sizes = n_lo + np.minimum((u * (n_hi - n_lo + 1)).astype(np.int64), n_hi - n_lo)
    offsets = np.zeros(n_graphs + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(sizes)
    fs, ls, lams, mus = [], [], [], []
    for g in range(n_graphs):
        n_g, seed_g = int(sizes[g]), 1000 * seed + g
        if device is None:
            sub = chung_lu(n_g, mean_degree, gamma, seed_g, sigma)
            f, l, lam, mu = sub.follower, sub.leader, sub.lam, sub.mu
        else:
            f, l = chung_lu_edges_torch(n_g, int(round(n_g * mean_degree)), gamma, seed_g,
                                        device=device)
            lam, mu = activity(n_g, seed_g, "lognormal", sigma)
        fs.append(f + int(offsets[g]))
        ls.append(l + int(offsets[g]))
        lams.append(lam)
        mus.append(mu)
    if device is None:
        follower, leader = np.concatenate(fs), np.concatenate(ls)
    else:
        import torch
        follower, leader = torch.cat(fs), torch.cat(ls)
    return Graph(int(offsets[-1]), follower, leader,
                 np.concatenate(lams), np.concatenate(mus), node_offsets=offsets,
                 meta=dict(kind="multi_graph", n_graphs=n_graphs, n_lo=n_lo, n_hi=n_hi,
                           mean_degree=mean_degree, gamma=gamma, seed=seed, sigma=sigma))


def random_small(n: int, p: float, seed: int, dangling: bool = True,
                 activity_kind: str = "lognormal", sigma: float = 1.0,
                 extra_self_loops: int = 0, extra_duplicates: int = 0) -> Graph:
    """Erdős–Rényi-style directed graph for brute-force sized cases.

    Every ordered pair (i, j), i != j, is an edge with probability p (stream
    0).  With ``dangling=False`` every user without a leader gets one (the next
    user, cyclically), so no row of the operator is empty.  Self-loops and
    duplicate edges can be appended to exercise the build's clean-up.
    """
    u = rng.uniform01(seed, STREAM_LEADER, n * n).reshape(n, n)
    adj = u < p
    np.fill_diagonal(adj, False)
    if not dangling:
        for i in range(n):
            if not adj[i].any():
                adj[i, (i + 1) % n] = True
    f, l = np.nonzero(adj)
    f = f.astype(np.int32)
    l = l.astype(np.int32)
    if extra_duplicates and f.size:
        pick = (rng.uniform01(seed, 6, extra_duplicates) * f.size).astype(np.int64)
        f = np.concatenate([f, f[pick]])
        l = np.concatenate([l, l[pick]])
    if extra_self_loops:
        s = (rng.uniform01(seed, 7, extra_self_loops) * n).astype(np.int32)
        f = np.concatenate([f, s])
        l = np.concatenate([l, s])
    # shuffle edge order so the build cannot rely on sorted input
    order = np.argsort(rng.words(seed, 8, 0, f.size), kind="stable")
    lam, mu = activity(n, seed, activity_kind, sigma)
    return Graph(n, f[order], l[order], lam, mu,
                 meta=dict(kind="random_small", n=n, p=p, seed=seed))


def star(n: int, seed: int, sigma: float = 1.0) -> Graph:
    """User 0 is the hub: every other user follows only the hub."""
    f = np.arange(1, n, dtype=np.int32)
    l = np.zeros(n - 1, dtype=np.int32)
    lam, mu = activity(n, seed, "lognormal", sigma)
    return Graph(n, f, l, lam, mu, meta=dict(kind="star", n=n, seed=seed))


def cycle(n: int) -> Graph:
    """Directed cycle: user i follows user i+1 (mod n); homogeneous activity."""
    f = np.arange(n, dtype=np.int32)
    l = ((np.arange(n) + 1) % n).astype(np.int32)
    lam, mu = activity(n, 0, "homogeneous")
    return Graph(n, f, l, lam, mu, meta=dict(kind="cycle", n=n))


def complete(n: int) -> Graph:
    """Every user follows every other user; homogeneous activity."""
    i, j = np.nonzero(~np.eye(n, dtype=bool))
    lam, mu = activity(n, 0, "homogeneous")
    return Graph(n, i.astype(np.int32), j.astype(np.int32), lam, mu,
                 meta=dict(kind="complete", n=n))


# Workloads: sizes, exponents and activity spreads of the measured cases.
WORKLOADS = {
    "cl_1k": dict(n=1_000, mean_degree=10, gamma=2.2, seed=1, sigma=1.0, tol=1e-10),
    "cl_1m": dict(n=1_000_000, mean_degree=20, gamma=2.2, seed=2, sigma=1.5, tol=1e-8),
    "cl_40m": dict(n=40_000_000, mean_degree=35, gamma=2.1, seed=3, sigma=2.0,
                   d_max=3_000_000, tol=1e-8),
    "cl_4m_k64": dict(n=4_000_000, mean_degree=20, gamma=2.2, seed=4, sigma=1.5,
                      scenarios=64, tol=1e-8),
    "cl_10m": dict(n=10_000_000, mean_degree=20, gamma=2.2, seed=5, sigma=1.5, tol=1e-8),
    "graphs256": dict(kind="multi", n_graphs=256, n_lo=1_000, n_hi=100_000, mean_degree=15,
                      gamma=2.2, seed=4, sigma=1.5, tol=1e-8),
}


def workload(name: str, device=None) -> Graph:
    """A named workload.  With ``device`` (a torch device) the edges are drawn
    there by the torch twin and returned as torch int32 tensors; λ, μ stay
    NumPy arrays.  Both routes give the same values."""
    w = dict(WORKLOADS[name])
    w.pop("tol", None)
    w.pop("scenarios", None)
    if w.pop("kind", None) == "multi":
        return multi_graph(**w, device=device)
    if device is None:
        return chung_lu(**w)
    n, seed, sigma = w["n"], w["seed"], w.get("sigma", 1.0)
    m_target = int(round(n * w["mean_degree"]))
    follower, leader = chung_lu_edges_torch(n, m_target, w["gamma"], seed, w.get("d_max"), device)
    lam, mu = activity(n, seed, "lognormal", sigma)
    return Graph(n, follower, leader, lam, mu,
                 meta=dict(kind="chung_lu", n=n, m_target=m_target, gamma=w["gamma"], seed=seed,
                           sigma=sigma, d_max=w.get("d_max") or n - 1, activity="lognormal"))
