"""Plain FP64 CPU oracle for the ψ-score (Arhachoui et al., ASONAM 2022).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link this module: only the test-suite, the package's smoke check and the
benchmark's CPU-baseline leg use it.  It shares no code with the HIP library.

Notation (Sec. II): (i, j) ∈ E means user i follows user j; L(j) is the set of
leaders of j; λ_n, μ_n are the posting and re-posting rates of user n.

Functions and the passages they follow:

* ``clean_edges``       — the graph is unweighted with no self-loops (Sec. II):
                          self-loops and repeated edges are dropped.
* ``operator``          — the matrices A, B and vectors c, d of the matrix form
                          (Sec. II, the definitions under eqs. (newsfeed)/(wall);
                          c and d are the diagonals of C and D, Sec. III-A).
* ``psi_by_definition`` — ψ_i = (1/N) Σ_n q_i^(n) (eq. psiscore) with p_i from
                          the newsfeed balance equations (4)–(5) and q_i from the
                          wall balance equations (2)–(3): N separate N-size
                          linear solves (LAPACK via numpy), one per origin.
* ``power_nf``          — Algorithm 1 (Power-NF) for one origin.
* ``psi_closed_form``   — eq. (ultimsol) with the series summed exactly: one
                          solve of (I − Aᵀ) s = c, then ψ = (Bᵀ s + d) / N.
* ``power_psi``         — Algorithm 2 (Power-ψ), FP64: the recursion of
                          eq. (power_psi) from s_0 = c, stopped by eq. (condition).
* ``pagerank_power``    — the PageRank power method, eq. (pagerank_power).
* ``fixed_point_residual``, ``b_norm``, ``kappa`` — the L1 fixed-point residual
                          of eq. (power_psi) and the norms used by the bound of
                          eq. (psi_diff).
* ``sampled_rows``      — for a few users i only, (Aᵀs)_i and (Bᵀs)_i from the
                          definitions of A and B (Sec. II) over the raw edge
                          list, without building the whole operator: the
                          residual of eq. (power_psi) and the last line of
                          Algorithm 2 at those users, for graphs too large for
                          the full oracle.

Readings where the paper is silent:

* users with no leaders have an empty newsfeed: their rows of A and B are zero
  (the sums in the definitions of A and B are empty) and p^(j) = 0;
* ‖·‖ is the L1 norm (the paper's stated implementation choice, Sec. III-C);
  ‖B‖ is the norm induced by L1 on row vectors, i.e. the largest row sum;
* the default stopping test is ‖s_t − s_{t−1}‖₁ ≤ ε (eq. condition, the
  "s-tolerance" of Sec. V); ``tol_mode="bnorm"`` multiplies the gap by ‖B‖ as
  Algorithm 2 prints it, ``"rel_l1"`` divides it by ‖s_t‖₁;
* ψ is formed from the final s (the last line of Algorithm 2).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

__all__ = [
    "clean_edges", "operator", "psi_by_definition", "power_nf", "psi_closed_form",
    "power_psi", "pagerank_power", "transition_matrix", "fixed_point_residual",
    "b_norm", "kappa", "rel_l1", "rel_l2", "max_rel", "sampled_rows",
]


def clean_edges(n, follower, leader):
    """Drop self-loops and repeated edges (Sec. II: unweighted, no self-loops).

    Returns (follower, leader, n_self_loops, n_duplicates) with the surviving
    edges sorted by (follower, leader).
    """
    f = np.asarray(follower, dtype=np.int64)
    l = np.asarray(leader, dtype=np.int64)
    if f.shape != l.shape:
        raise ValueError("follower and leader differ in length")
    if f.size and (f.min() < 0 or l.min() < 0 or f.max() >= n or l.max() >= n):
        raise ValueError("edge endpoint out of range")
    loops = f == l
    f, l = f[~loops], l[~loops]
    key = np.unique(f * n + l)
    n_dup = f.size - key.size
    return key // n, key % n, int(loops.sum()), int(n_dup)


def operator(n, follower, leader, lam, mu):
    """A, B (scipy CSR, row j = follower, column i = leader), c, d.

    a_ji = μ_i / Σ_{ℓ∈L(j)}(λ_ℓ+μ_ℓ) and b_ji = λ_i / Σ_{ℓ∈L(j)}(λ_ℓ+μ_ℓ) when
    i ∈ L(j), else 0;  c_i = μ_i/(λ_i+μ_i), d_i = λ_i/(λ_i+μ_i).
    """
    lam = np.asarray(lam, dtype=np.float64)
    mu = np.asarray(mu, dtype=np.float64)
    f, l, _, _ = clean_edges(n, follower, leader)
    den = np.zeros(n)
    np.add.at(den, f, lam[l] + mu[l])
    a_val = mu[l] / den[f]
    b_val = lam[l] / den[f]
    A = sp.csr_matrix((a_val, (f, l)), shape=(n, n))
    B = sp.csr_matrix((b_val, (f, l)), shape=(n, n))
    c = mu / (lam + mu)
    d = lam / (lam + mu)
    return A, B, c, d


def psi_by_definition(n, follower, leader, lam, mu):
    """ψ from its definition: N separate N-size solves (eqs. (2)–(5), psiscore).

    For every origin i the newsfeed shares p_i solve, for every user j,
        Σ_{k∈L(j)}(λ_k+μ_k) p_i^(j) − Σ_{k∈L(j)} μ_k p_i^(k) = λ_i 1{i∈L(j)}
    (eqs. (4)–(5); a user with no leaders has p_i^(j) = 0), then the wall
    shares are
        (λ_j+μ_j) q_i^(j) = μ_j p_i^(j)            for j ≠ i   (eq. 2)
        (λ_i+μ_i) q_i^(i) = λ_i + μ_i p_i^(i)                   (eq. 3)
    and ψ_i = (1/N) Σ_n q_i^(n).  Dense; meant for N of a few hundred.
    Returns (psi, P, Q) with p_i and q_i as column i of P and Q.
    """
    lam = np.asarray(lam, dtype=np.float64)
    mu = np.asarray(mu, dtype=np.float64)
    f, l, _, _ = clean_edges(n, follower, leader)
    leads = np.zeros((n, n), dtype=bool)  # leads[j, k]: k ∈ L(j)
    leads[f, l] = True
    M = np.zeros((n, n))
    for j in range(n):
        ks = np.nonzero(leads[j])[0]
        if ks.size == 0:
            M[j, j] = 1.0  # empty newsfeed: p^(j) = 0
            continue
        M[j, j] += np.sum(lam[ks] + mu[ks])
        M[j, ks] -= mu[ks]
    P = np.zeros((n, n))
    Q = np.zeros((n, n))
    for i in range(n):
        rhs = np.where(leads[:, i], lam[i], 0.0)
        p = np.linalg.solve(M, rhs)
        q = mu * p / (lam + mu)
        q[i] = (lam[i] + mu[i] * p[i]) / (lam[i] + mu[i])
        P[:, i] = p
        Q[:, i] = q
    psi = Q.sum(axis=0) / n
    return psi, P, Q


def _finite_gap(gap, what):
    """A NaN or infinite gap means the iteration has left the reals: raise
    instead of letting a NaN comparison end the loop as if it had converged."""
    if not np.isfinite(gap):
        raise FloatingPointError(f"{what}: the step size is {gap} (not finite)")
    return gap


def power_nf(A, b_i, tol, max_iter=100_000):
    """Algorithm 1 (Power-NF) for one origin i: the fixed point of
    p = A p + b_i (eq. fixpt_algo) by repeated substitution from p = b_i,
    ended by the p-tolerance ‖p_t − p_{t−1}‖₁ ≤ ε (Sec. V)."""
    p = np.array(b_i, dtype=np.float64)
    t = 0
    gap = 1.0
    while gap > tol:
        if t >= max_iter:
            raise RuntimeError("Power-NF did not converge")
        p_next = A @ p + b_i
        gap = _finite_gap(np.abs(p_next - p).sum(), "Power-NF")
        p = p_next
        t += 1
    return p, t


def psi_closed_form(A, B, c, d):
    """Eq. (ultimsol) with Σ_t cᵀAᵗ = cᵀ(I−A)⁻¹: solve (I − Aᵀ) s = c."""
    n = A.shape[0]
    I = sp.identity(n, format="csc")
    s = sp.linalg.spsolve((I - A.T).tocsc(), c)
    psi = (B.T @ s + d) / n
    return psi, s


def b_norm(B):
    """‖B‖ induced by L1 on row vectors: the largest row sum."""
    rs = np.asarray(abs(B).sum(axis=1)).ravel()
    return float(rs.max()) if rs.size else 0.0


def kappa(A):
    """Largest row sum of A: the contraction factor of s ↦ Aᵀs + c in L1."""
    rs = np.asarray(abs(A).sum(axis=1)).ravel()
    return float(rs.max()) if rs.size else 0.0


def power_psi(A, B, c, d, tol, tol_mode="abs_l1", max_iter=100_000, s0=None,
              record=False, steps=None):
    """Algorithm 2 (Power-ψ) in FP64.

    The iterate is the partial sum of the series of eq. (ultimsol): the
    recursion of eq. (power_psi), s_t = Aᵀ s_{t−1} + c, from s_0 = c (or a
    given start).  It stops at the first t whose step size ε_t = ‖s_t −
    s_{t−1}‖₁ (eq. eps_t) passes the test of eq. (condition); ``tol_mode``
    "bnorm" multiplies ε_t by ‖B‖ before the test, as Algorithm 2 does, and
    "rel_l1" divides it by ‖s_t‖₁.  Algorithm 2 starts from a gap of 1, so
    ε ≥ 1 takes no step.  ψ = (Bᵀ s + d) / N is formed from the final s.

    Returns a dict with psi, s, iterations t, the final gap and (optionally)
    every gap.  ``steps`` runs exactly that many iterations whatever the gap
    (used to inspect ψ_t at a fixed t).  A step size that is not finite
    raises FloatingPointError.
    """
    if not tol > 0:
        raise ValueError("tolerance must be positive")
    if tol_mode not in ("abs_l1", "bnorm", "rel_l1"):
        raise ValueError(f"unknown tol_mode {tol_mode!r}")
    n = A.shape[0]
    AT = A.T.tocsr()
    BT = B.T.tocsr()
    bnorm = b_norm(B)

    def scaled(step_l1, s_new):
        if tol_mode == "bnorm":
            return step_l1 * bnorm
        if tol_mode == "rel_l1":
            return step_l1 / np.abs(s_new).sum()
        return step_l1

    s = np.array(c if s0 is None else s0, dtype=np.float64)
    gaps = []
    gap = 1.0
    t = 0
    while (t < steps) if steps is not None else (gap > tol):
        if t >= max_iter:
            raise RuntimeError("Power-psi did not converge")
        s_next = AT @ s + c
        gap = _finite_gap(scaled(np.abs(s_next - s).sum(), s_next), "Power-psi")
        s = s_next
        t += 1
        if record:
            gaps.append(gap)
    psi = (BT @ s + d) / n
    return dict(psi=psi, s=s, iterations=t, gap=gap, gaps=gaps, bnorm=bnorm)


def transition_matrix(n, follower, leader):
    """W = D_out⁻¹ L with L_ji = 1 iff j follows i (Sec. III-D); rows of users
    who follow nobody are zero."""
    f, l, _, _ = clean_edges(n, follower, leader)
    deg = np.bincount(f, minlength=n).astype(np.float64)
    return sp.csr_matrix((1.0 / deg[f], (f, l)), shape=(n, n))


def pagerank_power(W, alpha, tol, max_iter=100_000):
    """Eq. (pagerank_power): π_t = α π_{t−1} W + (1−α)/N 1, from π_0 = 1/N,
    stopped on the π-tolerance ‖π_t − π_{t−1}‖₁ ≤ ε (Sec. V)."""
    n = W.shape[0]
    WT = W.T.tocsr()
    pi = np.full(n, 1.0 / n)
    t = 0
    gap = 1.0
    while gap > tol:
        if t >= max_iter:
            raise RuntimeError("PageRank power method did not converge")
        pi_next = alpha * (WT @ pi) + (1.0 - alpha) / n
        gap = _finite_gap(np.abs(pi_next - pi).sum(), "PageRank power method")
        pi = pi_next
        t += 1
    return pi, t


def fixed_point_residual(A, c, s):
    """‖Aᵀs + c − s‖₁: how far s is from the fixed point of eq. (power_psi)."""
    return float(np.abs(A.T @ s + c - s).sum())


def rel_l1(ref, x):
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.abs(np.asarray(x) - ref).sum() / np.abs(ref).sum())


def max_rel(ref, x):
    """Largest element-wise relative error max_i |x_i − ref_i| / |ref_i| (ψ_i ≥
    d_i/N > 0 and s_i ≥ c_i > 0, so the ratio is defined for both)."""
    ref = np.asarray(ref, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    if np.any(ref == 0):
        raise ValueError("max_rel needs a reference without zeros")
    return float(np.max(np.abs(x - ref) / np.abs(ref))) if ref.size else 0.0


def rel_l2(ref, x):
    """The paper's error measure, eq. (error)."""
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.linalg.norm(np.asarray(x) - ref) / np.linalg.norm(ref))


def sampled_rows(n, follower, leader, lam, mu, s, rows, chunk=1 << 26):
    """Residual of eq. (power_psi) and ψ (last line of Algorithm 2) at `rows`.

    For each sampled user i: F(i) = the distinct followers j ≠ i of i, and for
    each such j, den_j = Σ over the distinct leaders ℓ ≠ j of j of (λ_ℓ + μ_ℓ)
    (the definitions of A and B, Sec. II).  With y_i = Σ_{j∈F(i)} s_j / den_j:
        residual_i = c_i + μ_i y_i − s_i,   psi_i = (d_i + λ_i y_i) / N.
    The edge arrays are read in chunks, twice; memory stays proportional to
    the sampled rows and their followers.  Returns (residual, psi) in the
    order of `rows`.
    """
    rows = np.asarray(rows, dtype=np.int64)
    lam = np.asarray(lam, dtype=np.float64)
    mu = np.asarray(mu, dtype=np.float64)
    s = np.asarray(s, dtype=np.float64)
    m = len(follower)
    want = np.zeros(n, dtype=bool)
    want[rows] = True
    pairs = []  # (leader i, follower j) with i sampled
    for a in range(0, m, chunk):
        f = np.asarray(follower[a:a + chunk], dtype=np.int64)
        l = np.asarray(leader[a:a + chunk], dtype=np.int64)
        sel = want[l] & (f != l)
        pairs.append(l[sel] * n + f[sel])
    key = np.unique(np.concatenate(pairs))
    row_of, fol = key // n, key % n
    need = np.zeros(n, dtype=bool)
    need[fol] = True
    lead = []  # (follower j, leader ℓ) for the followers j of sampled rows
    for a in range(0, m, chunk):
        f = np.asarray(follower[a:a + chunk], dtype=np.int64)
        l = np.asarray(leader[a:a + chunk], dtype=np.int64)
        sel = need[f] & (f != l)
        lead.append(f[sel] * n + l[sel])
    key2 = np.unique(np.concatenate(lead))
    j2, l2 = key2 // n, key2 % n
    den = np.zeros(n)
    np.add.at(den, j2, lam[l2] + mu[l2])
    y = np.zeros(n)
    np.add.at(y, row_of, s[fol] / den[fol])
    c = mu / (lam + mu)
    d = lam / (lam + mu)
    yr = y[rows]
    residual = c[rows] + mu[rows] * yr - s[rows]
    psi = (d[rows] + lam[rows] * yr) / n
    return residual, psi
