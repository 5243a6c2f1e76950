"""Exact SimRank by FP64 power iteration, and the oracle's parameter formulas.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Eq. 1 defines s(u,u) = 1 and, for u != v,
    s(u,v) = c / (|I(u)||I(v)|) * sum_{u' in I(u), v' in I(v)} s(u',v').
With W[u, v] = 1/|I(v)| for u in I(v) (a zero column when I(v) is empty),
the off-diagonal part is (c * W^T S W)[u, v]; the diagonal is 1.  Since every
off-diagonal entry is >= 0 and c * (W^T S W)[u, u] <= c < 1, setting the
diagonal back to 1 is the same as the elementwise max(c * W^T S W, I), and the
iteration S_0 = I, S_{k+1} = max(c W^T S_k W, I) converges to S.

By Lemma 2, S_k(u, v) is also the probability that two sqrt(c)-walks from u
and v meet within k steps (induction on Eq. 1: both walks must survive a step,
probability sqrt(c) each, then move to uniform in-neighbours).  So a walk
estimator capped at L steps has expectation S_L, and 0 <= S - S_L <= c^(L+1).
"""
from __future__ import annotations

import math

import numpy as np


def transition(n: int, in_off: np.ndarray, in_src: np.ndarray) -> np.ndarray:
    """W[u, v] = (multiplicity of u in I(v)) / |I(v)|; columns of nodes without
    in-neighbours are zero."""
    W = np.zeros((n, n), np.float64)
    off = np.asarray(in_off, np.int64)
    src = np.asarray(in_src, np.int64)
    for v in range(n):
        row = src[off[v]:off[v + 1]]
        if row.size:
            np.add.at(W[:, v], row, 1.0 / row.size)
    return W


def simrank_iterates(n, in_off, in_src, c: float, k: int) -> np.ndarray:
    """S_k: k applications of S <- max(c W^T S W, I) starting from I."""
    W = transition(n, in_off, in_src)
    I = np.eye(n)
    S = I.copy()
    for _ in range(k):
        S = np.maximum(c * (W.T @ S @ W), I)
    return S


def exact_simrank(n, in_off, in_src, c: float, tol: float = 1e-15, max_iter: int = 10_000) -> np.ndarray:
    """The fixed point of Eq. 1 (to max change < tol, at least ceil(ln 1e-16 / ln c) sweeps)."""
    W = transition(n, in_off, in_src)
    I = np.eye(n)
    S = I.copy()
    min_iter = int(math.ceil(math.log(1e-16) / math.log(c)))
    for it in range(max_iter):
        S_new = np.maximum(c * (W.T @ S @ W), I)
        delta = float(np.max(np.abs(S_new - S)))
        S = S_new
        if it + 1 >= min_iter and delta < tol:
            break
    return S


# ---------------------------------------------------------------------------
# Parameters (Hoeffding sample size, Section 3 and Appendix B.4; truncation)
# ---------------------------------------------------------------------------

def continue_probability(c: float) -> float:
    """The walk continues iff a 32-bit word is below T = floor(sqrt(c) 2^32)."""
    T = math.floor(math.sqrt(c) * 4294967296.0)
    T = min(T, 4294967295)
    return T / 4294967296.0


def truncation_bias(c: float, L: int) -> float:
    """S - S_L <= c^(L+1): both walks must survive L+1 steps to meet after step L."""
    return c ** (L + 1)


def hoeffding_R(eps: float, delta: float, c: float, L: int, n: int | None = None) -> int:
    """Pairs per node so that Pr[|s_hat - S_L| >= eps - c^(L+1)] <= delta for one
    node (Hoeffding: 2 exp(-2 R lambda^2) <= delta); with n given, delta is split
    over all n estimates by the union bound, as in the warm-up's N = ln(2n^2)/(2 eps^2)."""
    lam = eps - truncation_bias(c, L)
    if lam <= 0:
        raise ValueError("eps must exceed the truncation bias c^(L+1)")
    numer = math.log(2.0 / delta) if n is None else math.log(2.0 * n / delta)
    return int(math.ceil(numer / (2.0 * lam * lam)))


# ---------------------------------------------------------------------------
# First-meeting probabilities and the length-stratified estimator's mean
# ---------------------------------------------------------------------------

def first_meet_probs(n, in_off, in_src, s: int, T: int) -> np.ndarray:
    """F[t, u] = probability that two uniform walks on the reversed graph (no
    stopping), from s and from u, first occupy the same node at step t,
    t = 0..T.  Pair dynamics: the joint law Q of the two positions moves by
    Q <- W Q W^T (column v of W is the law of the next position from v);
    after each step the mass on the diagonal is the first-meeting mass and is
    removed.  A walk at a node without in-neighbours loses its mass."""
    W = transition(n, in_off, in_src)
    F = np.zeros((T + 1, n), np.float64)
    F[0, s] = 1.0
    Q = np.zeros((n, n, n), np.float64)       # Q[u] = joint law for the pair (s, u)
    for u in range(n):
        if u != s:
            Q[u, s, u] = 1.0
    idx = np.arange(n)
    for t in range(1, T + 1):
        Q = np.einsum("ax,uxy,by->uab", W, Q, W, optimize=True)
        F[t] = Q[:, idx, idx].sum(axis=1)
        Q[:, idx, idx] = 0.0
    return F


def stratified_expectation(n, in_off, in_src, c: float, s: int, phi: int) -> np.ndarray:
    """Mean of the length-stratified estimate normalised by its N pairs, for
    every u, on a graph without dead ends: walk j of s and of u have lengths
    l1, l2 in 0..phi drawn with weights proportional to Zhat_l (the shuffle),
    and a meeting pair is weighted by the ratio of the geometric law
    p_l = sqrt(c)^l (1 - sqrt(c)) to that sampling law, so the mean is
        sum_{l1, l2 <= phi} p_l1 p_l2 Pr[meet within min(l1, l2) steps]
      = sum_{t=1..phi} F_t (sqrt(c)^t - sqrt(c)^(phi+1))^2,
    since both lengths lie in [t, phi] with probability
    (sqrt(c)^t - sqrt(c)^(phi+1))^2.  Algorithm 2's own normalisation by z
    multiplies this by z / N.  The value at u = s is 1."""
    F = first_meet_probs(n, in_off, in_src, s, phi)
    r = math.sqrt(c)
    tail = r ** (phi + 1)
    w = np.array([0.0] + [(r ** t - tail) ** 2 for t in range(1, phi + 1)])
    E = (w[:, None] * F).sum(axis=0)
    E[s] = 1.0
    return E
