"""Exact law of Algorithm 1 at one asset (d = 1), Gaussian returns, fresh samples every step.

With d = 1 the sample mean Rbar ~ N(mu, sigma^2/N) and V = (N-1) s^2 / sigma^2 ~ chi2_{N-1} are
independent (Cochran). The linear subproblem over W = [0, 1] picks e_1 exactly when the gradient
2 lambda s^2 w - Rbar is negative, so given the iterate w

    P(pick e_1 | w) = E_V[ Phi_bar( (2 lambda w sigma^2 V/(N-1) - mu) sqrt(N) / sigma ) ].

By the step rule 2/(t+2) the iterate after t >= 1 steps is w_t = 2 S_t / (t (t+1)) where S_t is the
sum of (s+1) over the steps s < t that picked e_1, so a dynamic program over the integer S_t gives
the exact law of w_T and of f(w_T) = lambda sigma^2 w^2 - mu w (Eq. (3)).

Independent of the oracle: plain numpy/scipy on the formulas above.
"""
from __future__ import annotations

import itertools
import math

import numpy as np
from scipy import special, stats


def pick_probability(w, mu, sigma, N, lam, nodes=80):
    """P(e_1 chosen | iterate w) for an array of w, by generalized Gauss-Laguerre over V."""
    w = np.atleast_1d(np.asarray(w, dtype=np.float64))
    k = N - 1
    alpha = k / 2.0 - 1.0
    x, wt = special.roots_genlaguerre(nodes, alpha)
    wt = wt / math.gamma(alpha + 1.0)          # chi2_k density with V = 2x
    V = 2.0 * x
    arg = (2.0 * lam * w[:, None] * sigma ** 2 * V[None, :] / (N - 1) - mu) * math.sqrt(N) / sigma
    return (stats.norm.sf(arg) * wt[None, :]).sum(axis=1)


def wsum_law(T, mu, sigma, N, lam, w0=0.0):
    """Exact probability vector over S_T in [0, T(T+1)/2]. N is the sample size of every step, or
    a sequence of T sizes (a schedule with fresh samples every step)."""
    prob = np.zeros(1)
    prob[0] = 1.0
    for t in range(T):
        S = np.arange(prob.shape[0])
        w = np.full(prob.shape[0], w0) if t == 0 else 2.0 * S / (t * (t + 1.0))
        Nt = int(N[t]) if hasattr(N, "__len__") else N
        p1 = pick_probability(w, mu, sigma, Nt, lam)
        new = np.zeros(prob.shape[0] + t + 1)
        new[: prob.shape[0]] += prob * (1.0 - p1)
        new[t + 1: t + 1 + prob.shape[0]] += prob * p1
        prob = new
    return prob


def wsum_law_bruteforce(T, mu, sigma, N, lam, w0=0.0):
    """The same law by enumerating all 2^T decision sequences (T <= 10)."""
    size = T * (T + 1) // 2 + 1
    prob = np.zeros(size)
    for seq in itertools.product((0, 1), repeat=T):
        p = 1.0
        w = w0
        S = 0
        for t, a in enumerate(seq):
            p1 = float(pick_probability(w, mu, sigma, N, lam)[0])
            p *= p1 if a else (1.0 - p1)
            w = w + 2.0 / (t + 2.0) * (a - w)
            S += (t + 1) * a
        prob[S] += p
    return prob


def outcome_moments(T, mu, sigma, N, lam, w0=0.0):
    """(E f(w_T), Var f(w_T)) exactly."""
    prob = wsum_law(T, mu, sigma, N, lam, w0)
    S = np.arange(prob.shape[0])
    w = 2.0 * S / (T * (T + 1.0))
    f = lam * sigma ** 2 * w ** 2 - mu * w
    m = float((prob * f).sum())
    v = float((prob * (f - m) ** 2).sum())
    return m, v
