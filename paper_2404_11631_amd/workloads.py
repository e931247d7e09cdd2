"""Seeded synthetic inputs for the batched Frank-Wolfe simulation.

This module draws instance parameters (mean returns mu, standard deviations sigma, dense
Cholesky factors L, the uneven batch of instances) and names the workload shapes. It holds none
of the method's arithmetic, so both the HIP path and the CPU oracle can take their inputs from
it. The path noise itself is not drawn here: each side generates it from the counter-based
Philox4x32-10 stream.

Parameter laws:
  * "unit" regime: mu_j ~ U(0,1) and sigma_j ~ U(0,1), Sigma = diag(sigma^2).
  * "paper" regime (Section 4.1, Task 1): mu_j ~ U(-1,1), sigma_j ~ U(0, 0.025).
  * dense factor: L_jj = sigma_j and L_jk = sigma_j a_jk / sqrt(j+1) for k < j, a_jk ~ U(-1,1).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

#: iterations at which Table 2 reports the relative squared error
TABLE2_ITERATIONS = (50, 100, 500, 1000)


def _rng(seed: int, instance: int, stream: int) -> np.random.Generator:
    key = np.array([seed & 0xFFFFFFFFFFFFFFFF, (instance << 8) | stream], dtype=np.uint64)
    return np.random.Generator(np.random.Philox(key=key))


def diag_instance(seed: int, instance: int, d: int, regime: str = "unit"):
    """(mu, sigma) for one instance, float64 arrays of length d."""
    g = _rng(seed, instance, 1)
    if regime == "unit":
        mu = g.uniform(0.0, 1.0, d)
        sigma = g.uniform(0.0, 1.0, d)
    elif regime == "paper":
        mu = g.uniform(-1.0, 1.0, d)
        sigma = g.uniform(0.0, 0.025, d)
    else:
        raise ValueError(f"unknown regime {regime!r}")
    return mu, sigma


def dense_instance(seed: int, instance: int, d: int, regime: str = "unit"):
    """(mu, L) with L lower triangular, row-major float64 (d, d), Sigma = L L'."""
    mu, sigma = diag_instance(seed, instance, d, regime)
    g = _rng(seed, instance, 2)
    a = g.uniform(-1.0, 1.0, (d, d))
    L = np.zeros((d, d))
    for j in range(d):
        L[j, j] = sigma[j]
        for k in range(j):
            L[j, k] = sigma[j] * a[j, k] / math.sqrt(j + 1)
    return mu, L


def newsvendor_instance(seed: int, instance: int, n: int):
    """Algorithm 2's products (Section 3.2): demand mu_j ~ U(20, 50), sigma_j ~ U(10, 20) (Section 4.1);
    the costs and the resource row, which the paper does not give: unit cost k_j ~ U(1, 2), selling
    value v_j = k_j U(1.5, 3), holding cost h_j = k_j U(0.1, 0.5), one resource row c = k (a budget in
    money) with level C = 0.5 sum_j k_j mu_j (half of stocking every product at its mean demand)."""
    g = _rng(seed, instance, 4)
    mu = g.uniform(20.0, 50.0, n)
    sigma = g.uniform(10.0, 20.0, n)
    k = g.uniform(1.0, 2.0, n)
    v = k * g.uniform(1.5, 3.0, n)
    h = k * g.uniform(0.1, 0.5, n)
    return dict(mu=mu, sigma=sigma, k=k, h=h, v=v, c=k.copy(), C=0.5 * float(np.dot(k, mu)))


def newsvendor_constraints(seed: int, instance: int, n: int, M: int):
    """Eq. (7)'s technology matrix for M resources, which the paper leaves open: row 0 the budget in
    money (c = k of newsvendor_instance with the same seed and instance), rows 1..M-1 other resources
    with use a_ij ~ U(0.5, 2) per unit; each level C_i = 0.5 sum_j a_ij mu_j (half of stocking every
    product at its mean demand). Returns (A float64 [M][n], C float64 [M])."""
    inst = newsvendor_instance(seed, instance, n)
    g = _rng(seed, instance, 6)
    A = np.empty((M, n))
    A[0] = inst["k"]
    if M > 1:
        A[1:] = g.uniform(0.5, 2.0, (M - 1, n))
    return A, 0.5 * (A @ inst["mu"])


def sqn_dataset(seed: int, n: int, N: int | None = None, density: float | None = None):
    """Task 3's synthetic classification data (Section 4.1): N = 30 n rows of n binary features, labels
    from a random linear combination of the features with 10% label noise. Here: features i.i.d.
    Bernoulli(p) with p = min(1/2, 25/n) (about 25 ones per row at every n >= 50, so the curvature of
    the loss, and with it the meaning of the step parameter beta, does not grow with n); weights
    a_j ~ N(0, 1); label 1 when x'a exceeds its mean p a'1; each label flipped with probability 0.1.
    Returns (X uint8 [N][n], z uint8 [N])."""
    N = 30 * n if N is None else N
    p = min(0.5, 25.0 / n) if density is None else density
    g = _rng(seed, 0, 5)
    X = np.empty((N, n), dtype=np.uint8)
    for i in range(0, N, 4096):                      # in row blocks, so no N x n float array is formed
        X[i:i + 4096] = g.random((min(4096, N - i), n)) < p
    a = g.standard_normal(n)
    mean = p * a.sum()
    z = np.empty(N, dtype=np.uint8)
    for i in range(0, N, 8192):
        z[i:i + 8192] = (X[i:i + 8192].astype(np.float64) @ a - mean) > 0
    flip = g.random(N) < 0.1
    z[flip] ^= 1
    return X, z


@dataclass
class BatchInstance:
    instance: int
    d: int
    N: int
    T: int
    R: int
    mu: np.ndarray = field(repr=False)
    sigma: np.ndarray = field(repr=False)


def uneven_batch(seed: int = 0, n_instances: int = 256, R: int = 4096, d_range=(2, 32),
                 n_range=(2, 50), t_range=(100, 100_000)):
    """Instances of uneven size and horizon: d ~ U{d_range}, N ~ U{n_range},
    T = round(exp(U(ln t_lo, ln t_hi))), mu and sigma from the unit regime."""
    g = _rng(seed, 0xFFFFFF, 3)
    out = []
    for i in range(n_instances):
        d = int(g.integers(d_range[0], d_range[1] + 1))
        N = int(g.integers(n_range[0], n_range[1] + 1))
        T = int(round(math.exp(g.uniform(math.log(t_range[0]), math.log(t_range[1])))))
        mu, sigma = diag_instance(seed, i, d)
        out.append(BatchInstance(i, d, N, T, R, mu, sigma))
    return out


#: workload shapes (R replications, T iterations, d assets, N samples per gradient, M = 1)
WORKLOADS = {
    "tiny": dict(R=1_000, T=100, d=2, N=2, M=1, precision="fp64", noise="gauss",
                 checkpoints=(50, 100), seed=0),
    "paper_scale": dict(R=1_000_000, T=10_000, d=10, N=10, M=1, precision="fp32", noise="gauss",
                        checkpoints=(50, 100, 500, 1000, 10_000), seed=0),
    "uneven": dict(n_instances=256, R=4_096, d_range=(2, 32), n_range=(2, 50),
                   t_range=(100, 100_000), precision="fp32", seed=0),
    "control_variate": dict(R=100_000, T=10_000, d=10, N=10, M=1, precision="fp32",
                            train_pairs=10_000_000, hidden=64, seed=100),
    "stress": dict(R=10_000_000, T=1_000, d=64, N=100, M=1, precision="fp32", noise="t", nu=3,
                   dense=True, checkpoints=(50, 100, 500, 1000), seed=0),
    # Section 4.1, Task 1: one replication per size, K = 1500 iterations, N = 25 samples per
    # gradient (50 at d = 1e5), the "paper" parameter regime
    "paper_shape": dict(R=1, T=1_500, sizes=(500, 5_000, 10_000, 50_000, 100_000),
                        N={500: 25, 5_000: 25, 10_000: 25, 50_000: 25, 100_000: 50}, M=1,
                        precision="fp32", noise="gauss", regime="paper",
                        checkpoints=(50, 100, 500, 1000, 1500), seed=0),
    # Section 4.1, Task 2 (Algorithm 2): one replication per size, K = 1500, S = 25 demand samples
    # per product (50 at 1e6), mu ~ U(20, 50), sigma ~ U(10, 20); costs and budget as newsvendor_instance
    "newsvendor_shape": dict(R=1, T=1_500, sizes=(100, 1_000, 10_000, 100_000, 1_000_000),
                             S={100: 25, 1_000: 25, 10_000: 25, 100_000: 25, 1_000_000: 50}, M=1,
                             checkpoints=(50, 100, 500, 1000, 1500), seed=0),
    # Task 2 over Eq. (7)'s general constraint set: M = 3 resource rows (newsvendor_constraints)
    "newsvendor_lp_shape": dict(R=1, T=1_500, sizes=(100, 1_000, 10_000), S=25, M=1, resources=3,
                                checkpoints=(50, 100, 500, 1000, 1500), seed=0),
    # Task 3 (Algorithms 3-4) at Section 4.1's settings: n features, N = 30 n rows, K = 2000
    "sqn_shape": dict(K=2_000, sizes=(50, 500, 1_000, 5_000), L=10, M=25, b=50, bH=(300, 600), beta=2.0,
                      checkpoints=(50, 100, 500, 1000, 2000), R_batch=1024, seed=0),
}
