"""Pins of the rounding bound the oracle's replay rule uses (Section 3.1, Eq. (4)-(5)).

The oracle accepts a binary32 decision that differs from its own only at a step whose vertex margin
is within twice the bound B_t it computes for unit roundoff 2^-24. These tests evaluate the same
sample gradient the way a binary32 system does, on the CPU, and check that B_t covers the error at
every step of real paths, in both evaluation orders the bound claims to cover:

* return-space / one-pass order with a diagonal L (one lane per replication): v = (kappa sigma) .* w,
  one pass over the samples accumulating s1 = sum_i z_i and s2 = sum_i z_i (z_i'v), then
  g = c2 (s2 - s1 (s1'v)/N) - mu - c1 s1 with normals divided by kappa = sqrt(2 ln 2);
* noise-space order with a dense L (four lanes per replication): v = (kappa L)'w, per-lane partial
  dot products combined over the four lanes, h = 2 lambda/(N-1) (s2 - s1 (s1'v)/N) - s1/N and
  g = (kappa L) h - mu, the products summed in blocks of four as the matrix cores do.

Each binary32 evaluation also perturbs every normal (absolute error up to 8 u (|z| + 1)) and the
t-noise scale (relative 4 u), a model of the hardware transcendentals' error, so the bound is shown
to cover the inputs' rounding too. Every operation is rounded to binary32 with numpy float32; a
fused multiply-add is one rounding of the exact product-sum (the product of two binary32 values is
exact in binary64). Gaussian and elliptical t(3) noise, d up to 64, lambda 1/2 and 1.

Each test also checks that the bound is not vacuous, in two ways: B_t stays below 0.5% of max_j |g_j|
at every step, and the largest binary32 error seen along the path reaches at least 1/3300 of B_t
(measured: 1/26 to 1/1600). A bound inflated tenfold (a wrong accumulation depth or |L| term that
would let a binary32 decision far from a tie through the replay) fails one of the two.
"""
import numpy as np
import pytest

import oracle
from paper_2404_11631_amd import workloads

U = 2.0 ** -24
KAPPA = float(np.sqrt(2.0 * np.log(2.0)))
F32 = np.float32


def f32(x):
    return np.asarray(x, dtype=np.float64).astype(np.float32)


def fma32(a, b, c):
    """One binary32 rounding of a*b + c (a, b, c binary32): the product is exact in binary64."""
    return (np.asarray(a, np.float64) * np.asarray(b, np.float64) + np.asarray(c, np.float64)).astype(np.float32)


def device_normals(P, rep, epoch, n, rng):
    """The path's normals as a binary32 system produces them: z / kappa, with the transcendentals'
    error modelled as an absolute perturbation of up to 8 u (|z| + 1)."""
    z = oracle.normals(P.p.seed, 0, P.p.instance, rep, epoch, 0, n)
    e = rng.uniform(-1.0, 1.0, size=n) * 8.0 * U * (np.abs(z) + 1.0)
    return f32((z + e) / KAPPA)


def t_scales(P, zx, nu, rng):
    """a_i = sqrt(nu - 2)/kappa * rsqrt(sum_k e_k^2) in binary32 (rsqrt with relative error 4 u)."""
    N = zx.shape[0] // nu
    tscale = f32(np.sqrt(nu - 2.0) / KAPPA)
    a = np.zeros(N, np.float32)
    for i in range(N):
        ss = F32(0.0)
        for k in range(nu):
            e = zx[nu * i + k]
            ss = fma32(e, e, ss)
        r = 1.0 / np.sqrt(np.float64(ss)) * (1.0 + rng.uniform(-4.0, 4.0) * U)
        a[i] = F32(tscale * F32(r))
    return a


def iterates(P, rep, T):
    """w_0 .. w_{T-1} of the oracle's own path (w_t = 2/(t(t+1)) sum_{s<t} (s+1) e_{a_s}) and the
    integer signatures S the binary32 system scales."""
    _, dec = P.path(rep, T, want_decisions=True)
    d = P.d
    S = np.zeros(d, np.int64)
    out = []
    for t in range(T):
        w = np.zeros(d) if t == 0 else 2.0 * S / (t * (t + 1.0))
        out.append((t, w.copy(), S.copy()))
        if dec[t] > 0:
            S[dec[t] - 1] += t + 1
    return out


def g32_diag(P, sig, rep, t, S, lam, noise, nu, fused, rng):
    d, N = P.d, P.N
    z = device_normals(P, rep, t, N * d + (N * nu if noise else 0), rng)
    zm = z[: N * d].reshape(N, d)
    if noise:
        a = t_scales(P, z[N * d:], nu, rng)
        zm = (zm * a[:, None]).astype(np.float32)
    sz = f32(KAPPA * sig)
    cw = F32(0.0) if t == 0 else f32(2.0 / (t * (t + 1.0)))
    w = (S.astype(np.float32) * cw).astype(np.float32)
    v = (sz * w).astype(np.float32)
    s1 = np.zeros(d, np.float32)
    s2 = np.zeros(d, np.float32)
    for i in range(N):
        dot = F32(0.0)
        for j in range(d):
            dot = fma32(zm[i, j], v[j], dot)
        s1 = (s1 + zm[i]).astype(np.float32)
        s2 = fma32(zm[i], dot, s2)
    dot1 = F32(0.0)
    for j in range(d):
        dot1 = fma32(s1[j], v[j], dot1)
    qn = F32(dot1 * f32(1.0 / N))
    c1 = f32(sz.astype(np.float64) / N)
    c2 = f32(2.0 * lam * sz.astype(np.float64) / (N - 1.0))
    mu = f32(P.mu)
    inner = (s2 - (s1 * qn).astype(np.float32)).astype(np.float32)
    if fused:   # contracted: fma(-c1, s1, c2 * inner - mu)
        return fma32(-c1, s1, ((c2 * inner).astype(np.float32) - mu).astype(np.float32))
    return (((c2 * inner).astype(np.float32) - mu).astype(np.float32) - (c1 * s1).astype(np.float32)).astype(np.float32)


def matvec_blocks4(A, x):
    """y = A x in binary32, each row summed in blocks of four products added to the accumulator in
    turn (the order of the 16x16x4 matrix-core step)."""
    m, k = A.shape
    y = np.zeros(m, np.float32)
    for k0 in range(0, k, 4):
        part = np.zeros(m, np.float64)
        for kk in range(k0, min(k0 + 4, k)):
            part += A[:, kk].astype(np.float64) * np.float64(x[kk])
        y = (y.astype(np.float64) + part).astype(np.float32)
    return y


def g32_dense(P, rep, t, S, lam, noise, nu, rng):
    d, N = P.d, P.N
    L = P.chol
    z = device_normals(P, rep, t, N * d + (N * nu if noise else 0), rng)
    zm = z[: N * d].reshape(N, d)
    a = t_scales(P, z[N * d:], nu, rng) if noise else np.ones(N, np.float32)
    cw = F32(0.0) if t == 0 else f32(2.0 / (t * (t + 1.0)))
    w = (S.astype(np.float32) * cw).astype(np.float32)
    Ag = f32(KAPPA * L)
    v = matvec_blocks4(Ag.T.copy(), w)
    lanes = [np.arange(d)[(np.arange(d) // 4) % 4 == p] for p in range(4)]   # blocks of four, every fourth

    def rep_sum(terms):
        part = []
        for idx in lanes:
            acc = F32(0.0)
            for k in idx:
                acc = fma32(terms[0][k], terms[1][k], acc)
            part.append(acc)
        x = [F32(part[p] + part[p ^ 2]) for p in range(4)]   # lane ^ 32, then lane ^ 16
        return F32(x[0] + x[1])

    s1 = np.zeros(d, np.float32)
    s2 = np.zeros(d, np.float32)
    for i in range(N):
        dot = rep_sum((zm[i], v))
        a2dot = F32(F32(a[i] * a[i]) * dot) if noise else dot
        s1 = fma32(a[i], zm[i], s1) if noise else (s1 + zm[i]).astype(np.float32)
        s2 = fma32(zm[i], a2dot, s2)
    dot1 = rep_sum((s1, v))
    inv_n = f32(1.0 / N)
    qn = F32(dot1 * inv_n)
    cu = f32(2.0 * lam / (N - 1.0))
    h = ((cu * (s2 - (s1 * qn).astype(np.float32)).astype(np.float32)).astype(np.float32)
         - (s1 * inv_n).astype(np.float32)).astype(np.float32)
    return (matvec_blocks4(Ag, h) - f32(P.mu)).astype(np.float32)


def check_path(P, T, g32_fn, frac=5e-3, floor=3e-4):
    worst = 0.0
    for t, w, S in iterates(P, 0, T):
        g64, B = P.gradient_bound(0, t, w, U)
        g32 = g32_fn(t, S)
        err = np.abs(g32.astype(np.float64) - g64).max()
        assert err <= B, (t, err, B)
        assert B < frac * np.abs(g64).max(), (t, B, np.abs(g64).max())
        worst = max(worst, err / B)
    assert worst >= floor, worst
    return worst


@pytest.mark.parametrize("d,N,lam,noise", [(2, 2, 0.5, 0), (10, 10, 0.5, 0), (10, 10, 1.0, 0), (32, 50, 0.5, 0),
                                           (7, 25, 0.5, 1), (16, 100, 1.0, 1)])
@pytest.mark.parametrize("fused", [False, True])
def test_bound_covers_binary32_one_pass_diagonal(d, N, lam, noise, fused):
    mu, sig = workloads.diag_instance(3, 0, d)
    P = oracle.OracleProblem(mu, sig, N=N, lam=lam, noise=noise, nu=3, seed=11)
    rng = np.random.default_rng(d * 1000 + N)
    check_path(P, 30, lambda t, S: g32_diag(P, sig, 0, t, S, lam, noise, 3, fused, rng))


@pytest.mark.parametrize("d,N,noise", [(16, 10, 0), (32, 25, 1), (64, 100, 1)])
def test_bound_covers_binary32_noise_space_dense(d, N, noise):
    mu, L = workloads.dense_instance(4, 0, d)
    P = oracle.OracleProblem(mu, chol=L, N=N, noise=noise, nu=3, seed=12)
    rng = np.random.default_rng(d + N)
    T = 12 if d == 64 else 25
    check_path(P, T, lambda t, S: g32_dense(P, 0, t, S, 0.5, noise, 3, rng))


def test_bound_scales_with_unit_roundoff_and_depth():
    """B is linear in the unit roundoff and grows with the accumulation depth N + d + 8."""
    mu, sig = workloads.diag_instance(5, 0, 8)
    w = np.full(8, 0.1)
    P10 = oracle.OracleProblem(mu, sig, N=10, seed=1)
    g, b24 = P10.gradient_bound(0, 3, w, 2.0 ** -24)
    _, b53 = P10.gradient_bound(0, 3, w, 2.0 ** -53)
    assert b53 == pytest.approx(b24 * 2.0 ** -29, rel=1e-12)
    _, b0 = P10.gradient_bound(0, 3, w, 0.0)
    assert b0 == 0.0
    g2, _ = P10.gradient_bound(0, 3, w, 2.0 ** -24)
    np.testing.assert_array_equal(g, g2)
    np.testing.assert_allclose(g, P10.sample_gradient(0, 3, w)[0], rtol=0, atol=0)
