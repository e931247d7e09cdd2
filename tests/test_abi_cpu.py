"""The C-ABI library without a GPU: it loads, exports every symbol include/sim.h declares, the
ctypes layouts match the header, and host-side validation rejects what the header says it does."""
import ctypes
import math
import os
import re
import subprocess
import tempfile

import numpy as np
import pytest

from paper_2404_11631_amd import sim, workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sim.h")


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(sim_\w+)\s*\(", text, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(sim.LIB_PATH):
        pytest.skip("libsim.so not built")
    return sim.load()


def test_exports_every_declared_symbol(lib):
    declared = header_functions()
    assert set(declared) == set(sim.EXPORTS)
    for name in declared:
        assert hasattr(lib, name), name
    nm = subprocess.run(["nm", "-D", "--defined-only", sim.LIB_PATH], capture_output=True, text=True)
    if nm.returncode == 0:
        for name in declared:
            assert re.search(rf"\bT {name}\b", nm.stdout), name


def test_struct_layout_matches_header():
    """sizeof/offsetof from a C compile of the header equal the ctypes mirrors."""
    mirrors = {"sim_params": sim.SimParams, "sim_stats_out": sim.SimStats,
               "sim_path_view": sim.SimPathView, "sim_batch_config": sim.SimBatchConfig,
               "sim_cv_opts": sim.SimCvOpts, "sim_cv_fit_out": sim.SimCvFitOut,
               "sim_cv_stats_out": sim.SimCvStats, "sim_cv_view": sim.SimCvView,
               "sim_wide_view": sim.SimWideView, "sim_nv_params": sim.SimNvParams,
               "sim_sqn_params": sim.SimSqnParams, "sim_sqn_view": sim.SimSqnView,
               "sim_sqn_hessian_view": sim.SimSqnHessianView}
    fields = {name: [f[0] for f in cls._fields_] for name, cls in mirrors.items()}
    lines = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{HEADER}"', "int main(void){"]
    for st, fs in fields.items():
        lines.append(f'printf("{st} %zu\\n", sizeof({st}));')
        for f in fs:
            lines.append(f'printf("{st}.{f} %zu\\n", offsetof({st}, {f}));')
    lines.append("return 0;}")
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "layout.c")
        open(src, "w").write("\n".join(lines))
        exe = os.path.join(d, "layout")
        subprocess.check_call(["gcc", "-std=c11", "-Wall", "-o", exe, src])
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split("\n")
    got = dict(line.split() for line in out if line)
    for st, cls in mirrors.items():
        assert int(got[st]) == ctypes.sizeof(cls), st
        for f in fields[st]:
            assert int(got[f"{st}.{f}"]) == getattr(cls, f).offset, (st, f)


def test_strerror(lib):
    assert lib.sim_strerror(0) == b"ok"
    assert lib.sim_strerror(-1) == b"invalid argument"
    assert lib.sim_strerror(-5) == b"unsupported combination"
    assert lib.sim_strerror(-99) == b"unknown error"


def _ok_problem(**kw):
    base = dict(mu=np.array([0.3, 0.6]), sigma=np.array([0.5, 0.2]), N=4, checkpoints=(5, 10))
    base.update(kw)
    return sim.Problem(**base)


@pytest.mark.parametrize("kw,R,T,code", [
    ({}, 100, 10, 0),
    ({}, 0, 10, -1),                                   # R >= 1
    ({}, 2 ** 32, 10, -1),                             # R < 2^32
    ({}, 10, 0, -1),                                   # T >= 1
    ({"N": 1}, 10, 10, -1),                            # Eq. (4) needs N >= 2
    ({"M": 0}, 10, 10, -1),
    ({"lam": 0.0}, 10, 10, -1),
    ({"lam": float("nan")}, 10, 10, -1),
    ({"sigma": np.array([0.5, -0.1])}, 10, 10, -1),
    ({"mu": np.array([0.3, np.inf])}, 10, 10, -1),
    ({"w0": np.array([0.7, 0.4])}, 10, 10, -1),        # outside W
    ({"w0": np.array([-0.1, 0.4])}, 10, 10, -1),
    ({"w0": np.array([0.5, 0.5])}, 10, 10, 0),          # on the face 1'w = 1
    ({"checkpoints": (10, 5)}, 10, 10, -1),            # strictly increasing
    ({"checkpoints": (0,)}, 10, 10, -1),
    ({"checkpoints": (11,)}, 10, 10, -1),              # <= T
    ({"checkpoints": tuple(range(1, 10))}, 10, 10, -1),  # at most 8
    ({"noise": sim.NOISE_T, "nu": 2}, 10, 10, -1),
    ({"noise": 7}, 10, 10, -1),
    ({"precision": 3}, 10, 10, -1),
    ({"gap_eps": -1.0}, 10, 10, -1),
    ({"instance_id": 1 << 24}, 10, 10, -1),
    ({"log_reps": (5, 10)}, 10, 10, -1),               # beyond R
    ({"log_reps": (0, 10)}, 10, 10, 0),
    ({"chol": np.eye(2)}, 10, 10, -5),                  # dense factors need d = 32 or 64
])
def test_validation(lib, kw, R, T, code):
    rc, msg = sim.validate(_ok_problem(**kw), R, T)
    assert rc == code, msg
    if code:
        assert msg


def test_dense_validation(lib):
    mu, L = workloads.dense_instance(0, 0, 32)
    ok = dict(mu=mu, chol=L, N=10)
    assert sim.validate(sim.Problem(**ok), 100, 65535)[0] == 0
    assert sim.validate(sim.Problem(**ok), 100, 65536)[0] == -5            # 16-bit counts
    assert sim.validate(sim.Problem(**ok, precision=sim.FP64), 100, 10)[0] == -5
    up = L.copy()
    up[3, 7] = 1e-3
    assert sim.validate(sim.Problem(mu=mu, chol=up, N=10), 100, 10)[0] == -1   # not lower triangular
    bad = L.copy()
    bad[5, 2] = np.nan
    assert sim.validate(sim.Problem(mu=mu, chol=bad, N=10), 100, 10)[0] == -1
    mu64, L64 = workloads.dense_instance(0, 0, 64)
    assert sim.validate(sim.Problem(mu=mu64, chol=L64, N=10, noise=sim.NOISE_T, nu=3), 100, 10)[0] == 0
    mu16, L16 = workloads.dense_instance(0, 0, 16)
    assert sim.validate(sim.Problem(mu=mu16, chol=L16, N=10), 100, 10)[0] == -5


def test_validation_d_range(lib):
    rc, _ = sim.validate(sim.Problem(mu=np.zeros(65), sigma=np.ones(65)), 10, 10)
    assert rc == -1
    # per-lane kernels: diagonal d <= 32 in FP32, d <= 16 in FP64
    assert sim.validate(sim.Problem(mu=np.zeros(32), sigma=np.ones(32)), 10, 10)[0] == 0
    rc, msg = sim.validate(sim.Problem(mu=np.zeros(33), sigma=np.ones(33)), 10, 10)
    assert rc == -5 and "sim_run_wide" in msg
    assert sim.validate(sim.Problem(mu=np.zeros(16), sigma=np.ones(16), precision=sim.FP64), 10, 10)[0] == 0
    assert sim.validate(sim.Problem(mu=np.zeros(17), sigma=np.ones(17), precision=sim.FP64), 10, 10)[0] == -5


def test_wide_validation(lib):
    """The wide path (sim_run_wide): d a multiple of 4 up to SIM_WIDE_MAX_D, diagonal Sigma, Gaussian
    noise, FP32, R <= 64, N <= 1024, R T <= 2^30."""
    d = 100_000
    mu, sig = workloads.diag_instance(0, 0, d, "paper")
    ok = dict(mu=mu, sigma=sig, N=50)
    assert sim.validate_wide(sim.Problem(**ok), 1, 1500)[0] == 0
    assert sim.validate_wide(sim.Problem(**ok), 64, 1500)[0] == 0
    assert sim.validate_wide(sim.Problem(**ok), 65, 10)[0] == -1
    assert sim.validate_wide(sim.Problem(**ok), 64, 2 ** 25)[0] == -1          # decision record
    assert sim.validate_wide(sim.Problem(mu=mu[:102], sigma=sig[:102], N=25), 1, 10)[0] == -1
    assert sim.validate_wide(sim.Problem(mu=mu[:4], sigma=sig[:4], N=2), 1, 10)[0] == 0
    assert sim.validate_wide(sim.Problem(**ok, noise=sim.NOISE_T), 1, 10)[0] == -5
    assert sim.validate_wide(sim.Problem(**ok, precision=sim.FP64), 1, 10)[0] == -5
    assert sim.validate_wide(sim.Problem(mu=mu[:64], chol=np.diag(sig[:64]), N=5), 1, 10)[0] == -5
    assert sim.validate_wide(sim.Problem(mu=mu, sigma=sig, N=1025), 1, 10)[0] == -1
    assert sim.validate_wide(sim.Problem(**ok, cv_features=True), 1, 10)[0] == -1
    neg = sig.copy()
    neg[7] = -1.0
    assert sim.validate_wide(sim.Problem(mu=mu, sigma=neg, N=50), 1, 10)[0] == -1
    assert sim.validate_wide(sim.Problem(**ok, checkpoints=(10, 5)), 1, 20)[0] == -1


def test_sample_size_schedule_validation(lib):
    """Per-epoch sample sizes N_k: every entry of the ceil(T/M) epochs in [2, 1024] on the wide path,
    in [2, 2^24] on the per-lane path with a diagonal Sigma; a dense factor, control-variate
    features and batches reject a schedule as unsupported."""
    mu, sig = workloads.diag_instance(0, 0, 64, "paper")
    sch = [2 + k for k in range(50)]
    assert sim.validate_wide(sim.Problem(mu=mu, sigma=sig, N=10, n_schedule=sch), 1, 50)[0] == 0
    assert sim.validate_wide(sim.Problem(mu=mu, sigma=sig, N=10, M=3, n_schedule=sch[:17]), 1, 50)[0] == 0
    bad = list(sch)
    bad[49] = 1
    assert sim.validate_wide(sim.Problem(mu=mu, sigma=sig, N=10, n_schedule=bad), 1, 50)[0] == -1
    bad[49] = 1025
    assert sim.validate_wide(sim.Problem(mu=mu, sigma=sig, N=10, n_schedule=bad), 1, 50)[0] == -1
    assert sim.validate_wide(sim.Problem(mu=mu, sigma=sig, N=10, n_schedule=bad), 1, 49)[0] == 0   # 49 epochs
    assert sim.validate(sim.Problem(mu=mu[:8], sigma=sig[:8], N=10, n_schedule=sch), 10, 50)[0] == 0
    assert sim.validate(sim.Problem(mu=mu[:8], sigma=sig[:8], N=10, M=4, n_schedule=sch[:13]), 10, 50)[0] == 0
    assert sim.validate(sim.Problem(mu=mu[:8], sigma=sig[:8], N=10, n_schedule=bad[:49] + [1]), 10, 50)[0] == -1
    L = np.tril(np.ones((32, 32))) * 0.1
    assert sim.validate(sim.Problem(mu=mu[:32], chol=L, N=10, n_schedule=sch), 10, 50)[0] == -5
    assert sim.validate(sim.Problem(mu=mu[:8], sigma=sig[:8], N=10, n_schedule=sch, cv_features=True,
                                    cv_ref=-mu[:8]), 10, 50)[0] == -5
    with pytest.raises(sim.SimError) as e:
        sim.plan_batch([sim.Problem(mu=mu[:8], sigma=sig[:8], N=10, n_schedule=sch)], [64], [50])
    assert e.value.code == -5


def test_newsvendor_validation(lib):
    """Algorithm 2 (sim_run_newsvendor): n a multiple of 4, c > 0, C > 0, sigma >= 0, x0 in X,
    1 <= S <= 1024, R <= 64, R T <= 2^30."""
    inst = workloads.newsvendor_instance(0, 0, 1000)
    assert sim.validate_newsvendor(inst, 1, 1500, S=25)[0] == 0
    assert sim.validate_newsvendor(inst, 65, 10, S=25)[0] == -1
    assert sim.validate_newsvendor(inst, 64, 2 ** 25, S=25)[0] == -1
    assert sim.validate_newsvendor(dict(inst, C=0.0), 1, 10, S=25)[0] == -1
    assert sim.validate_newsvendor(inst, 1, 10, S=0)[0] == -1
    assert sim.validate_newsvendor(inst, 1, 10, S=1025)[0] == -1
    bad = {f: (inst[f][:998] if f != "C" else inst[f]) for f in inst}
    assert sim.validate_newsvendor(bad, 1, 10, S=25)[0] == -1            # not a multiple of 4
    c0 = dict(inst, c=np.where(np.arange(1000) == 3, 0.0, inst["c"]))
    assert sim.validate_newsvendor(c0, 1, 10, S=25)[0] == -1
    x0 = np.zeros(1000)
    x0[5] = 1.01 * inst["C"] / inst["c"][5]
    assert sim.validate_newsvendor(inst, 1, 10, S=25, x0=x0)[0] == -1     # outside the budget
    x0[5] = 0.5 * inst["C"] / inst["c"][5]
    assert sim.validate_newsvendor(inst, 1, 10, S=25, x0=x0)[0] == 0
    assert sim.validate_newsvendor(inst, 1, 20, S=25, checkpoints=(20, 30))[0] == -1


def test_sqn_validation(lib):
    """Algorithms 3-4 (sim_run_sqn): 1 <= n <= 8192, 1 <= N < 2^31, R <= 4096, 1 <= K < 2^32, L >= 1,
    1 <= M <= 32, 1 <= b, b_H <= 1024, beta > 0, checkpoints increasing in [1, K]."""
    assert sim.validate_sqn(1500, 50, 1, 2000)[0] == 0
    assert sim.validate_sqn(150000, 5000, 512, 2000, bH=600, checkpoints=(50, 100, 500, 1000))[0] == 0
    assert sim.validate_sqn(1500, 0, 1, 10)[0] == -1
    assert sim.validate_sqn(1500, 8193, 1, 10)[0] == -1
    assert sim.validate_sqn(0, 50, 1, 10)[0] == -1
    assert sim.validate_sqn(1500, 50, 4097, 10)[0] == -1
    assert sim.validate_sqn(1500, 50, 1, 0)[0] == -1
    assert sim.validate_sqn(1500, 50, 1, 2 ** 32)[0] == -1
    assert sim.validate_sqn(1500, 50, 1, 10, L=0)[0] == -1
    assert sim.validate_sqn(1500, 50, 1, 10, M=33)[0] == -1
    assert sim.validate_sqn(1500, 50, 1, 10, M=0)[0] == -1
    assert sim.validate_sqn(1500, 50, 1, 10, b=1025)[0] == -1
    assert sim.validate_sqn(1500, 50, 1, 10, bH=0)[0] == -1
    assert sim.validate_sqn(1500, 50, 1, 10, beta=0.0)[0] == -1
    assert sim.validate_sqn(1500, 50, 1, 10, beta=float("nan"))[0] == -1
    assert sim.validate_sqn(1500, 50, 1, 10, checkpoints=(5, 5))[0] == -1
    assert sim.validate_sqn(1500, 50, 1, 10, checkpoints=(11,))[0] == -1
    assert sim.validate_sqn(1500, 50, 1, 10, instance_id=1 << 24)[0] == -1


def test_create_without_gpu_fails_cleanly(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p()
    assert lib.sim_create(0, None, ctypes.byref(h)) == -3
    assert not h.value


@pytest.mark.parametrize("d,N,M,T", [(10, 10, 1, 10_000), (1, 2, 1, 7), (5, 4, 3, 100), (32, 6, 1, 500)])
def test_cv_law_matches_oracle(lib, d, N, M, T):
    """The library's reference-decision probabilities (Gauss-Legendre) against the oracle's
    (Simpson): two independent quadratures of the same integrals."""
    import oracle
    g = np.random.default_rng(d)
    mu = g.uniform(0.1, 0.9, d)
    sigma = g.uniform(0.1, 0.9, d)
    b = sigma ** 2 * np.full(d, 0.8 / d) - mu
    p = sim.Problem(mu=mu, sigma=sigma, N=N, M=M, cv_ref=b)
    probs, S2, S4 = sim.cv_law(p, T)
    ref, tot = oracle.cv_pick_probs(b, sigma / np.sqrt(N))
    assert abs(probs.sum() - 1) < 1e-12 and abs(tot - 1) < 1e-11
    assert np.max(np.abs(probs - ref)) < 1e-12
    oS2, oS4 = oracle.cv_weights(T, M)[:2]
    assert S2 == oS2 and math.isclose(S4, oS4, rel_tol=1e-13)


def test_cv_feature_validation(lib):
    mu, sigma = workloads.diag_instance(0, 0, 4)
    b = sigma ** 2 * 0.2 - mu
    assert sim.validate(sim.Problem(mu=mu, sigma=sigma, N=4, cv_features=True, cv_ref=b), 10, 100)[0] == 0
    assert sim.validate(sim.Problem(mu=mu, sigma=sigma, N=4, cv_features=True), 10, 100)[0] == -1
    z = sigma.copy()
    z[1] = 0.0
    assert sim.validate(sim.Problem(mu=mu, sigma=z, N=4, cv_features=True, cv_ref=b), 10, 100)[0] == -5
    assert sim.validate(sim.Problem(mu=mu, sigma=sigma, N=4, cv_features=True, cv_ref=b,
                                    precision=sim.FP64), 10, 100)[0] == -5
    assert sim.validate(sim.Problem(mu=mu, sigma=sigma, N=4, cv_features=True, cv_ref=b), 10, 100_000)[0] == -5


def test_create_ex_without_gpu_fails_cleanly(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p()
    rc = lib.sim_create_ex(0, None, 1 << 20, ctypes.byref(h))
    assert rc != 0 and not h.value


def test_param_gen_regimes():
    """sim_param_gen: the paper's ranges (Section 4.1) and U(0,1); a fixed seed gives fixed values,
    another seed others; the sample moments of 1e5 draws match those of the uniform law (five
    standard errors)."""
    d = 100_000
    for regime, (lo, hi), smax in ((sim.REGIME_UNIT, (0.0, 1.0), 1.0), (sim.REGIME_PAPER, (-1.0, 1.0), 0.025)):
        mu, sigma = sim.param_gen(d, regime, 7)
        assert mu.min() >= lo and mu.max() < hi and sigma.min() >= 0.0 and sigma.max() < smax
        for x, a, b in ((mu, lo, hi), (sigma, 0.0, smax)):
            m, v = (a + b) / 2, (b - a) ** 2 / 12
            assert abs(x.mean() - m) < 5 * np.sqrt(v / d)
            assert abs(x.var() - v) < 5 * np.sqrt((b - a) ** 4 / 180 / d)
        mu2, sigma2 = sim.param_gen(d, regime, 7)
        assert np.array_equal(mu, mu2) and np.array_equal(sigma, sigma2)
        mu3, _ = sim.param_gen(d, regime, 8)
        assert not np.array_equal(mu, mu3)
    with pytest.raises(sim.SimError):
        sim.param_gen(10, 5, 0)
    with pytest.raises(sim.SimError):
        sim.param_gen(0, sim.REGIME_UNIT, 0)


def test_newsvendor_lp_validation(lib):
    n = 16
    inst = workloads.newsvendor_instance(1, 0, n)
    A, C = workloads.newsvendor_constraints(1, 0, n, 3)
    ok = dict(S=5)
    assert sim.validate_newsvendor_lp(inst, A, C, 2, 100, **ok)[0] == 0
    general = {k: v for k, v in inst.items() if k not in ("c", "C")}      # c and C are not needed
    assert sim.validate_newsvendor_lp(general, A, C, 2, 100, **ok)[0] == 0
    bad = A.copy()
    bad[1, 2] = -1.0
    assert sim.validate_newsvendor_lp(inst, bad, C, 2, 100, **ok)[0] == -1
    zero = A.copy()
    zero[:, 5] = 0.0
    assert sim.validate_newsvendor_lp(inst, zero, C, 2, 100, **ok)[0] == -1
    assert sim.validate_newsvendor_lp(inst, A, np.array([1.0, 0.0, 1.0]), 2, 100, **ok)[0] == -1
    A9, C9 = workloads.newsvendor_constraints(1, 0, n, 9)
    assert sim.validate_newsvendor_lp(inst, A9, C9, 2, 100, **ok)[0] == -1
    assert sim.validate_newsvendor_lp(inst, A, C, 64, 1 << 19, **ok)[0] == -1        # R T above 2^24
    x0 = np.full(n, 1e6)
    assert sim.validate_newsvendor_lp(inst, A, C, 1, 10, x0=x0, **ok)[0] == -1
    big = workloads.newsvendor_instance(1, 0, 262148)
    Ab, Cb = workloads.newsvendor_constraints(1, 0, 262148, 1)
    assert sim.validate_newsvendor_lp(big, Ab, Cb, 1, 10, **ok)[0] == -5
