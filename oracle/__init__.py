"""Plain serial FP64 CPU oracle for Algorithm 1 (Section 3.1) run over replications.

TEST INFRASTRUCTURE: only the test suite, the smoke check and the CPU-baseline leg of the
benchmark import this package. It never serves the product path, and it shares no code with
the HIP library.

The arithmetic lives in ``oracle.c`` (plain C, FP64, built with ``-ffp-contract=off``); this
module only builds it and marshals arguments through ctypes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

MAX_D = 64
MAX_CKPT = 8
TAU_NONE = 0xFFFFFFFF
NOISE_GAUSS, NOISE_T = 0, 1
U32 = 2.0 ** -24
U64 = 2.0 ** -53


def build(force: bool = True) -> str:
    """Compile oracle.c, wide.c, newsvendor.c, sqn.c and cv.c into liboracle.so (plain gcc, no
    fast-math, no FMA contraction)."""
    srcs = [os.path.join(HERE, f) for f in ("oracle.c", "wide.c", "newsvendor.c", "sqn.c", "cv.c")]
    stale = any(os.path.getmtime(LIB_PATH) < os.path.getmtime(f) for f in srcs) if os.path.exists(LIB_PATH) else True
    if force or stale:
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
                               "-Wall", "-Wextra", "-fPIC", "-shared", "-o", tmp] + srcs + ["-lm"],
                              cwd=HERE)
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


class Problem(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int32), ("N", ctypes.c_int32), ("M", ctypes.c_int32),
                ("noise", ctypes.c_int32), ("nu", ctypes.c_int32), ("n_ckpt", ctypes.c_int32),
                ("instance", ctypes.c_uint32), ("pad_", ctypes.c_uint32),
                ("seed", ctypes.c_uint64), ("lam", ctypes.c_double), ("gap_eps", ctypes.c_double),
                ("mu", ctypes.POINTER(ctypes.c_double)), ("chol", ctypes.POINTER(ctypes.c_double)),
                ("w0", ctypes.POINTER(ctypes.c_double)), ("ckpt", ctypes.c_int64 * MAX_CKPT),
                ("cv_ref", ctypes.POINTER(ctypes.c_double)), ("n_sched", ctypes.POINTER(ctypes.c_int32))]


class PathOut(ctypes.Structure):
    _fields_ = [("y", ctypes.c_double), ("f_ckpt", ctypes.c_double * MAX_CKPT),
                ("cnt", ctypes.c_uint32 * (MAX_D + 1)), ("wsum", ctypes.c_uint64 * MAX_D),
                ("tau", ctypes.c_uint32), ("tau_lo", ctypes.c_uint32), ("tau_hi", ctypes.c_uint32),
                ("n_ambiguous", ctypes.c_uint64), ("n_replayed", ctypes.c_uint64),
                ("n_mismatch", ctypes.c_uint64), ("first_mismatch", ctypes.c_int64),
                ("identity_err", ctypes.c_double), ("min_margin", ctypes.c_double),
                ("cv_count", ctypes.c_double * (MAX_D + 1)), ("cv_count1", ctypes.c_double * (MAX_D + 1)),
                ("cv_amb", ctypes.c_double)]


class WideProblem(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int64), ("N", ctypes.c_int32), ("M", ctypes.c_int32),
                ("instance", ctypes.c_uint32), ("n_ckpt", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("lam", ctypes.c_double), ("gap_eps", ctypes.c_double),
                ("mu", ctypes.POINTER(ctypes.c_double)), ("sigma", ctypes.POINTER(ctypes.c_double)),
                ("w0", ctypes.POINTER(ctypes.c_double)), ("ckpt", ctypes.c_int64 * MAX_CKPT),
                ("n_sched", ctypes.POINTER(ctypes.c_int32))]


class WideOut(ctypes.Structure):
    _fields_ = [("y", ctypes.c_double), ("f_ckpt", ctypes.c_double * MAX_CKPT),
                ("cnt", ctypes.POINTER(ctypes.c_uint32)), ("wsum", ctypes.POINTER(ctypes.c_uint64)),
                ("tau", ctypes.c_uint32), ("tau_lo", ctypes.c_uint32), ("tau_hi", ctypes.c_uint32),
                ("pad_", ctypes.c_uint32), ("n_ambiguous", ctypes.c_uint64), ("n_replayed", ctypes.c_uint64),
                ("n_mismatch", ctypes.c_uint64), ("first_mismatch", ctypes.c_int64),
                ("identity_err", ctypes.c_double), ("min_margin", ctypes.c_double)]


class NvProblem(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("S", ctypes.c_int32), ("M", ctypes.c_int32), ("instance", ctypes.c_uint32),
                ("n_ckpt", ctypes.c_int32), ("seed", ctypes.c_uint64), ("C", ctypes.c_double),
                ("gap_eps", ctypes.c_double)] + [(f, ctypes.POINTER(ctypes.c_double)) for f in
                                                 ("mu", "sigma", "k", "h", "v", "c", "x0")] + \
               [("ckpt", ctypes.c_int64 * MAX_CKPT)]


class NvOut(ctypes.Structure):
    _fields_ = [("y", ctypes.c_double), ("f_ckpt", ctypes.c_double * MAX_CKPT),
                ("cnt", ctypes.POINTER(ctypes.c_uint32)), ("wsum", ctypes.POINTER(ctypes.c_uint64)),
                ("tau", ctypes.c_uint32), ("tau_lo", ctypes.c_uint32), ("tau_hi", ctypes.c_uint32),
                ("pad_", ctypes.c_uint32), ("n_ambiguous", ctypes.c_uint64), ("n_replayed", ctypes.c_uint64),
                ("n_mismatch", ctypes.c_uint64), ("first_mismatch", ctypes.c_int64),
                ("identity_err", ctypes.c_double), ("min_margin", ctypes.c_double)]


class SqnProblem(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("N", ctypes.c_int64), ("L", ctypes.c_int32), ("M", ctypes.c_int32),
                ("b", ctypes.c_int32), ("bH", ctypes.c_int32), ("beta", ctypes.c_double),
                ("instance", ctypes.c_uint32), ("n_ckpt", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("X", ctypes.POINTER(ctypes.c_uint8)), ("z", ctypes.POINTER(ctypes.c_uint8)),
                ("ckpt", ctypes.c_int64 * MAX_CKPT), ("pairs_fp32", ctypes.c_int32), ("pad_", ctypes.c_int32)]


class SqnOut(ctypes.Structure):
    _fields_ = [("F", ctypes.c_double), ("F_ckpt", ctypes.c_double * MAX_CKPT),
                ("w", ctypes.POINTER(ctypes.c_double)), ("pairs", ctypes.c_int64)]


class CvStats(ctypes.Structure):
    _fields_ = [("n", ctypes.c_uint64), ("n_aux", ctypes.c_uint64), ("beta", ctypes.c_double),
                ("mean_plain", ctypes.c_double), ("var_plain", ctypes.c_double),
                ("ci95_plain", ctypes.c_double), ("mean_resid", ctypes.c_double),
                ("var_resid", ctypes.c_double), ("mean_h_aux", ctypes.c_double),
                ("var_h_aux", ctypes.c_double), ("mean_cv", ctypes.c_double),
                ("var_est", ctypes.c_double), ("ci95_cv", ctypes.c_double)]


class Stats(ctypes.Structure):
    _fields_ = [("R", ctypes.c_uint64), ("T", ctypes.c_uint64), ("mean", ctypes.c_double),
                ("var", ctypes.c_double), ("ci95", ctypes.c_double), ("ymin", ctypes.c_double),
                ("ymax", ctypes.c_double), ("f_mean", ctypes.c_double * MAX_CKPT),
                ("f_sd", ctypes.c_double * MAX_CKPT), ("rse_mean", ctypes.c_double * MAX_CKPT),
                ("rse_sd", ctypes.c_double * MAX_CKPT), ("rse_undef", ctypes.c_uint64 * MAX_CKPT),
                ("decision_total", ctypes.c_uint64 * (MAX_D + 1)), ("tau_count", ctypes.c_uint64),
                ("tau_mean", ctypes.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        L.or_philox4x32_10.argtypes = [ctypes.POINTER(ctypes.c_uint32)] * 3
        L.or_uniform.argtypes = [ctypes.c_uint32]
        L.or_uniform.restype = ctypes.c_double
        L.or_normals.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint64,
                                 ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64, dp]
        L.or_draw_returns.argtypes = [ctypes.POINTER(Problem), ctypes.c_uint64, ctypes.c_uint64, dp]
        L.or_sample_gradient.argtypes = [ctypes.POINTER(Problem), ctypes.c_uint64, ctypes.c_uint64,
                                         dp, dp, dp, dp]
        L.or_sample_gradient_bound.argtypes = [ctypes.POINTER(Problem), ctypes.c_uint64, ctypes.c_uint64,
                                               dp, ctypes.c_double, dp, dp]
        L.or_objective.argtypes = [ctypes.POINTER(Problem), dp]
        L.or_objective.restype = ctypes.c_double
        L.or_path.argtypes = [ctypes.POINTER(Problem), ctypes.c_uint64, ctypes.c_uint64,
                              ctypes.POINTER(ctypes.c_uint8), ctypes.c_double,
                              ctypes.POINTER(PathOut), ctypes.POINTER(ctypes.c_uint8)]
        L.or_run_range.argtypes = [ctypes.POINTER(Problem), ctypes.c_uint64, ctypes.c_uint64,
                                   ctypes.c_uint64, ctypes.POINTER(PathOut)]
        L.or_reduce.argtypes = [ctypes.POINTER(Problem), ctypes.c_uint64, ctypes.POINTER(PathOut),
                                ctypes.c_uint64, ctypes.POINTER(Stats)]
        u64 = ctypes.c_uint64
        L.or_cv_pick_probs.argtypes = [ctypes.c_int, dp, dp, dp]
        L.or_cv_pick_probs.restype = ctypes.c_double
        L.or_cv_weights.argtypes = [u64, ctypes.c_int, dp]
        L.or_cv_top.argtypes = [ctypes.c_int, dp]
        L.or_cv_top.restype = ctypes.c_int
        L.or_cv_features.argtypes = [ctypes.c_int, dp, dp, dp, dp, dp]
        L.or_cv_aux.argtypes = [ctypes.POINTER(Problem), u64, dp, u64, dp, dp]
        L.or_cv_aux.restype = None
        L.or_bf16.argtypes = [ctypes.c_double]
        L.or_bf16.restype = ctypes.c_double
        L.or_mlp_param_count.argtypes = [ctypes.c_int]
        L.or_mlp_param_count.restype = ctypes.c_size_t
        L.or_mlp_forward.argtypes = [dp, ctypes.c_int, dp, u64, ctypes.c_int, dp]
        L.or_mlp_grad.argtypes = [dp, ctypes.c_int, dp, dp, u64, ctypes.c_int, dp]
        L.or_mlp_grad.restype = ctypes.c_double
        L.or_wide_path.argtypes = [ctypes.POINTER(WideProblem), u64, u64, ctypes.POINTER(ctypes.c_uint32),
                                   ctypes.c_double, ctypes.POINTER(WideOut), ctypes.POINTER(ctypes.c_uint32)]
        L.or_wide_gradient.argtypes = [ctypes.POINTER(WideProblem), u64, u64, dp, dp, ctypes.c_double, dp]
        L.or_wide_gradient.restype = None
        L.or_wide_objective.argtypes = [ctypes.POINTER(WideProblem), dp]
        L.or_wide_objective.restype = ctypes.c_double
        L.or_nv_path.argtypes = [ctypes.POINTER(NvProblem), u64, u64, ctypes.POINTER(ctypes.c_uint32),
                                 ctypes.c_double, ctypes.POINTER(NvOut), ctypes.POINTER(ctypes.c_uint32)]
        L.or_nv_gradient.argtypes = [ctypes.POINTER(NvProblem), u64, u64, dp, dp, ctypes.POINTER(ctypes.c_uint32)]
        L.or_nv_gradient.restype = None
        L.or_nv_gradient_bound.argtypes = [ctypes.POINTER(NvProblem), u64, u64, dp, ctypes.c_double, dp]
        L.or_nv_gradient_bound.restype = None
        L.or_nv_cost.argtypes = [ctypes.POINTER(NvProblem), dp]
        L.or_nv_cost.restype = ctypes.c_double
        u32p = ctypes.POINTER(ctypes.c_uint32)
        L.or_sqn_indices.argtypes = [ctypes.POINTER(SqnProblem), u64, u64, ctypes.c_uint32, ctypes.c_uint32, u32p]
        L.or_sqn_indices.restype = None
        L.or_sqn_loss.argtypes = [ctypes.POINTER(SqnProblem), dp]
        L.or_sqn_loss.restype = ctypes.c_double
        L.or_sqn_gradient.argtypes = [ctypes.POINTER(SqnProblem), u32p, ctypes.c_uint32, dp, dp]
        L.or_sqn_gradient.restype = None
        L.or_sqn_hessian_vector.argtypes = [ctypes.POINTER(SqnProblem), u32p, ctypes.c_uint32, dp, dp, dp]
        L.or_sqn_hessian_vector.restype = None
        L.or_sqn_hessian_approx.argtypes = [ctypes.c_int64, ctypes.c_int, dp, dp, dp]
        L.or_sqn_hessian_approx.restype = None
        L.or_sqn_run.argtypes = [ctypes.POINTER(SqnProblem), u64, u64, ctypes.POINTER(SqnOut)]
        L.or_cv_beta.argtypes = [dp, dp, u64, dp, dp]
        L.or_cv_estimate.argtypes = [dp, dp, u64, dp, u64, ctypes.c_double, ctypes.POINTER(CvStats)]
        _lib = L
    return _lib


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class OracleProblem:
    """Keeps the numpy buffers of one problem alive next to its ctypes struct."""

    def __init__(self, mu, sigma=None, chol=None, *, N, M=1, lam=0.5, w0=None, noise=NOISE_GAUSS,
                 nu=3, seed=0, instance=0, ckpt=(), gap_eps=1e-2, cv_ref=None, n_sched=None):
        self.mu = np.ascontiguousarray(mu, dtype=np.float64)
        d = self.mu.shape[0]
        if chol is None:
            chol = np.diag(np.asarray(sigma, dtype=np.float64))
        self.chol = np.ascontiguousarray(chol, dtype=np.float64).reshape(d, d)
        self.w0 = None if w0 is None else np.ascontiguousarray(w0, dtype=np.float64)
        ck = list(ckpt)
        if len(ck) > MAX_CKPT:
            raise ValueError("at most 8 checkpoints")
        p = Problem()
        p.d, p.N, p.M, p.noise, p.nu, p.n_ckpt = d, N, M, noise, nu, len(ck)
        p.instance, p.seed, p.lam, p.gap_eps = instance, seed, lam, gap_eps
        p.mu, p.chol = _dptr(self.mu), _dptr(self.chol)
        p.w0 = _dptr(self.w0) if self.w0 is not None else ctypes.POINTER(ctypes.c_double)()
        self.cv_ref = None if cv_ref is None else np.ascontiguousarray(cv_ref, dtype=np.float64)
        p.cv_ref = _dptr(self.cv_ref) if self.cv_ref is not None else ctypes.POINTER(ctypes.c_double)()
        self.n_sched = None if n_sched is None else np.ascontiguousarray(n_sched, dtype=np.int32)
        p.n_sched = (self.n_sched.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)) if self.n_sched is not None
                     else ctypes.POINTER(ctypes.c_int32)())
        for i, c in enumerate(ck):
            p.ckpt[i] = int(c)
        self.p = p
        self.d, self.N, self.ckpt = d, N, ck

    def path(self, rep, T, replay=None, uroff=0.0, want_decisions=False):
        out = PathOut()
        dec = np.zeros(T, dtype=np.uint8) if want_decisions else None
        rp = None
        if replay is not None:
            replay = np.ascontiguousarray(replay, dtype=np.uint8)
            assert replay.shape[0] >= T
            rp = replay.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
        rc = lib().or_path(ctypes.byref(self.p), rep, T, rp, uroff, ctypes.byref(out),
                           dec.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)) if dec is not None else None)
        if rc:
            raise ValueError("or_path rejected the problem")
        return (out, dec) if want_decisions else out

    def run(self, R, T, r0=0):
        outs = (PathOut * R)()
        rc = lib().or_run_range(ctypes.byref(self.p), r0, r0 + R, T, outs)
        if rc:
            raise ValueError("or_run_range rejected the problem")
        return outs

    def reduce(self, outs, T):
        st = Stats()
        lib().or_reduce(ctypes.byref(self.p), T, outs, len(outs), ctypes.byref(st))
        return st

    def sample_gradient(self, rep, epoch, w):
        w = np.ascontiguousarray(w, dtype=np.float64)
        g, rbar, sw = (np.zeros(self.d) for _ in range(3))
        lib().or_sample_gradient(ctypes.byref(self.p), rep, epoch, _dptr(w), _dptr(g), _dptr(rbar),
                                 _dptr(sw))
        return g, rbar, sw

    def gradient_bound(self, rep, epoch, w, uroff):
        """(gradient, bound): the sample gradient at w and the rounding bound the replay rule of
        `path` applies there for a system with unit roundoff `uroff`."""
        w = np.ascontiguousarray(w, dtype=np.float64)
        g = np.zeros(self.d)
        b = ctypes.c_double()
        lib().or_sample_gradient_bound(ctypes.byref(self.p), rep, epoch, _dptr(w), uroff, _dptr(g), ctypes.byref(b))
        return g, b.value

    def draw_returns(self, rep, epoch):
        R = np.zeros((self.N, self.d))
        lib().or_draw_returns(ctypes.byref(self.p), rep, epoch, _dptr(R))
        return R

    def objective(self, w):
        w = np.ascontiguousarray(w, dtype=np.float64)
        return lib().or_objective(ctypes.byref(self.p), _dptr(w))


class WideOracle:
    """Algorithm 1 at the paper's experimental shape (many assets, diagonal Sigma): wide.c."""

    def __init__(self, mu, sigma, *, N, M=1, lam=0.5, w0=None, seed=0, instance=0, ckpt=(), gap_eps=1e-2,
                 n_sched=None):
        self.mu = np.ascontiguousarray(mu, dtype=np.float64)
        self.sigma = np.ascontiguousarray(sigma, dtype=np.float64)
        d = self.mu.shape[0]
        self.w0 = None if w0 is None else np.ascontiguousarray(w0, dtype=np.float64)
        ck = list(ckpt)
        if len(ck) > MAX_CKPT:
            raise ValueError("at most 8 checkpoints")
        p = WideProblem()
        p.d, p.N, p.M, p.instance, p.n_ckpt, p.seed = d, N, M, instance, len(ck), seed
        p.lam, p.gap_eps = lam, gap_eps
        p.mu, p.sigma = _dptr(self.mu), _dptr(self.sigma)
        p.w0 = _dptr(self.w0) if self.w0 is not None else ctypes.POINTER(ctypes.c_double)()
        for i, c in enumerate(ck):
            p.ckpt[i] = int(c)
        self.n_sched = None if n_sched is None else np.ascontiguousarray(n_sched, dtype=np.int32)
        p.n_sched = (self.n_sched.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)) if self.n_sched is not None
                     else ctypes.POINTER(ctypes.c_int32)())
        self.p = p
        self.d, self.N, self.M, self.ckpt = d, N, M, ck

    def path(self, rep, T, replay=None, uroff=0.0):
        """One replication: a dict of y, f_ckpt, cnt, wsum, tau (and its bound range), the replay
        counters, identity_err and the decisions taken."""
        cnt = np.zeros(self.d + 1, dtype=np.uint32)
        wsum = np.zeros(self.d, dtype=np.uint64)
        dec = np.zeros(T, dtype=np.uint32)
        out = WideOut()
        out.cnt = cnt.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))
        out.wsum = wsum.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))
        rp = None
        if replay is not None:
            replay = np.ascontiguousarray(replay, dtype=np.uint32)
            assert replay.shape[0] >= T
            rp = replay.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))
        rc = lib().or_wide_path(ctypes.byref(self.p), rep, T, rp, uroff, ctypes.byref(out),
                                dec.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)))
        if rc:
            raise ValueError("or_wide_path rejected the problem")
        return dict(y=out.y, f_ckpt=np.array(out.f_ckpt[:len(self.ckpt)]), cnt=cnt, wsum=wsum, tau=out.tau,
                    tau_lo=out.tau_lo, tau_hi=out.tau_hi, n_ambiguous=out.n_ambiguous,
                    n_replayed=out.n_replayed, n_mismatch=out.n_mismatch, first_mismatch=out.first_mismatch,
                    identity_err=out.identity_err, min_margin=out.min_margin, decisions=dec)

    def gradient(self, rep, epoch, w, uroff=0.0):
        w = np.ascontiguousarray(w, dtype=np.float64)
        g = np.zeros(self.d)
        b = ctypes.c_double(0.0)
        lib().or_wide_gradient(ctypes.byref(self.p), rep, epoch, _dptr(w), _dptr(g), uroff, ctypes.byref(b))
        return g, b.value

    def objective(self, w):
        w = np.ascontiguousarray(w, dtype=np.float64)
        return lib().or_wide_objective(ctypes.byref(self.p), _dptr(w))


class NvOracle:
    """Algorithm 2, the multi-product newsvendor with one resource row (newsvendor.c)."""

    FIELDS = ("mu", "sigma", "k", "h", "v", "c")

    def __init__(self, inst: dict, *, S, M=1, x0=None, seed=0, instance=0, ckpt=(), gap_eps=1e-2):
        self.arrays = {f: np.ascontiguousarray(inst[f], dtype=np.float64) for f in self.FIELDS}
        n = self.arrays["mu"].shape[0]
        self.x0 = None if x0 is None else np.ascontiguousarray(x0, dtype=np.float64)
        ck = list(ckpt)
        if len(ck) > MAX_CKPT:
            raise ValueError("at most 8 checkpoints")
        p = NvProblem()
        p.n, p.S, p.M, p.instance, p.n_ckpt, p.seed = n, S, M, instance, len(ck), seed
        p.C, p.gap_eps = float(inst["C"]), gap_eps
        for f in self.FIELDS:
            setattr(p, f, _dptr(self.arrays[f]))
        p.x0 = _dptr(self.x0) if self.x0 is not None else ctypes.POINTER(ctypes.c_double)()
        for i, c in enumerate(ck):
            p.ckpt[i] = int(c)
        self.p = p
        self.n, self.S, self.M, self.ckpt, self.C = n, S, M, ck, float(inst["C"])

    def path(self, rep, T, replay=None, uroff=0.0):
        cnt = np.zeros(self.n + 1, dtype=np.uint32)
        wsum = np.zeros(self.n, dtype=np.uint64)
        dec = np.zeros(T, dtype=np.uint32)
        out = NvOut()
        out.cnt = cnt.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))
        out.wsum = wsum.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))
        rp = None
        if replay is not None:
            replay = np.ascontiguousarray(replay, dtype=np.uint32)
            assert replay.shape[0] >= T
            rp = replay.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))
        rc = lib().or_nv_path(ctypes.byref(self.p), rep, T, rp, uroff, ctypes.byref(out),
                              dec.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)))
        if rc:
            raise ValueError("or_nv_path rejected the problem")
        return dict(y=out.y, f_ckpt=np.array(out.f_ckpt[:len(self.ckpt)]), cnt=cnt, wsum=wsum, tau=out.tau,
                    tau_lo=out.tau_lo, tau_hi=out.tau_hi, n_ambiguous=out.n_ambiguous,
                    n_replayed=out.n_replayed, n_mismatch=out.n_mismatch, first_mismatch=out.first_mismatch,
                    identity_err=out.identity_err, min_margin=out.min_margin, decisions=dec)

    def gradient(self, rep, epoch, x):
        x = np.ascontiguousarray(x, dtype=np.float64)
        g = np.zeros(self.n)
        cnt = np.zeros(self.n, dtype=np.uint32)
        lib().or_nv_gradient(ctypes.byref(self.p), rep, epoch, _dptr(x), _dptr(g),
                             cnt.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)))
        return g, cnt

    def cost(self, x):
        x = np.ascontiguousarray(x, dtype=np.float64)
        return lib().or_nv_cost(ctypes.byref(self.p), _dptr(x))


class NvLpOracle:
    """Algorithm 2 over Eq. (7)'s general constraint set X = {A x <= C, x >= 0} with M resource rows.
    Test infrastructure: Eq. (9)'s gradient comes from the C oracle's demand samples (or_nv_gradient,
    with its binary32 uncertainty or_nv_gradient_bound). The linear subproblem min_{s in X} s'g is
    solved by scipy's linprog (HiGHS), a library LP primitive. The step is 2/(t+2) and the update
    x + gamma (s - x), each operation rounded on its own (numpy does not fuse them). Eq. (6) comes
    from or_nv_cost."""

    FIELDS = ("mu", "sigma", "k", "h", "v")

    def __init__(self, inst: dict, A, C, *, S, M=1, x0=None, seed=0, instance=0, ckpt=(), gap_eps=1e-2):
        self.arrays = {f: np.ascontiguousarray(inst[f], dtype=np.float64) for f in self.FIELDS}
        n = self.arrays["mu"].shape[0]
        self.arrays["c"] = np.ones(n)             # the single-row fields are not used here
        self.A = np.ascontiguousarray(A, dtype=np.float64).reshape(-1, n)
        self.Cv = np.ascontiguousarray(C, dtype=np.float64).reshape(-1)
        self.x0 = np.zeros(n) if x0 is None else np.ascontiguousarray(x0, dtype=np.float64)
        ck = list(ckpt)
        if len(ck) > MAX_CKPT:
            raise ValueError("at most 8 checkpoints")
        p = NvProblem()
        p.n, p.S, p.M, p.instance, p.n_ckpt, p.seed = n, S, M, instance, len(ck), seed
        p.C, p.gap_eps = 1.0, gap_eps
        for f in self.FIELDS + ("c",):
            setattr(p, f, _dptr(self.arrays[f]))
        p.x0 = ctypes.POINTER(ctypes.c_double)()
        for i, c in enumerate(ck):
            p.ckpt[i] = int(c)
        self.p = p
        self.n, self.S, self.M, self.ckpt, self.gap_eps = n, S, M, ck, gap_eps

    def gradient(self, rep, epoch, x):
        x = np.ascontiguousarray(x, dtype=np.float64)
        g = np.zeros(self.n)
        cnt = np.zeros(self.n, dtype=np.uint32)
        lib().or_nv_gradient(ctypes.byref(self.p), rep, epoch, _dptr(x), _dptr(g),
                             cnt.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)))
        return g, cnt

    def bound(self, rep, epoch, x, u):
        x = np.ascontiguousarray(x, dtype=np.float64)
        e = np.zeros(self.n)
        lib().or_nv_gradient_bound(ctypes.byref(self.p), rep, epoch, _dptr(x), u, _dptr(e))
        return e

    def cost(self, x):
        x = np.ascontiguousarray(x, dtype=np.float64)
        return lib().or_nv_cost(ctypes.byref(self.p), _dptr(x))

    def lp(self, g):
        """(min s'g over X, a minimiser) by HiGHS with tight tolerances."""
        from scipy.optimize import linprog
        res = linprog(g, A_ub=self.A, b_ub=self.Cv, bounds=(0, None), method="highs",
                      options=dict(primal_feasibility_tolerance=1e-10, dual_feasibility_tolerance=1e-10))
        if res.status != 0:
            raise RuntimeError(f"linprog: {res.message}")
        return float(res.fun), np.asarray(res.x, dtype=np.float64)

    def path(self, rep, T, replay=None, uroff=0.0, rtol=1e-9):
        """One replication. With replay = (basis [T][M], value [T][M]) of a device run, each iteration's
        recorded vertex is checked and then followed. It must be feasible, and its value under this
        oracle's gradient must lie within the bound of the LP optimum: the gradient's uncertainty
        (uroff) over the vertex and over the optimiser, plus rtol of the values. Without replay the
        oracle follows its own LP solution."""
        n, A, Cv = self.n, self.A, self.Cv
        x = self.x0.copy()
        f_ckpt, ck = [], 0
        tau_lo = tau_hi = tau = None
        n_mismatch, first_mismatch, worst = 0, -1, 0.0
        for t in range(T):
            epoch = t // self.M
            g, _ = self.gradient(rep, epoch, x)
            e = self.bound(rep, epoch, x, uroff) if uroff > 0 else np.zeros(n)
            vstar, sstar = self.lp(g)
            if replay is not None:
                basis, value = replay
                s = np.zeros(n)
                for b, v in zip(basis[t], value[t]):
                    if b < n:
                        s[b] = v
                feasible = bool(np.all(s >= 0.0) and np.all(A @ s <= Cv * (1.0 + rtol) + 1e-300))
                val = float(g @ s)
                slack = float(e @ (s + sstar)) + rtol * (abs(vstar) + float(np.abs(g) @ (s + sstar)))
                excess = (val - vstar) / max(slack, 1e-300)
                worst = max(worst, excess)
                if not (feasible and vstar - slack <= val <= vstar + slack):
                    n_mismatch += 1
                    if first_mismatch < 0:
                        first_mismatch = t
            else:
                s = sstar
            gap = float(g @ x) - float(g @ s)
            gap_bound = float(e @ (x + s)) + rtol * float(np.abs(g) @ (x + s))
            if tau is None and gap <= self.gap_eps:
                tau = t
            if tau_lo is None and gap <= self.gap_eps + gap_bound:
                tau_lo = t
            if tau_hi is None and gap <= self.gap_eps - gap_bound:
                tau_hi = t
            gamma = 2.0 / (t + 2.0)
            x = x + gamma * (s - x)
            while ck < len(self.ckpt) and self.ckpt[ck] == t + 1:
                f_ckpt.append(self.cost(x))
                ck += 1
        none = TAU_NONE
        return dict(y=self.cost(x), f_ckpt=np.array(f_ckpt), x=x, tau=none if tau is None else tau,
                    tau_lo=none if tau_lo is None else tau_lo, tau_hi=none if tau_hi is None else tau_hi,
                    n_mismatch=n_mismatch, first_mismatch=first_mismatch, worst_excess=worst)


class SqnOracle:
    """Algorithms 3-4, stochastic quasi-Newton for the logistic loss (sqn.c)."""

    DOMAIN_GRAD, DOMAIN_HESS = 5, 6

    def __init__(self, X, z, *, L=10, M=25, b=50, bH=300, beta=2.0, seed=0, instance=0, ckpt=(), pairs_fp32=False):
        self.X = np.ascontiguousarray(X, dtype=np.uint8)
        self.z = np.ascontiguousarray(z, dtype=np.uint8)
        N, n = self.X.shape
        ck = list(ckpt)
        p = SqnProblem()
        p.n, p.N, p.L, p.M, p.b, p.bH, p.beta = n, N, L, M, b, bH, beta
        p.instance, p.n_ckpt, p.seed = instance, len(ck), seed
        p.X = self.X.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
        p.z = self.z.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
        for i, c in enumerate(ck):
            p.ckpt[i] = int(c)
        p.pairs_fp32 = 1 if pairs_fp32 else 0
        self.p, self.n, self.N, self.ckpt = p, n, N, ck

    def indices(self, rep, k, domain, count):
        idx = np.zeros(count, dtype=np.uint32)
        lib().or_sqn_indices(ctypes.byref(self.p), rep, k, domain, count,
                             idx.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)))
        return idx

    def loss(self, w):
        w = np.ascontiguousarray(w, dtype=np.float64)
        return lib().or_sqn_loss(ctypes.byref(self.p), _dptr(w))

    def gradient(self, idx, w):
        idx = np.ascontiguousarray(idx, dtype=np.uint32)
        w = np.ascontiguousarray(w, dtype=np.float64)
        g = np.zeros(self.n)
        lib().or_sqn_gradient(ctypes.byref(self.p), idx.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
                              len(idx), _dptr(w), _dptr(g))
        return g

    def hessian_vector(self, idx, w, v):
        idx = np.ascontiguousarray(idx, dtype=np.uint32)
        w = np.ascontiguousarray(w, dtype=np.float64)
        v = np.ascontiguousarray(v, dtype=np.float64)
        out = np.zeros(self.n)
        lib().or_sqn_hessian_vector(ctypes.byref(self.p), idx.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
                                    len(idx), _dptr(w), _dptr(v), _dptr(out))
        return out

    @staticmethod
    def hessian_approx(S, Y):
        S = np.ascontiguousarray(S, dtype=np.float64)
        Y = np.ascontiguousarray(Y, dtype=np.float64)
        m, n = S.shape
        H = np.zeros((n, n))
        lib().or_sqn_hessian_approx(n, m, _dptr(S), _dptr(Y), _dptr(H))
        return H

    def run(self, rep, K):
        w = np.zeros(self.n)
        out = SqnOut()
        out.w = _dptr(w)
        if lib().or_sqn_run(ctypes.byref(self.p), rep, K, ctypes.byref(out)):
            raise ValueError("or_sqn_run rejected the problem")
        return dict(F=out.F, F_ckpt=np.array(out.F_ckpt[:len(self.ckpt)]), w=w, pairs=out.pairs)


def philox(ctr, key):
    c = (ctypes.c_uint32 * 4)(*[int(x) & 0xFFFFFFFF for x in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(x) & 0xFFFFFFFF for x in key])
    o = (ctypes.c_uint32 * 4)()
    lib().or_philox4x32_10(c, k, o)
    return [int(x) for x in o]


def uniform(x):
    return lib().or_uniform(int(x) & 0xFFFFFFFF)


def normals(seed, domain, instance, rep, epoch, q0, n):
    out = np.zeros(n, dtype=np.float64)
    lib().or_normals(seed, domain, instance, rep, epoch, q0, n, _dptr(out))
    return out


def path_arrays(outs, d, n_ckpt):
    """Per-path outputs as numpy arrays (Y, f_ckpt, cnt, wsum, tau)."""
    R = len(outs)
    Y = np.array([o.y for o in outs])
    F = np.array([[o.f_ckpt[c] for c in range(n_ckpt)] for o in outs]).reshape(R, n_ckpt)
    cnt = np.array([[o.cnt[j] for j in range(d + 1)] for o in outs], dtype=np.uint64)
    wsum = np.array([[o.wsum[j] for j in range(d)] for o in outs], dtype=np.uint64)
    tau = np.array([o.tau for o in outs], dtype=np.uint64)
    return Y, F, cnt, wsum, tau


# ---- control-variate pieces ----------------------------------------------------------------


def _arr(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def cv_pick_probs(b, s):
    """(p, sum): probabilities of the reference decision, p[0] the origin, p[j+1] vertex e_j."""
    b, s = _arr(b), _arr(s)
    p = np.zeros(b.shape[0] + 1)
    tot = lib().or_cv_pick_probs(b.shape[0], _dptr(b), _dptr(s), _dptr(p))
    return p, tot


def cv_weights(T: int, M: int):
    """(S2, S4, S1, S11, S12): sums over epochs of W2_e, W2_e^2, W1_e, W1_e^2, W1_e W2_e."""
    w = np.zeros(5)
    lib().or_cv_weights(T, M, _dptr(w))
    return tuple(w)


class CvLaw:
    """The features' law for a problem (diagonal L) with reference gradient cv_ref and T iterations."""

    def __init__(self, P: OracleProblem, T: int):
        if P.cv_ref is None:
            raise ValueError("the features' law needs a reference gradient (cv_ref)")
        sig = np.diag(P.chol).copy()
        self.P, self.T, self.d = P, T, P.d
        self.probs, self.total = cv_pick_probs(P.cv_ref, sig / np.sqrt(P.N))
        self.w = np.array(cv_weights(T, P.p.M))
        self.S2, self.S4, self.S1, self.S11, self.S12 = self.w
        self.top = lib().or_cv_top(self.d, _dptr(self.probs))

    def standardize(self, count, count1):
        x = np.zeros(self.d + 2)
        c, c1 = _arr(count), _arr(count1)
        lib().or_cv_features(self.d, _dptr(self.probs), _dptr(self.w), _dptr(c), _dptr(c1), _dptr(x))
        return x

    def path_features(self, o):
        return self.standardize([o.cv_count[c] for c in range(self.d + 1)],
                                [o.cv_count1[c] for c in range(self.d + 1)])

    def aux(self, k0: int, n: int):
        """Draws k0 .. k0+n-1 from the exact law: (standardized (n, d+2), counts (n, d+1), counts1 (n, d+1))."""
        X = np.zeros((n, self.d + 2))
        C = np.zeros((n, self.d + 1))
        C1 = np.zeros((n, self.d + 1))
        cnt, cnt1 = np.zeros(self.d + 1), np.zeros(self.d + 1)
        for i in range(n):
            lib().or_cv_aux(ctypes.byref(self.P.p), self.T, _dptr(self.probs), k0 + i, _dptr(cnt), _dptr(cnt1))
            C[i], C1[i] = cnt, cnt1
            X[i] = self.standardize(cnt, cnt1)
        return X, C, C1


def bf16(v: float) -> float:
    return lib().or_bf16(float(v))


def mlp_param_count(F: int) -> int:
    return lib().or_mlp_param_count(F)


def mlp_forward(theta, F: int, x, quantize: bool = False):
    theta, x = _arr(theta), _arr(x).reshape(-1, F)
    out = np.zeros(x.shape[0])
    lib().or_mlp_forward(_dptr(theta), F, _dptr(x), x.shape[0], int(quantize), _dptr(out))
    return out


def mlp_grad(theta, F: int, x, y, quantize: bool = False):
    """(loss, gradient) of the mean squared error of h over the rows of x against y."""
    theta, x, y = _arr(theta), _arr(x).reshape(-1, F), _arr(y)
    g = np.zeros_like(theta)
    loss = lib().or_mlp_grad(_dptr(theta), F, _dptr(x), _dptr(y), x.shape[0], int(quantize), _dptr(g))
    return loss, g


def cv_beta(Y, H):
    Y, H = _arr(Y), _arr(H)
    b, r = ctypes.c_double(), ctypes.c_double()
    lib().or_cv_beta(_dptr(Y), _dptr(H), Y.shape[0], ctypes.byref(b), ctypes.byref(r))
    return b.value, r.value


def cv_estimate(Y, H, Haux, beta: float) -> CvStats:
    Y, H, Haux = _arr(Y), _arr(H), _arr(Haux)
    st = CvStats()
    lib().or_cv_estimate(_dptr(Y), _dptr(H), Y.shape[0], _dptr(Haux), Haux.shape[0], beta, ctypes.byref(st))
    return st
