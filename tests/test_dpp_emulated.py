"""The wavefront reductions on DPP lane moves and lane swaps (csrc/wave_dpp.hpp), in the CPU
emulation of the device, against the xor shuffle butterfly they replace: sums (binary32 over 32 and
64 lanes, binary64 over 64), (value, index) minima (lowest index among equal values; binary32 over
32 and 64 lanes, binary64 over 64) and the integer sums over groups of P lanes. The kernels rely on
the two giving the same bits (the same lane pairing at every level), so the values are chosen to
make the order of the additions visible: magnitudes spread over many binades, signs mixed, and
repeated values so that ties decide the index. The emulation models each DPP control and lane swap
by its lane mapping; the GPU parity tests check the kernels that use them on the device.
"""
import ctypes
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.fixture(scope="module")
def emu():
    gxx = shutil.which("g++")
    if not gxx:
        pytest.skip("g++ not available")
    d = tempfile.mkdtemp(prefix="dpp_emu_")
    so = os.path.join(d, "libemudpp.so")
    subprocess.check_call([gxx, "-std=c++20", "-O2", "-fPIC", "-shared", "-I", os.path.join(HERE, "emu", "shim"),
                           "-I", os.path.join(ROOT, "include"), "-o", so, os.path.join(HERE, "emu", "emu_dpp.cpp"),
                           "-lpthread"])
    L = ctypes.CDLL(so)
    L.emu_dpp_case.argtypes = [ctypes.c_void_p] * 4
    L.emu_dpp_case.restype = ctypes.c_int
    yield L
    shutil.rmtree(d, ignore_errors=True)


def _case(rng, kind):
    if kind == "spread":
        xf = (rng.standard_normal(64) * 2.0 ** rng.integers(-20, 20, 64)).astype(np.float32)
    elif kind == "ties":
        xf = rng.choice(np.array([-1.5, -1.5, 0.25, 3.0], np.float32), 64)
    elif kind == "inf":
        xf = rng.standard_normal(64).astype(np.float32)
        xf[rng.random(64) < 0.5] = np.inf
    else:
        xf = np.full(64, np.inf, np.float32)
    xd = xf.astype(np.float64) * (1.0 + 2.0 ** -40 * rng.standard_normal(64))
    if kind == "ties":
        xd = xf.astype(np.float64)
    jx = rng.permutation(64).astype(np.uint32) * 3 + 1
    if kind == "all_inf":
        jx[:] = 0xFFFFFFFF
    cx = rng.integers(0, 1 << 20, 64).astype(np.uint32)
    return xf, xd, jx, cx


@pytest.mark.parametrize("kind", ["spread", "ties", "inf", "all_inf"])
def test_dpp_reductions_match_butterfly(emu, kind):
    rng = np.random.default_rng(17)
    for _ in range(20):
        xf, xd, jx, cx = _case(rng, kind)
        bad = emu.emu_dpp_case(xf.ctypes.data, xd.ctypes.data, jx.ctypes.data, cx.ctypes.data)
        assert bad == 0, (kind, bad)


def test_dpp_sum_order_is_visible():
    """The check can fail: with a sequential sum in place of the butterfly the spread values give
    other bits in most cases, so equal bits above are not an accident of the data."""
    rng = np.random.default_rng(5)
    differ = 0
    for _ in range(20):
        xf, _, _, _ = _case(rng, "spread")
        seq = np.float32(0)
        for v in xf:
            seq = np.float32(seq + v)
        tree = xf.copy()
        m = 1
        while m < 64:
            tree = (tree + tree[np.arange(64) ^ m]).astype(np.float32)
            m <<= 1
        differ += int(seq != tree[0])
    assert differ >= 5, differ
