"""Accuracy of the FP64 device math the kernels use in place of library calls:
sin and cos by Cody-Waite reduction modulo pi/2 and Taylor series on
|r| <= pi/4, sqrt and 1/sqrt and 1/x by Newton-Raphson refinement of the
hardware estimates.  Evaluated on the GPU through the probe library and
compared with NumPy (IEEE double, correctly rounded or within an ulp)."""
import ctypes
import os

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def probe():
    path = os.path.join(ROOT, "paper_2112_06316_amd", "libifgf_probe.so")
    if not os.path.exists(path):
        pytest.fail("libifgf_probe.so is not built")
    lib = ctypes.CDLL(path)
    lib.ifgf_probe_math64.restype = ctypes.c_int
    lib.ifgf_probe_math64.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p]
    return lib


def test_fp64_math_against_numpy():
    rng = np.random.default_rng(71)
    x = np.concatenate([
        rng.uniform(-4.0, 4.0, 200_000),          # leaf phases
        rng.uniform(-2000.0, 2000.0, 200_000),    # target phases k r
        rng.uniform(-1.0e5, 1.0e5, 50_000),
        rng.uniform(-1.0e7, 1.0e7, 1_000),        # past 2^20: the library path
        np.pi / 4 * np.arange(-64, 65),           # quadrant boundaries
        [1e-8, -1e-8, 1e-300, 3e-5, 0.5, 1.0, 2.0],
    ])
    x = x[x != 0.0]
    n = len(x)
    xd = torch.from_numpy(x).cuda()
    out = torch.empty(5 * n, dtype=torch.float64, device="cuda")
    st = probe().ifgf_probe_math64(xd.data_ptr(), out.data_ptr(), n, torch.cuda.current_stream().cuda_stream)
    assert st == 0
    torch.cuda.synchronize()
    o = out.cpu().numpy().reshape(n, 5)
    es = np.abs(o[:, 0] - np.sin(x)).max()
    ec = np.abs(o[:, 1] - np.cos(x)).max()
    a = np.abs(x)
    eq = (np.abs(o[:, 2] - np.sqrt(a)) / np.sqrt(a)).max()
    er = (np.abs(o[:, 3] - 1.0 / np.sqrt(a)) * np.sqrt(a)).max()
    ei = (np.abs(o[:, 4] - 1.0 / x) * a).max()
    print(f"sin {es:.2e}, cos {ec:.2e} (absolute); sqrt {eq:.2e}, 1/sqrt {er:.2e}, 1/x {ei:.2e} (relative)")
    assert es <= 1e-15 and ec <= 1e-15
    assert eq <= 4.5e-16 and er <= 4.5e-16 and ei <= 4.5e-16
