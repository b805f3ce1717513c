"""GPU test of the allocation-free batch apply (ifgf_batch_apply_noalloc).

The entry point runs the same ragged-batch launch as ifgf_batch_apply with
the launch's completion counters in the library's fixed per-device array.
Called through the C ABI twice in a row - a batch of three geometries, then
a smaller batch of two, so the second call starts from the counters the
first one left - each result must equal ifgf_batch_apply's on the same
inputs (same kernels and work items: FP32 to 1e-6, FP64 to 1e-13 relative),
and the calls must leave the device's free memory unchanged.
"""
import ctypes

import numpy as np
import pytest
import torch

from paper_2112_06316_amd import Batch, Plan, inputs
from paper_2112_06316_amd import _lib as L

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def log(msg):
    print(msg, flush=True)


def _batch(sizes, precision):
    geoms = inputs.ragged_batch(sizes)
    plans = [Plan(g["points"], g["normals"], g["weights"], g["k"], g["eta"], precision=precision,
                  leaf_h_lambda=0.5) for g in geoms]
    cdt = torch.complex64 if precision == "fp32" else torch.complex128
    sig = [torch.from_numpy(inputs.random_density(g["n"], seed=g["seed"])).to(DEV).to(cdt) for g in geoms]
    return plans, Batch(plans), sig


def _noalloc(lib, bt, sig, outs, dtype):
    sp = (ctypes.c_void_p * len(sig))(*[s.data_ptr() for s in sig])
    up = (ctypes.c_void_p * len(outs))(*[u.data_ptr() for u in outs])
    return lib.ifgf_batch_apply_noalloc(bt._h, sp, up, dtype, torch.cuda.current_stream().cuda_stream)


@pytest.mark.parametrize("precision,tol", [("fp32", 1e-6), ("fp64", 1e-13)])
def test_noalloc_batch_equals_batch_apply(precision, tol):
    lib = L.load()
    dtype = L.C64 if precision == "fp32" else L.C128
    for call, sizes in enumerate(((32, 48, 64), (24, 40))):
        log(f"case noalloc batch {precision} call {call}: n_b = {sizes}")
        plans, bt, sig = _batch(sizes, precision)
        ref = [u.cpu().numpy() for u in bt.apply(sig)]
        outs = [torch.full_like(s, complex(np.nan, np.nan)) for s in sig]
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        st = _noalloc(lib, bt, sig, outs, dtype)
        torch.cuda.synchronize()
        free1 = torch.cuda.mem_get_info()[0]
        assert st == L.OK, L.load().ifgf_last_error()
        assert free1 == free0, (free0, free1)
        for g, (o, r) in enumerate(zip(outs, ref)):
            o = o.cpu().numpy()
            e = float(np.linalg.norm(o - r) / np.linalg.norm(r))
            log(f"  geometry {g}: N = {len(r)}, rel diff {e:.2e}, bitwise equal {bool(np.array_equal(o, r))}")
            assert e <= tol, (call, g, e)
        assert bt.check() == 0
        assert all(p.check() == 0 for p in plans)


def test_noalloc_batch_argument_errors():
    lib = L.load()
    plans, bt, sig = _batch((24,), "fp32")
    outs = [torch.empty_like(s) for s in sig]
    assert _noalloc(lib, bt, sig, sig, L.C64) == L.EINVAL      # output aliases the input
    assert _noalloc(lib, bt, sig, outs, 7) == L.EINVAL         # bad dtype
    sp = (ctypes.c_void_p * 1)(sig[0].data_ptr())
    assert lib.ifgf_batch_apply_noalloc(None, sp, sp, L.C64, None) == L.EINVAL
    assert _noalloc(lib, bt, sig, outs, L.C64) == L.OK
    torch.cuda.synchronize()
