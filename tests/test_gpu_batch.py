"""GPU tests of the ragged multi-geometry batch (one launch for many plans).

A batch apply must give, for every geometry, what ifgf_apply gives on that
plan alone: the same stages run on the same plan data, only scheduled as work
items of one launch.  The leaf, coefficient, upward-pass and target items sum
in the same order as the separate kernels; the near-field item splits its
source loop over a different number of threads, so results agree to rounding
(FP32: 1e-5 relative, FP64: 1e-12) rather than bitwise.  Against the oracle's
direct sum each geometry is within the IFGF tolerance.
"""
import ctypes

import numpy as np
import pytest
import torch

from oracle import direct
from paper_2112_06316_amd import Batch, Plan, inputs
from paper_2112_06316_amd import _lib as L

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def log(msg):
    print(msg, flush=True)


def to_dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def make_plans(geoms, precision, **kw):
    return [Plan(g["points"], g["normals"], g["weights"], g["k"], g["eta"], precision=precision,
                 leaf_h_lambda=0.5, **kw) for g in geoms]


@pytest.mark.parametrize("precision,tol", [("fp32", 1e-5), ("fp64", 1e-12)])
def test_ragged_batch_equals_separate_applies(precision, tol):
    geoms = inputs.ragged_batch()
    log(f"case ragged batch {precision}: N = {[g['n'] for g in geoms]}")
    plans = make_plans(geoms, precision)
    sig = [to_dev(inputs.random_density(g["n"], seed=g["seed"])) for g in geoms]
    if precision == "fp32":
        sig = [s.to(torch.complex64) for s in sig]
    sep = [p.apply(s).cpu().numpy() for p, s in zip(plans, sig)]
    b = Batch(plans)
    log(f"  queue {b.info()}")
    for rep in range(2):   # the second apply reuses the queue and its counters
        out = [u.cpu().numpy() for u in b.apply(sig)]
        es = []
        for g, (o, r) in enumerate(zip(out, sep)):
            e = np.abs(o - r).max() / np.abs(r).max()
            es.append(e)
            assert e <= tol, (rep, g, e)
        log(f"  apply {rep}: max rel diff {max(es):.2e}, bitwise equal {all(np.array_equal(o, r) for o, r in zip(out, sep))}")
    assert b.check() == 0
    assert all(p.check() == 0 for p in plans)


def test_ragged_batch_accuracy_against_direct_sum():
    geoms = inputs.ragged_batch()
    plans = make_plans(geoms, "fp32")
    sig = [inputs.random_density(g["n"], seed=g["seed"]) for g in geoms]
    out = [u.cpu().numpy() for u in Batch(plans).apply([to_dev(s) for s in sig])]
    for g, (geo, s, o) in enumerate(zip(geoms, sig, out)):
        tg = inputs.sample_targets(geo["n"], 256, seed=geo["seed"] + 100)
        ref = direct.apply_c(geo["points"], geo["normals"], geo["weights"], geo["k"], geo["eta"], s, targets=tg)
        err = rel(o[tg], ref)
        log(f"  geometry {g}: N={geo['n']} D={plans[g].stats()['depth']} rel err {err:.6e}")
        assert err < 1e-4


def test_mixed_batch_constant_kernel_and_shallow_tree():
    # constant kernel: exact sum_{j != i} w_j sigma_j; D <= 2: everything near, exact direct sum
    p1, n1, w1 = inputs.cubed_sphere(24)
    p2, n2, w2 = inputs.ellipsoid(10, (0.5, 0.375, 0.25))
    p3, n3, w3 = inputs.cubed_sphere(20)
    k = 6 * np.pi
    plans = [Plan(p1, n1, w1, k, k, depth=5, kernel="constant", precision="fp64"),
             Plan(p2, n2, w2, k, 2.0, depth=2, precision="fp64"),
             Plan(p3, n3, w3, k, k, depth=4, precision="fp64")]
    s = [inputs.random_density(len(p), seed=40 + i) for i, p in enumerate((p1, p2, p3))]
    out = [u.cpu().numpy() for u in Batch(plans).apply([to_dev(x) for x in s])]
    ref0 = w1 * s[0]
    ref0 = ref0.sum() - ref0
    assert np.abs(out[0] - ref0).max() <= 1e-11 * np.abs(w1 * s[0]).sum()
    ref1 = direct.apply_c(p2, n2, w2, k, 2.0, s[1])
    assert np.abs(out[1] - ref1).max() <= 1e-12 * np.abs(ref1).max()
    ref2 = plans[2].apply(to_dev(s[2])).cpu().numpy()
    assert np.abs(out[2] - ref2).max() <= 1e-12 * np.abs(ref2).max()


def test_single_plan_batch_and_order_p35():
    p, nr, w = inputs.cubed_sphere(32)
    k = 8 * np.pi
    plan = Plan(p, nr, w, k, k, depth=4, precision="fp32", p_s=3, p_ang=5, ns0=1, nc0=2)
    s = to_dev(inputs.random_density(len(p), seed=50)).to(torch.complex64)
    ref = plan.apply(s).cpu().numpy()
    out = Batch([plan]).apply([s])[0].cpu().numpy()
    assert np.abs(out - ref).max() <= 1e-5 * np.abs(ref).max()


def test_batch_argument_errors():
    p, nr, w = inputs.cubed_sphere(8)
    a = Plan(p, nr, w, 5.0, 5.0, depth=3, precision="fp32")
    b = Plan(p, nr, w, 5.0, 5.0, depth=3, precision="fp64")
    c = Plan(p, nr, w, 5.0, 5.0, depth=3, precision="fp32", p_s=3, p_ang=5)
    for plans in ([a, b], [a, c], [a, a]):
        with pytest.raises(L.IFGFError) as e:
            Batch(plans)
        assert e.value.status == L.EINVAL
    lib = L.load()
    h = ctypes.c_void_p()
    assert lib.ifgf_batch_create(ctypes.byref(h), 0, None) == L.EINVAL
    hs = (ctypes.c_void_p * 65)(*([a._h] * 65))
    assert lib.ifgf_batch_create(ctypes.byref(h), 65, hs) == L.EINVAL
    bt = Batch([a])
    s = to_dev(inputs.random_density(len(p), seed=51))
    with pytest.raises(ValueError):
        bt.apply([s, s])
    with pytest.raises(ValueError):    # the binding rejects an output aliasing an input
        bt.apply([s], outs=[s])
    # and so does the library itself, called through the C ABI
    sp = (ctypes.c_void_p * 1)(s.data_ptr())
    st = lib.ifgf_batch_apply(bt._h, sp, sp, L.C128, torch.cuda.current_stream().cuda_stream)
    assert st == L.EINVAL


def test_bounded_wait_returns_and_flags():
    # With a poll limit of 0 an item whose inputs are not complete goes ahead
    # at once; the launch still ends and either the flag is raised or (every
    # input happened to be ready) the results are the normal ones.
    geoms = inputs.ragged_batch((32, 48, 64))
    plans = make_plans(geoms, "fp32")
    sig = [to_dev(inputs.random_density(g["n"], seed=g["seed"])).to(torch.complex64) for g in geoms]
    ref = [p.apply(s).cpu().numpy() for p, s in zip(plans, sig)]
    bt = Batch(plans)
    bt.set_spin_limit(0)
    out = [u.cpu().numpy() for u in bt.apply(sig)]
    torch.cuda.synchronize()
    flags = bt.check()
    log(f"  flags with poll limit 0: {flags}")
    if not flags & 1:
        for o, r in zip(out, ref):
            assert np.abs(o - r).max() <= 1e-5 * np.abs(r).max()
    b2 = Batch(plans)   # a fresh batch with the default limit is exact again
    out2 = [u.cpu().numpy() for u in b2.apply(sig)]
    assert b2.check() == 0
    for o, r in zip(out2, ref):
        assert np.abs(o - r).max() <= 1e-5 * np.abs(r).max()
