"""GPU tests of the formulation autotuner (ifgf_plan_autotune).

The tuner only chooses among formulations that compute the same operator,
so a tuned plan's apply must equal the untuned plan's to rounding (and stay
within the IFGF tolerance of the direct sum); it reports a measurement for
every candidate it ran and refuses plans a batch points into.
"""
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


@pytest.mark.parametrize("precision,tol", [("fp32", 2e-6), ("fp64", 1e-12)])
def test_autotuned_plan_computes_the_same_operator(precision, tol):
    wl = inputs.workload("sphere16")                          # N = 98,304, D = 6
    p, nr, w = inputs.build_surface(wl)
    k = wl["k"]
    sig = inputs.random_density(len(p), seed=61)
    s = torch.from_numpy(sig).to(DEV)
    if precision == "fp32":
        s = s.to(torch.complex64)
    ref_plan = Plan(p, nr, w, k, k, depth=wl["depth"], precision=precision)
    u0 = ref_plan.apply(s).cpu().numpy()
    plan = Plan(p, nr, w, k, k, depth=wl["depth"], precision=precision)
    rep = plan.autotune(reps=2)
    log(f"case autotune {precision}: {rep}")
    assert sorted(rep["prop"]) == [3, 4, 5]
    for d, e in rep["prop"].items():
        assert e["choice"] in e["ms"] and all(v > 0 for v in e["ms"].values())
        assert "node" in e["ms"]
        assert plan.stats()["prop_kernel"][d + 1] == {"node": "node", "pairs": "pairs"}.get(e["choice"], "cone")
    assert rep["targets"] in ("rows", "wave", "pairs")
    assert rep["targets"] in rep["targets_ms"] and set(rep["targets_ms"]) == {"rows", "wave", "pairs"}
    u1 = plan.apply(s).cpu().numpy()
    assert np.linalg.norm(u1 - u0) / np.linalg.norm(u0) <= tol
    tg = inputs.sample_targets(len(p), 256, seed=62)
    ref = direct.apply_c(p, nr, w, k, k, sig, targets=tg)
    assert np.linalg.norm(u1[tg] - ref) / np.linalg.norm(ref) < 1e-4
    assert plan.check() == 0


def test_autotune_refuses_a_batched_plan():
    p, nr, w = inputs.cubed_sphere(24)
    plan = Plan(p, nr, w, 8 * np.pi, 8 * np.pi, depth=4)
    b = Batch([plan])
    with pytest.raises(L.IFGFError) as e:
        plan.autotune(reps=1)
    assert e.value.status == L.EBUSY
    b.close()
    plan.autotune(reps=1)
    with pytest.raises(L.IFGFError) as e:
        plan.autotune(reps=0)
    assert e.value.status == L.EINVAL
