"""GPU tests of the batched right-hand-side path (MFMA contraction over
groups of 16 RHS in FP32 mode): an R-RHS apply equals R single applies, and
plane-wave densities (the batched workload of the paper's incidences,
Sec. 5, eq. PlaneWave) agree with the direct sum."""
import numpy as np
import pytest
import torch

from oracle import direct
from paper_2112_06316_amd import Plan, inputs

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def log(msg):
    print(msg, flush=True)


def to_dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


@pytest.mark.parametrize("R", [16, 32])
@pytest.mark.parametrize("opts", [dict(), dict(p_s=3, p_ang=5, ns0=1, nc0=2)])
@pytest.mark.parametrize("surf,D", [("sphere", 4), ("ellipsoid", 5)])
def test_batched_equals_single(R, opts, surf, D):
    log(f"case batched R={R} {opts} {surf}")
    if surf == "sphere":
        p, nr, w = inputs.cubed_sphere(24)
    else:
        p, nr, w = inputs.ellipsoid(20, (0.5, 0.375, 0.25))
    k = 10 * np.pi
    S = inputs.random_density(len(p), nrhs=R, seed=31)
    plan = Plan(p, nr, w, k, k, depth=D, precision="fp32", max_rhs=R, **opts)
    U = plan.apply(to_dev(S)).cpu().numpy()
    assert plan.check() == 0
    for r in (0, 5, R - 1):
        ur = plan.apply(to_dev(S[:, r])).cpu().numpy()
        assert np.abs(U[:, r] - ur).max() <= 2e-5 * np.abs(ur).max(), r


def test_batched_plane_waves_against_direct_sum():
    log("case batched plane waves")
    p, nr, w = inputs.cubed_sphere(32)          # 4 wavelengths
    k = 8 * np.pi
    R = 16
    S = inputs.plane_wave_densities(p, k, R, seed=inputs.config_seed(3))
    plan = Plan(p, nr, w, k, k, depth=4, precision="fp32", max_rhs=R)
    U = plan.apply(to_dev(S.astype(np.complex64))).cpu().numpy()
    tg = inputs.sample_targets(len(p), 512, seed=5)
    ref = direct.apply_c(p, nr, w, k, k, S, targets=tg)
    err = np.linalg.norm(U[tg] - ref) / np.linalg.norm(ref)
    log(f"  rel l2 err {err:.3e}")
    assert err < 1e-4


def test_batched_constant_kernel_exact():
    p, nr, w = inputs.cubed_sphere(48)
    R = 16
    S = inputs.random_density(len(p), nrhs=R, seed=32)
    plan = Plan(p, nr, w, 16 * np.pi, 16 * np.pi, depth=5, kernel="constant", precision="fp32", max_rhs=R)
    U = plan.apply(to_dev(S)).cpu().numpy()
    A = w[:, None] * S
    ref = A.sum(0)[None, :] - A
    assert np.abs(U - ref).max() <= 2e-5 * np.abs(A).sum(0).max()


def test_batched_64_plane_waves_sphere16_sampled():
    # the batched workload at full size: N = 98,304 (16 wavelengths), D = 6,
    # 64 plane-wave right-hand sides on MFMA; four columns against the FP64
    # direct sum at 256 seeded targets
    log("case batched sphere16, 64 RHS")
    wl = inputs.workload("sphere16")
    p, nr, w = inputs.build_surface(wl)
    k = wl["k"]
    R = 64
    S = inputs.plane_wave_densities(p, k, R, seed=inputs.config_seed(3))
    plan = Plan(p, nr, w, k, k, depth=wl["depth"], precision="fp32", max_rhs=R)
    U = plan.apply(to_dev(S.astype(np.complex64))).cpu().numpy()
    assert plan.check() == 0
    tg = inputs.sample_targets(len(p), 256, seed=inputs.config_seed(3) + 100)
    cols = [0, 21, 42, 63]
    ref = direct.apply_c(p, nr, w, k, k, S[:, cols], targets=tg)
    err = np.linalg.norm(U[tg][:, cols] - ref) / np.linalg.norm(ref)
    log(f"  rel l2 err {err:.3e}")
    assert err < 1e-4
