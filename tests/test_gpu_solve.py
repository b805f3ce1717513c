"""GPU tests of the GMRES solve of the combined-field integral equation
(eq. CombLayIE): (1/2 I + A) sigma = f.

The oracle is the dense linear solve of the same discrete system (numpy's
LU on the oracle's dense matrix).  With depth 2 the plan's operator is the
exact direct sum (everything is near field), so GMRES must reproduce the
dense solution to its own tolerance; at 4 wavelengths with the IFGF the
residual of the returned density is checked with the oracle's direct sum.
"""
import ctypes

import numpy as np
import pytest
import torch

from oracle import direct
from paper_2112_06316_amd import Plan, inputs
from paper_2112_06316_amd import _lib as L

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def log(msg):
    print(msg, flush=True)


def plane_wave_rhs(p, k, seed):
    d = np.random.default_rng(seed).normal(size=3)
    d /= np.linalg.norm(d)
    return -np.exp(1j * k * (p @ d))     # f = -u^i on the surface (eq. CombLayIE)


@pytest.mark.parametrize("restart", [60, 7])
def test_gmres_matches_dense_solve_exact_operator(restart):
    p, nr, w = inputs.cubed_sphere(12)                       # N = 864
    k = 4 * np.pi
    eta = max(3.0, 1.0 / (2 * np.pi / k))                    # eq. gamma: max(3, diameter / wavelength)
    f = plane_wave_rhs(p, k, 31)
    A = direct.dense_np(p, nr, w, k, eta)
    ref = np.linalg.solve(0.5 * np.eye(len(p)) + A, f)
    plan = Plan(p, nr, w, k, eta, depth=2, precision="fp64")  # depth 2: the exact direct sum
    x, info = plan.solve(torch.from_numpy(f).to(DEV), tol=1e-12, restart=restart, max_iter=600)
    x = x.cpu().numpy()
    log(f"case gmres exact restart={restart}: {info['iters']} iterations, rel res {info['rel_res']:.2e}")
    assert info["rel_res"] <= 1e-12
    assert np.linalg.norm(x - ref) / np.linalg.norm(ref) <= 1e-10
    res = np.linalg.norm(f - (0.5 * x + A @ x)) / np.linalg.norm(f)
    assert res <= 1e-11
    hist = info["history"]
    assert len(hist) == info["iters"] + 1 and hist[0] == pytest.approx(1.0)


def test_gmres_initial_guess_and_determinism():
    p, nr, w = inputs.cubed_sphere(12)
    k = 4 * np.pi
    f = torch.from_numpy(plane_wave_rhs(p, k, 32)).to(DEV)
    plan = Plan(p, nr, w, k, 3.0, depth=4, precision="fp64")
    x1, i1 = plan.solve(f, tol=1e-10, restart=20)
    x2, i2 = plan.solve(f, tol=1e-10, restart=20)
    assert torch.equal(x1, x2) and i1["iters"] == i2["iters"]
    # started from the solution, GMRES stops at once
    x3, i3 = plan.solve(f, tol=1e-9, restart=20, x0=x1)
    assert i3["iters"] == 0 and i3["rel_res"] <= 1e-9
    assert torch.equal(x3, x1)


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_gmres_ifgf_sphere_4_wavelengths(precision):
    p, nr, w = inputs.cubed_sphere(32)                       # N = 6,144
    k = 8 * np.pi
    eta = 4.0                                                # eq. gamma: max(3, 4 wavelengths)
    f = plane_wave_rhs(p, k, 33)
    plan = Plan(p, nr, w, k, eta, depth=4, precision=precision)
    x, info = plan.solve(torch.from_numpy(f).to(DEV), tol=1e-4)
    x = x.cpu().numpy()
    log(f"case gmres ifgf {precision}: {info['iters']} iterations, rel res {info['rel_res']:.2e}")
    assert info["rel_res"] <= 1e-4
    assert info["iters"] < 60
    # residual of the returned density with the oracle's exact operator: the
    # GMRES tolerance plus the IFGF error of the apply
    Ax = direct.apply_c(p, nr, w, k, eta, x)
    res = np.linalg.norm(f - (0.5 * x + Ax)) / np.linalg.norm(f)
    log(f"  residual with the direct sum {res:.2e}")
    assert res <= 2e-4


def test_gmres_argument_errors():
    p, nr, w = inputs.cubed_sphere(4)
    plan = Plan(p, nr, w, 4.0, 4.0, depth=3, precision="fp64")
    lib = L.load()
    f = torch.ones(len(p), dtype=torch.complex128, device=DEV)
    x = torch.empty_like(f)
    it, rr = ctypes.c_int32(), ctypes.c_double()
    o = L.GmresOptions()
    lib.ifgf_gmres_options_default(ctypes.byref(o))
    assert (o.restart, o.max_iter, o.tol, o.alpha_re, o.alpha_im, o.use_guess) == (30, 300, 1e-4, 0.5, 0.0, 0)
    st = lib.ifgf_gmres_solve(plan._h, f.data_ptr(), f.data_ptr(), ctypes.byref(o), ctypes.byref(it),
                              ctypes.byref(rr), None, None)
    assert st == L.EINVAL                      # f and sigma alias
    o.restart = 0
    st = lib.ifgf_gmres_solve(plan._h, f.data_ptr(), x.data_ptr(), ctypes.byref(o), ctypes.byref(it),
                              ctypes.byref(rr), None, None)
    assert st == L.EINVAL
    # a zero right-hand side gives sigma = 0 with no iteration
    z = torch.zeros_like(f)
    xz, info = plan.solve(z)
    assert info["iters"] == 0 and bool((xz == 0).all())
