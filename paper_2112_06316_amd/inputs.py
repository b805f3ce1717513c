"""Seeded synthetic inputs: surfaces, quadrature weights, densities, targets.

This module holds no arithmetic of the accelerated method: it only builds
the point sets, normals, quadrature weights and densities that both the
HIP path and the test oracle consume.  Every generator is deterministic
given its seed.

Surfaces stand in for the sphere benchmarks of the paper (Section 5.1,
Table "AcouSphere"): the paper discretizes each of its patches with a
Chebyshev grid; here a cubed sphere with an equiangular grid per face is
used instead, with exact normals and exact area-element weights, so the
discrete sum of the combined-field operator (eq. field1) has the same
structure (a smooth closed surface, about 10 points per wavelength at the
benchmark sizes).
"""
from __future__ import annotations

import numpy as np

SEED_BASE = 2112063160


def config_seed(config: int) -> int:
    """Seed used for the densities of workload `config` (1-based)."""
    return SEED_BASE + int(config)


def _cube_face_grid(n: int):
    """Equiangular grid on the 6 faces of a cube projected on the unit sphere.

    Returns unit points p (6n^2, 3) and the unit-sphere area element times
    the grid cell (dalpha*dbeta), i.e. quadrature weights on the unit sphere.
    """
    if n < 1:
        raise ValueError("n must be >= 1")
    h = np.pi / (2.0 * n)
    a = -np.pi / 4.0 + (np.arange(n) + 0.5) * h
    ta = np.tan(a)
    X, Y = np.meshgrid(ta, ta, indexing="ij")
    X = X.ravel()
    Y = Y.ravel()
    dens = 1.0 + X * X + Y * Y
    # area element of the gnomonic equiangular map on the unit sphere
    w_face = h * h * (1.0 + X * X) * (1.0 + Y * Y) / dens ** 1.5
    pts = []
    wts = []
    for axis in range(3):
        for sign in (1.0, -1.0):
            d = np.empty((X.size, 3))
            d[:, axis] = sign
            d[:, (axis + 1) % 3] = X
            d[:, (axis + 2) % 3] = Y
            d /= np.sqrt(dens)[:, None]
            pts.append(d)
            wts.append(w_face)
    return np.concatenate(pts), np.concatenate(wts)


def cubed_sphere(n: int, radius: float = 0.5, center=(0.0, 0.0, 0.0)):
    """Cubed sphere of the given radius with n x n points per face.

    Returns (points (N,3), normals (N,3), weights (N,)) with N = 6 n^2,
    float64.  Normals are the exact outward unit normals and the weights
    are the exact area element times the parameter cell, so that
    sum(weights) approaches 4 pi radius^2.
    """
    p, w = _cube_face_grid(n)
    pts = radius * p + np.asarray(center, dtype=np.float64)[None, :]
    return np.ascontiguousarray(pts), np.ascontiguousarray(p.copy()), np.ascontiguousarray(w * radius * radius)


def ellipsoid(n: int, semi_axes=(1.0, 1.0, 5.0), center=(0.0, 0.0, 0.0)):
    """Ellipsoid x = (a p1, b p2, c p3) over the unit cubed-sphere grid p.

    Normals are proportional to (x1/a^2, x2/b^2, x3/c^2), normalized; the
    weights are the unit-sphere weights times the exact area Jacobian
    abc * |(p1/a, p2/b, p3/c)|.
    """
    a, b, c = (float(v) for v in semi_axes)
    p, w = _cube_face_grid(n)
    ax = np.array([a, b, c])
    pts = p * ax[None, :]
    g = p / ax[None, :]
    gn = np.linalg.norm(g, axis=1)
    nrm = g / gn[:, None]
    wts = w * a * b * c * gn
    pts = pts + np.asarray(center, dtype=np.float64)[None, :]
    return np.ascontiguousarray(pts), np.ascontiguousarray(nrm), np.ascontiguousarray(wts)


def random_density(n: int, nrhs: int = 1, seed: int = SEED_BASE, dtype=np.complex128):
    """sigma ~ N(0,1) + i N(0,1), shape (n,) if nrhs == 1 else (n, nrhs)."""
    rng = np.random.default_rng(seed)
    re = rng.standard_normal((n, nrhs))
    im = rng.standard_normal((n, nrhs))
    s = (re + 1j * im).astype(dtype)
    return s[:, 0].copy() if nrhs == 1 else s


def plane_wave_directions(nrhs: int, seed: int):
    """Unit directions drawn uniformly on the sphere (normalized N(0, I3))."""
    rng = np.random.default_rng(seed)
    d = rng.standard_normal((nrhs, 3))
    return d / np.linalg.norm(d, axis=1)[:, None]


def plane_wave_densities(points, k: float, nrhs: int, seed: int, dtype=np.complex128):
    """sigma[j, r] = exp(i k d_r . y_j): plane-wave traces (paper eq. PlaneWave)."""
    d = plane_wave_directions(nrhs, seed)
    ph = k * (points @ d.T)
    return np.exp(1j * ph).astype(dtype)


def sample_targets(n: int, m: int, seed: int):
    """m distinct target indices out of n, sorted ascending."""
    rng = np.random.default_rng(seed)
    m = min(int(m), int(n))
    return np.sort(rng.choice(n, m, replace=False)).astype(np.int64)


# Named workloads: (surface builder, wavenumber, coupling, depth).
def workload(name: str):
    """Return a dict describing one named synthetic workload.

    sphere4:   unit-diameter sphere, 4 wavelengths (k = 8 pi), 6 x 32^2 points
    sphere32:  unit-diameter sphere, 32 wavelengths (k = 64 pi), 6 x 256^2 points
    sphere16:  unit-diameter sphere, 16 wavelengths (k = 32 pi), 6 x 128^2 points
    spheroid40: spheroid (1,1,5), 40 wavelengths long (k = 8 pi), 6 x 500^2 points
    sphere128: unit-diameter sphere, 128 wavelengths (k = 256 pi), 6 x 1024^2 points
    """
    table = {
        "sphere4": dict(kind="sphere", n=32, k=8 * np.pi, depth=4, config=1),
        "sphere16": dict(kind="sphere", n=128, k=32 * np.pi, depth=6, config=3),
        "sphere32": dict(kind="sphere", n=256, k=64 * np.pi, depth=7, config=2),
        "spheroid40": dict(kind="spheroid", n=500, k=8 * np.pi, depth=7, config=4),
        "sphere128": dict(kind="sphere", n=1024, k=256 * np.pi, depth=9, config=5),
    }
    if name not in table:
        raise KeyError(name)
    w = dict(table[name])
    w["eta"] = w["k"]
    return w


def build_surface(w: dict):
    if w["kind"] == "sphere":
        return cubed_sphere(w["n"], 0.5)
    if w["kind"] == "spheroid":
        return ellipsoid(w["n"], (1.0, 1.0, 5.0))
    raise KeyError(w["kind"])


RAGGED_N = (32, 48, 64, 80, 96, 112, 128, 128)


def ragged_batch(sizes=RAGGED_N):
    """Ragged multi-geometry batch: geometry b has 6 x n_b^2 points; even b a
    sphere of radius 0.5, odd b an ellipsoid with semi-axes (0.5, 0.375,
    0.25).  Both have largest diameter 1, and k_b = 2 pi (n_b / 8), so the
    diameter is n_b / 8 wavelengths (about 10 points per wavelength, as the
    16-wavelength sphere); eta_b = k_b.  Returns a list of dicts with keys
    points, normals, weights, k, eta, n, seed."""
    out = []
    for b, nb in enumerate(sizes):
        if b % 2 == 0:
            p, nr, w = cubed_sphere(nb, 0.5)
        else:
            p, nr, w = ellipsoid(nb, (0.5, 0.375, 0.25))
        k = 2.0 * np.pi * nb / 8.0
        out.append(dict(points=p, normals=nr, weights=w, k=k, eta=k, n=len(p), seed=config_seed(3) + 1000 + b))
    return out
