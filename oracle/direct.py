"""FP64 direct sums of the discrete combined-field operator (oracle O1).

Test infrastructure only.  Two independent implementations of the same plain
definition (paper Section 3, eq. field1; kernel of Section 2.2, eqs.
CombinedLayer, GreenFunction, double_layer):

    u_i = sum_{j != i} w_j sigma_j K(x_i, x_j)
    K(x, y) = exp(ikr)/(4 pi r) * [ (1 - ikr) <x - y, n_y> / r^2 - i eta ]

`apply_c`   : the C/OpenMP loop in direct.c (timed as the CPU baseline)
`apply_np`  : NumPy, vectorized over sources, row blocks of targets
`dense_np`  : the dense N x N matrix A_ij = w_j K(x_i, x_j) (A_ii = 0)

`kind=1` selects the constant test kernel K = 1, for which the discrete sum
is sum_{j != i} w_j sigma_j.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import build as _build

_lib = None


def _load():
    global _lib
    if _lib is None:
        path = _build.build()
        lib = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        lp = ctypes.POINTER(ctypes.c_int64)
        for name in ("oracle_direct_apply", "oracle_direct_apply_transpose"):
            f = getattr(lib, name)
            f.argtypes = [ctypes.c_int64, dp, dp, dp, ctypes.c_double, ctypes.c_double,
                          ctypes.c_int, dp, ctypes.c_int, lp, ctypes.c_int64, dp]
            f.restype = None
        lib.oracle_num_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def _prep(points, normals, weights, sigma):
    pts = np.ascontiguousarray(points, dtype=np.float64)
    nrm = np.ascontiguousarray(normals, dtype=np.float64)
    w = np.ascontiguousarray(weights, dtype=np.float64)
    s = np.asarray(sigma, dtype=np.complex128)
    squeeze = s.ndim == 1
    if squeeze:
        s = s[:, None]
    s = np.ascontiguousarray(s)
    n = pts.shape[0]
    if pts.shape != (n, 3) or nrm.shape != (n, 3) or w.shape != (n,) or s.shape[0] != n:
        raise ValueError("shape mismatch")
    if s.shape[1] > 64:
        raise ValueError("the C oracle handles at most 64 right-hand sides per call")
    return pts, nrm, w, s, squeeze


def _call(name, points, normals, weights, k, eta, sigma, targets, kind):
    pts, nrm, w, s, squeeze = _prep(points, normals, weights, sigma)
    n, r = s.shape
    lib = _load()
    dp = ctypes.POINTER(ctypes.c_double)
    if targets is None:
        tg = None
        m = n
        tptr = None
    else:
        tg = np.ascontiguousarray(targets, dtype=np.int64)
        if tg.size and (tg.min() < 0 or tg.max() >= n):
            raise ValueError("target index out of range")
        m = tg.size
        tptr = tg.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    out = np.zeros((m, r), dtype=np.complex128)
    getattr(lib, name)(n, pts.ctypes.data_as(dp), nrm.ctypes.data_as(dp), w.ctypes.data_as(dp),
                       float(k), float(eta), int(kind), s.ctypes.data_as(dp), r, tptr, m,
                       out.ctypes.data_as(dp))
    return out[:, 0] if squeeze else out


def apply_c(points, normals, weights, k, eta, sigma, targets=None, kind=0):
    """u at `targets` (all points if None) by the C/OpenMP double loop."""
    return _call("oracle_direct_apply", points, normals, weights, k, eta, sigma, targets, kind)


def apply_transpose_c(points, normals, weights, k, eta, v, outputs=None, kind=0):
    """(A^T v) at `outputs` (all if None): w_j sum_{i != j} v_i K(x_i, x_j)."""
    return _call("oracle_direct_apply_transpose", points, normals, weights, k, eta, v, outputs, kind)


def kernel_np(x, y, ny, k, eta, kind=0):
    """K(x, y) for broadcastable arrays x (...,3), y (...,3), ny (...,3)."""
    if kind == 1:
        return np.ones(np.broadcast_shapes(x.shape[:-1], y.shape[:-1]), dtype=np.complex128)
    d = x - y
    r2 = np.sum(d * d, axis=-1)
    r = np.sqrt(r2)
    dn = np.sum(d * ny, axis=-1)
    g = np.exp(1j * k * r) / (4.0 * np.pi * r)
    return g * ((1.0 - 1j * k * r) * dn / r2 - 1j * eta)


def apply_np(points, normals, weights, k, eta, sigma, targets=None, kind=0, block=256):
    """NumPy direct sum; independent of the C loop."""
    pts = np.asarray(points, dtype=np.float64)
    nrm = np.asarray(normals, dtype=np.float64)
    w = np.asarray(weights, dtype=np.float64)
    s = np.asarray(sigma, dtype=np.complex128)
    squeeze = s.ndim == 1
    if squeeze:
        s = s[:, None]
    n = pts.shape[0]
    tg = np.arange(n) if targets is None else np.asarray(targets, dtype=np.int64)
    a = w[:, None] * s
    out = np.zeros((tg.size, s.shape[1]), dtype=np.complex128)
    for b0 in range(0, tg.size, block):
        rows = tg[b0:b0 + block]
        with np.errstate(divide="ignore", invalid="ignore"):
            K = kernel_np(pts[rows][:, None, :], pts[None, :, :], nrm[None, :, :], k, eta, kind)
        K[np.arange(rows.size), rows] = 0.0
        out[b0:b0 + block] = K @ a
    return out[:, 0] if squeeze else out


def dense_np(points, normals, weights, k, eta, kind=0):
    """Dense matrix A with A[i, j] = w_j K(x_i, x_j), A[i, i] = 0 (small N only)."""
    pts = np.asarray(points, dtype=np.float64)
    nrm = np.asarray(normals, dtype=np.float64)
    w = np.asarray(weights, dtype=np.float64)
    n = pts.shape[0]
    if n > 8192:
        raise ValueError("dense matrix limited to N <= 8192")
    with np.errstate(divide="ignore", invalid="ignore"):
        K = kernel_np(pts[:, None, :], pts[None, :, :], nrm[None, :, :], k, eta, kind)
    K[np.arange(n), np.arange(n)] = 0.0
    return K * w[None, :]


def far_field_np(points, normals, weights, k, eta, sigma, dirs, block=512):
    """Far-field pattern of the combined-field potential with density sigma
    (Sec. 5, eq. FarField, coupling gamma = eta):

        u_inf(xh) = 1/(4 pi) sum_j w_j sigma_j exp(-i k xh.y_j) (-i k <xh, n_j> - i eta)

    for unit directions dirs (m, 3); the derivative along n_j of
    exp(-i k xh.y) is -i k <xh, n_j> exp(-i k xh.y)."""
    pts = np.asarray(points, dtype=np.float64)
    nrm = np.asarray(normals, dtype=np.float64)
    a = np.asarray(weights, dtype=np.float64) * np.asarray(sigma, dtype=np.complex128)
    xh = np.asarray(dirs, dtype=np.float64)
    out = np.zeros(xh.shape[0], dtype=np.complex128)
    for b0 in range(0, xh.shape[0], block):
        d = xh[b0:b0 + block]
        ph = np.exp(-1j * k * (d @ pts.T))
        out[b0:b0 + block] = (ph * (-1j * k * (d @ nrm.T) - 1j * eta)) @ a / (4.0 * np.pi)
    return out


def field_np(points, normals, weights, k, eta, sigma, targets, block=256):
    """The combined-field potential (eq. CombinedLayer, discretized as in
    eq. field1) at arbitrary points x distinct from the surface points:
    u(x) = sum_j w_j sigma_j K(x, x_j), every j included."""
    pts = np.asarray(points, dtype=np.float64)
    nrm = np.asarray(normals, dtype=np.float64)
    a = np.asarray(weights, dtype=np.float64) * np.asarray(sigma, dtype=np.complex128)
    x = np.asarray(targets, dtype=np.float64)
    out = np.zeros(x.shape[0], dtype=np.complex128)
    for b0 in range(0, x.shape[0], block):
        K = kernel_np(x[b0:b0 + block][:, None, :], pts[None, :, :], nrm[None, :, :], k, eta)
        out[b0:b0 + block] = K @ a
    return out
