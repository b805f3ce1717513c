"""Python binding: argument marshalling to the C ABI of libifgf.so.

Every computation runs in the HIP library; torch provides device memory and
the current stream only.  There is no CPU fallback.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib as L


def load_library():
    return L.load()


def library_path() -> str:
    return L.LIB_PATH


_PREC = {"fp64": L.PREC_FP64, "fp32": L.PREC_FP32_INTERP}
_KERNEL = {"combined": L.KERNEL_COMBINED, "constant": L.KERNEL_CONSTANT}
_PROP = {"auto": L.PROP_AUTO, "node": L.PROP_NODE, "cone": L.PROP_CONE, "pairs": L.PROP_PAIRS}
_TARGET = {"auto": L.TARGET_AUTO, "wave": L.TARGET_WAVE, "rows": L.TARGET_ROWS, "pairs": L.TARGET_PAIRS}


def _stream_ptr(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _check_out(out, like, name="out", inp=None):
    """A caller's output buffer must match the shape, dtype and device the
    library writes (those of `like`) and must not overlap the input (`inp`,
    default `like`): the library sees raw pointers only, so a smaller or
    mistyped buffer would be written past its end on the device."""
    if not isinstance(out, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if out.dtype != like.dtype:
        raise TypeError(f"{name} has dtype {out.dtype}, expected {like.dtype}")
    if out.device != like.device:
        raise ValueError(f"{name} is on {out.device}, expected {like.device}")
    if out.dim() == 1 and like.dim() == 2 and like.shape[1] == 1:
        out = out[:, None]
    if tuple(out.shape) != tuple(like.shape):
        raise ValueError(f"{name} has shape {tuple(out.shape)}, expected {tuple(like.shape)}")
    if not out.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    src = like if inp is None else inp
    if out.numel() and src.numel():
        o0, o1 = out.data_ptr(), out.data_ptr() + out.numel() * out.element_size()
        l0, l1 = src.data_ptr(), src.data_ptr() + src.numel() * src.element_size()
        if o0 < l1 and l0 < o1:
            raise ValueError(f"{name} overlaps the input")
    return out


def _dev_f64(x, device, shape):
    t = torch.as_tensor(x, dtype=torch.float64)
    t = t.to(device).contiguous()
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"expected shape {shape}, got {tuple(t.shape)}")
    return t


class Plan:
    """IFGF plan for the operator u_i = sum_{j != i} w_j sigma_j K(x_i, x_j).

    points, normals: (n, 3) float64 (numpy or torch); weights: (n,) float64.
    Options mirror ifgf_options (include/ifgf.h).
    """

    def __init__(self, points, normals, weights, k, eta, *, p_s=4, p_ang=6, ns0=2, nc0=4, depth=0,
                 leaf_h_lambda=0.5, precision="fp32", max_rhs=1, kernel="combined", prop_kernel="auto",
                 target_kernel="auto", far_field=False, targets=None, device="cuda"):
        lib = L.load()
        self._lib = lib
        self.device = torch.device(device)
        if self.device.type != "cuda":
            raise ValueError("the IFGF library runs on a ROCm device only")
        n = int(np.shape(points)[0])
        self.n = n
        self.k, self.eta = float(k), float(eta)
        self.precision = precision
        pts = _dev_f64(points, self.device, (n, 3))
        nrm = _dev_f64(normals, self.device, (n, 3))
        w = _dev_f64(weights, self.device, (n,))
        o = L.Options()
        lib.ifgf_options_default(ctypes.byref(o))
        o.p_s, o.p_ang, o.ns0, o.nc0, o.depth = int(p_s), int(p_ang), int(ns0), int(nc0), int(depth)
        o.leaf_h_lambda = float(leaf_h_lambda)
        o.precision = _PREC[precision]
        o.max_rhs = int(max_rhs)
        o.kernel = _KERNEL[kernel]
        o.prop_kernel = _PROP[prop_kernel]
        o.target_kernel = _TARGET[target_kernel]
        o.far_field = 1 if far_field else 0
        self.options = o
        h = ctypes.c_void_p()
        self.n_out = n
        if targets is None:
            st = lib.ifgf_plan_create(ctypes.byref(h), n, pts.data_ptr(), nrm.data_ptr(), w.data_ptr(),
                                      self.k, self.eta, ctypes.byref(o), _stream_ptr(self.device))
            L.check(st, "ifgf_plan_create")
        else:
            nt = int(np.shape(targets)[0])
            tg = _dev_f64(targets, self.device, (nt, 3))
            st = lib.ifgf_plan_create_targets(ctypes.byref(h), n, pts.data_ptr(), nrm.data_ptr(), w.data_ptr(), nt,
                                              tg.data_ptr(), self.k, self.eta, ctypes.byref(o),
                                              _stream_ptr(self.device))
            L.check(st, "ifgf_plan_create_targets")
            self.n_out = nt
        self._h = h
        self.max_rhs = int(max_rhs)

    # -- lifetime ------------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None):
            self._lib.ifgf_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- applies ---------------------------------------------------------------
    def _prep(self, x):
        x = torch.as_tensor(x)
        if not torch.is_complex(x):
            raise TypeError("complex input required")
        squeeze = x.dim() == 1
        if squeeze:
            x = x[:, None]
        if x.dim() != 2 or x.shape[0] != self.n:
            raise ValueError(f"expected ({self.n},) or ({self.n}, nrhs)")
        x = x.to(self.device).contiguous()
        dtype = L.C128 if x.dtype == torch.complex128 else L.C64
        if x.dtype not in (torch.complex64, torch.complex128):
            raise TypeError("complex64 or complex128 required")
        return x, squeeze, dtype

    def apply(self, sigma, out=None):
        """u = A sigma (forward IFGF apply); for a plan with targets, u at the targets."""
        s, squeeze, dtype = self._prep(sigma)
        like = s if self.n_out == self.n else s.new_empty((self.n_out, s.shape[1]))
        u = torch.empty_like(like) if out is None else _check_out(out, like, inp=s)
        st = self._lib.ifgf_apply(self._h, s.data_ptr(), u.data_ptr(), s.shape[1], dtype, _stream_ptr(self.device))
        L.check(st, "ifgf_apply")
        return u[:, 0] if squeeze else u

    def apply_stages(self, sigma, stage_mask=3, level_lo=0, level_hi=99):
        s, squeeze, dtype = self._prep(sigma)
        u = torch.empty_like(s)
        st = self._lib.ifgf_apply_stages(self._h, s.data_ptr(), u.data_ptr(), s.shape[1], dtype, int(stage_mask),
                                         int(level_lo), int(level_hi), _stream_ptr(self.device))
        L.check(st, "ifgf_apply_stages")
        return u[:, 0] if squeeze else u

    def apply_adjoint(self, v, conjugate=True):
        """A~^T v (conjugate=False) or A~^H v (conjugate=True) through the same tree."""
        x, squeeze, dtype = self._prep(v)
        out = torch.empty_like(x)
        st = self._lib.ifgf_apply_adjoint(self._h, x.data_ptr(), out.data_ptr(), x.shape[1], dtype,
                                          1 if conjugate else 0, _stream_ptr(self.device))
        L.check(st, "ifgf_apply_adjoint")
        return out[:, 0] if squeeze else out

    def autotune(self, reps=5) -> dict:
        """Measure and keep the fastest one-RHS formulation of every upward-pass
        level (node, cone-major tiles of 8/16/32 boxes, or the pair list) and of
        the cousin targets (rows, wave or pairs).  Returns the measurements."""
        r = L.TuneReport()
        L.check(self._lib.ifgf_plan_autotune(self._h, int(reps), ctypes.byref(r), _stream_ptr(self.device)),
                "ifgf_plan_autotune")
        names = ["node", "tile8", "tile16", "tile32", "pairs"]
        levels = {}
        for i in range(r.nlevels):
            ch = r.choice[i]
            levels[r.parent_level[i]] = {
                "choice": "node" if ch == 0 else ("pairs" if ch == 1 else f"tile{ch}"),
                "ms": {names[c]: r.ms[i][c] for c in range(5) if r.ms[i][c] >= 0},
            }
        tgt = {L.TARGET_ROWS: "rows", L.TARGET_WAVE: "wave", L.TARGET_PAIRS: "pairs"}.get(r.target_choice)
        ms = {name: r.target_ms[i] for i, name in enumerate(("rows", "wave", "pairs")) if r.target_ms[i] >= 0}
        return {"prop": levels, "targets": tgt, "targets_ms": ms if tgt else None}

    def far_field(self, sigma, dirs):
        """Far-field pattern u_inf at unit directions dirs (m, 3) (eq. FarField),
        through the tree (plan created with far_field=True unless depth <= 2)."""
        s, squeeze, dtype = self._prep(sigma)
        if s.shape[1] != 1:
            raise ValueError("one density")
        d = _dev_f64(dirs, self.device, (int(np.shape(dirs)[0]), 3))
        out = torch.empty(d.shape[0], dtype=s.dtype, device=self.device)
        st = self._lib.ifgf_far_field(self._h, s.data_ptr(), d.shape[0], d.data_ptr(), out.data_ptr(), dtype,
                                      _stream_ptr(self.device))
        L.check(st, "ifgf_far_field")
        return out

    def solve(self, f, tol=1e-4, restart=30, max_iter=300, alpha=0.5, x0=None):
        """GMRES solution of (alpha I + A) sigma = f (eq. CombLayIE with alpha = 1/2,
        f = -u^i).  f: (n,) complex; x0: optional initial iterate.  Returns
        (sigma complex128, info) with info = {iters, rel_res, history}."""
        fx = torch.as_tensor(f)
        if not torch.is_complex(fx) or fx.dim() != 1 or fx.shape[0] != self.n:
            raise ValueError(f"expected a complex ({self.n},) right-hand side")
        fx = fx.to(self.device, torch.complex128).contiguous()
        if x0 is None:
            x = torch.empty_like(fx)
        else:
            x = torch.as_tensor(x0).to(self.device, torch.complex128).clone().contiguous()
            if x.shape != fx.shape:
                raise ValueError("x0 must have the shape of f")
        o = L.GmresOptions()
        self._lib.ifgf_gmres_options_default(ctypes.byref(o))
        o.restart, o.max_iter, o.tol = int(restart), int(max_iter), float(tol)
        a = complex(alpha)
        o.alpha_re, o.alpha_im = a.real, a.imag
        o.use_guess = 0 if x0 is None else 1
        iters, res = ctypes.c_int32(0), ctypes.c_double(0.0)
        hist = (ctypes.c_double * (int(max_iter) + 1))()
        st = self._lib.ifgf_gmres_solve(self._h, fx.data_ptr(), x.data_ptr(), ctypes.byref(o), ctypes.byref(iters),
                                        ctypes.byref(res), hist, _stream_ptr(self.device))
        L.check(st, "ifgf_gmres_solve")
        return x, {"iters": iters.value, "rel_res": res.value, "history": list(hist[:iters.value + 1])}

    # -- introspection -------------------------------------------------------
    def stats(self) -> dict:
        s = L.Stats()
        L.check(self._lib.ifgf_plan_get_stats(self._h, ctypes.byref(s)), "ifgf_plan_get_stats")
        D = s.depth
        return {
            "depth": D, "n": s.n, "root_side": s.root_side, "root_corner": list(s.root_corner),
            "p_s": s.p_s, "p_ang": s.p_ang, "precision": s.precision,
            "boxes": {d: s.boxes[d] for d in range(1, D + 1)},
            "ns": {d: s.ns[d] for d in range(1, D + 1)},
            "nc": {d: s.nc[d] for d in range(1, D + 1)},
            "cones": {d: s.cones[d] for d in range(3, D + 1)},
            "cousin_pairs": {d: s.cousin_pairs[d] for d in range(3, D + 1)},
            "prop_evals": {d: s.prop_evals[d] for d in range(4, D + 1)},
            "near_pairs": s.near_pairs, "device_bytes": s.device_bytes,
            "prop_kernel": {d: {1: "node", 2: "cone", 3: "pairs"}.get(s.prop_kernel[d], "none") for d in range(4, D + 1)},
            "pair_rows": {d: s.pair_rows[d] for d in range(3, D + 1)},
            "pair_row_cones": {d: s.pair_row_cones[d] for d in range(3, D + 1)},
        }

    def set_profiling(self, max_launches: int):
        """Time up to max_launches kernel launches with HIP events (0 = off)."""
        L.check(self._lib.ifgf_plan_set_profiling(self._h, int(max_launches)), "ifgf_plan_set_profiling")

    def read_profile(self) -> dict:
        """{stage: (total ms, launches)} of the launches timed since the last read."""
        ms = (ctypes.c_double * len(L.STAGES))()
        cnt = (ctypes.c_int64 * len(L.STAGES))()
        L.check(self._lib.ifgf_plan_read_profile(self._h, ms, cnt), "ifgf_plan_read_profile")
        return {name: (ms[i], cnt[i]) for i, name in enumerate(L.STAGES) if cnt[i]}

    def check(self) -> int:
        f = ctypes.c_int32(0)
        L.check(self._lib.ifgf_plan_check(self._h, ctypes.byref(f)), "ifgf_plan_check")
        return int(f.value)

    def export_order(self):
        perm = torch.empty(self.n, dtype=torch.int32, device=self.device)
        keys = torch.empty(self.n, dtype=torch.int32, device=self.device)
        L.check(self._lib.ifgf_plan_export_order(self._h, perm.data_ptr(), keys.data_ptr()), "export_order")
        return perm.cpu().numpy(), keys.cpu().numpy().view(np.uint32)

    def export_boxes(self, d):
        nb = self.stats()["boxes"][d]
        start = torch.empty(nb + 1, dtype=torch.int32, device=self.device)
        coords = torch.empty(max(1, 3 * nb), dtype=torch.int32, device=self.device)
        L.check(self._lib.ifgf_plan_export_boxes(self._h, d, start.data_ptr(), coords.data_ptr()), "export_boxes")
        return start.cpu().numpy(), coords[:3 * nb].cpu().numpy().reshape(nb, 3)

    def export_lists(self, d, kind):
        nb = self.stats()["boxes"][d]
        ln = ctypes.c_int64(0)
        L.check(self._lib.ifgf_plan_export_lists(self._h, d, kind, None, None, ctypes.byref(ln)), "export_lists")
        off = torch.empty(nb + 1, dtype=torch.int32, device=self.device)
        idx = torch.empty(max(1, ln.value), dtype=torch.int32, device=self.device)
        L.check(self._lib.ifgf_plan_export_lists(self._h, d, kind, off.data_ptr(), idx.data_ptr(), ctypes.byref(ln)),
                "export_lists")
        off = off.cpu().numpy()
        idx = idx[:ln.value].cpu().numpy()
        return [idx[off[b]:off[b + 1]] for b in range(nb)]

    def export_cones(self, d):
        nr = self.stats()["cones"][d]
        box = torch.empty(max(1, nr), dtype=torch.int32, device=self.device)
        cone = torch.empty(max(1, nr), dtype=torch.int32, device=self.device)
        L.check(self._lib.ifgf_plan_export_cones(self._h, d, box.data_ptr(), cone.data_ptr()), "export_cones")
        return box[:nr].cpu().numpy(), cone[:nr].cpu().numpy()

    def export_field(self, d, what=0, nrhs=1):
        """Level-d field of the last apply: (cones, nrhs, P) complex, node values (0) or coefficients (1).

        The library stores (cones, P, nrhs); the result is transposed to (cones, nrhs, P)."""
        nr = self.stats()["cones"][d]
        P = self.options.p_s * self.options.p_ang ** 2
        dt = torch.complex64 if self.precision == "fp32" else torch.complex128
        buf = torch.empty(max(1, nr * P * nrhs), dtype=dt, device=self.device)
        L.check(self._lib.ifgf_plan_export_field(self._h, d, what, buf.data_ptr()), "export_field")
        return buf[:nr * P * nrhs].cpu().numpy().reshape(nr, P, nrhs).transpose(0, 2, 1)


class Batch:
    """Ragged batch of plans applied in one launch (ifgf_batch_* in include/ifgf.h).

    All plans share precision, p_s and p_ang; each takes one right-hand side.
    The batch keeps references to its plans so that they outlive it.
    """

    def __init__(self, plans):
        plans = list(plans)
        if not plans:
            raise ValueError("empty batch")
        self._lib = L.load()
        self.plans = plans
        self.device = plans[0].device
        hs = (ctypes.c_void_p * len(plans))(*[p._h for p in plans])
        h = ctypes.c_void_p()
        L.check(self._lib.ifgf_batch_create(ctypes.byref(h), len(plans), hs), "ifgf_batch_create")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            self._lib.ifgf_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def apply(self, sigmas, outs=None):
        """[u_g = A_g sigma_g for each plan g]; sigma_g of shape (n_g,), one complex dtype for all."""
        if len(sigmas) != len(self.plans):
            raise ValueError("one density per plan")
        xs, dtype = [], None
        for p, x in zip(self.plans, sigmas):
            x = torch.as_tensor(x)
            if x.dim() == 2 and x.shape[1] == 1:
                x = x[:, 0]
            if x.dim() != 1 or x.shape[0] != p.n:
                raise ValueError(f"expected a ({p.n},) density")
            if x.dtype not in (torch.complex64, torch.complex128):
                raise TypeError("complex64 or complex128 required")
            d = L.C128 if x.dtype == torch.complex128 else L.C64
            if dtype is not None and d != dtype:
                raise TypeError("all densities must share one dtype")
            dtype = d
            xs.append(x.to(self.device).contiguous())
        if outs is None:
            us = [torch.empty_like(x) for x in xs]
        else:
            outs = list(outs)
            if len(outs) != len(xs):
                raise ValueError("one output per plan")
            us = [_check_out(o, x, f"outs[{g}]") for g, (o, x) in enumerate(zip(outs, xs))]
        sp = (ctypes.c_void_p * len(xs))(*[x.data_ptr() for x in xs])
        up = (ctypes.c_void_p * len(us))(*[u.data_ptr() for u in us])
        L.check(self._lib.ifgf_batch_apply(self._h, sp, up, dtype, _stream_ptr(self.device)), "ifgf_batch_apply")
        return us

    def check(self) -> int:
        f = ctypes.c_int32(0)
        L.check(self._lib.ifgf_batch_check(self._h, ctypes.byref(f)), "ifgf_batch_check")
        return int(f.value)

    def set_spin_limit(self, limit: int):
        L.check(self._lib.ifgf_batch_set_spin_limit(self._h, int(limit)), "ifgf_batch_set_spin_limit")

    def info(self) -> dict:
        items, segs, grid, block = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        L.check(self._lib.ifgf_batch_get_info(self._h, ctypes.byref(items), ctypes.byref(segs), ctypes.byref(grid),
                                              ctypes.byref(block)), "ifgf_batch_get_info")
        return {"items": items.value, "segments": segs.value, "grid": grid.value, "block": block.value}


class IFGFApply(torch.autograd.Function):
    """u = A sigma with backward grad_sigma = A~^H grad_u (PyTorch's complex convention)."""

    @staticmethod
    def forward(ctx, sigma, plan: Plan):
        ctx.plan = plan
        return plan.apply(sigma.detach())

    @staticmethod
    def backward(ctx, grad_u):
        return ctx.plan.apply_adjoint(grad_u.contiguous(), conjugate=True), None
