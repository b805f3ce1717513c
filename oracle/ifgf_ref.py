"""Plain NumPy FP64 reference of the IFGF method (oracle O2).

Test infrastructure only; never imported by the product path.

It follows Section 3 of the paper in its own order and notation, for small
inputs (a few thousand points), so that each stage of the GPU path can be
compared array-for-array:

  * octree of D levels, root box B^1 containing all points, boxes of side
    H_d = H_1 / 2^(d-1), half-open as in eq. (box)            [Sec. 3.4]
  * relevant boxes, neighbours N B, cousins M B, cousin points V B
                                  [eqs. RelevantBoxes, NeighborsCousins]
  * cone segments E_gamma in (s, theta, phi), s = h / r, h = sqrt(3) H / 2,
    s in [0, sqrt(3)/3]                [eqs. def_eps, deltas, ConeIntervals]
  * cone refinement: (n_s, n_C) = (n_S0, n_C0) at d = D, doubled on each
    transition d -> d-1 while k H_d > 1/2               [Remark cone_seg_size]
  * relevant cones, top-down from d = 3                   [eq. RelevantCones]
  * tensor Chebyshev interpolation with P_s x P_ang x P_ang first-kind nodes
                                        [eqs. ChebyPoly, ChebyNodes; C10 note]
  * Algorithm 1: leaf factors F at the interpolation nodes; for d = D..3,
    interpolation at cousin points times the centred factor, and for d > 3
    interpolation at the parent's nodes times K(x, y_k) / K(x, y_j).
  * level-D neighbour interactions by direct summation (Remark
    level_D_neighboring).

The analytic factor interpolated is the combined one,
    W_c = W~2 - i k W3 - i eta W1                  (eqs. hgn2, W2W2, w23)
so that K(x, y) = exp(i k r) / (4 pi r) * W_c with r = |x - y0|, by
linearity of eq. (exponential_sum_linearity) with q = 1 for every term.

Readings of the paper taken here (each listed in the design notes):
  * Chebyshev coefficients: the printed coefficient formula (eq.
    ChebyCoeffs) does not interpolate at the printed first-kind nodes; the
    standard first-kind formula a_i = (2 - delta_i0)/n sum_k u(x_k) T_i(x_k)
    is used, which gives the unique interpolant of degree n - 1.
  * P_s = 3 and P_ang = 5 are numbers of points (degrees 2 and 4).
  * cone intervals are taken half-open with floor indices, clamped to the
    last interval (so s = sqrt(3)/3, theta = pi, phi -> 2 pi are included);
  * the polar angle is computed as atan2(sqrt(dx^2 + dy^2), dz), which is
    the same angle as acos(dz / r) and well conditioned at the poles;
  * the root box is the bounding cube of the points, its side enlarged by a
    factor (1 + 2^-20) around the bounding-box midpoint;
  * Morton keys interleave x into bit 3b, y into 3b+1, z into 3b+2; ties
    are broken by the original index.

`kind = 1` replaces K by the constant kernel K = 1 (W_c = 1, centred factor
1, ratio 1): the IFGF must then return sum_{j != i} a_j exactly, which pins
the tree traversal (every pair counted once).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

ETA_S = math.sqrt(3.0) / 3.0          # maximum s, eq. (s_rest)
ROOT_PAD = 2.0 ** -20


# ----------------------------------------------------------------------------
# Chebyshev interpolation (eqs. ChebyPoly, ChebyNodes)
# ----------------------------------------------------------------------------

def cheb_nodes(n: int) -> np.ndarray:
    """First-kind Chebyshev points x_k = cos((2k+1) pi / (2n)), k = 0..n-1."""
    k = np.arange(n)
    return np.cos((2 * k + 1) * np.pi / (2 * n))


def cheb_T(n: int, t: np.ndarray) -> np.ndarray:
    """T_i(t) for i = 0..n-1, shape t.shape + (n,), T_i(t) = cos(i arccos t)."""
    t = np.asarray(t, dtype=np.float64)
    out = np.empty(t.shape + (n,))
    out[..., 0] = 1.0
    if n > 1:
        out[..., 1] = t
    for i in range(2, n):
        out[..., i] = 2.0 * t * out[..., i - 1] - out[..., i - 2]
    return out


def cheb_coeff_matrix(n: int) -> np.ndarray:
    """M with a = M @ u: a_i = (2 - delta_i0)/n * sum_k u(x_k) T_i(x_k)."""
    x = cheb_nodes(n)
    T = cheb_T(n, x)            # T[k, i] = T_i(x_k)
    M = T.T * (2.0 / n)
    M[0, :] *= 0.5
    return M


def cheb_coeffs_3d(vals: np.ndarray) -> np.ndarray:
    """Node values (..., Ps, Pa, Pa) -> tensor Chebyshev coefficients."""
    ps, pa = vals.shape[-3], vals.shape[-1]
    Ms, Ma = cheb_coeff_matrix(ps), cheb_coeff_matrix(pa)
    c = np.einsum("ia,...abc->...ibc", Ms, vals)
    c = np.einsum("jb,...ibc->...ijc", Ma, c)
    c = np.einsum("kc,...ijc->...ijk", Ma, c)
    return c


def cheb_eval_3d(coef: np.ndarray, ts, tt, tp) -> np.ndarray:
    """sum_ijk coef[..., i, j, k] T_i(ts) T_j(tt) T_k(tp), per row."""
    ps, pa = coef.shape[-3], coef.shape[-1]
    Ts, Tt, Tp = cheb_T(ps, ts), cheb_T(pa, tt), cheb_T(pa, tp)
    return np.einsum("mijk,mi,mj,mk->m", coef, Ts, Tt, Tp)


# ----------------------------------------------------------------------------
# Octree (Section 3.4) and Morton order (Section 3.5)
# ----------------------------------------------------------------------------

def morton3(ix, iy, iz, bits: int) -> np.ndarray:
    """Interleave: bit b of ix -> 3b, of iy -> 3b+1, of iz -> 3b+2."""
    key = np.zeros(np.shape(ix), dtype=np.uint64)
    ix = np.asarray(ix, dtype=np.uint64)
    iy = np.asarray(iy, dtype=np.uint64)
    iz = np.asarray(iz, dtype=np.uint64)
    for b in range(bits):
        one = np.uint64(1)
        key |= ((ix >> np.uint64(b)) & one) << np.uint64(3 * b)
        key |= ((iy >> np.uint64(b)) & one) << np.uint64(3 * b + 1)
        key |= ((iz >> np.uint64(b)) & one) << np.uint64(3 * b + 2)
    return key


def root_box(points: np.ndarray):
    """Root cube: bounding-box midpoint, side = largest extent * (1 + 2^-20)."""
    lo = points.min(axis=0)
    hi = points.max(axis=0)
    c = (lo + hi) / 2.0
    L = float((hi - lo).max()) * (1.0 + ROOT_PAD)
    if L == 0.0:
        L = 1.0
    corner = c - L / 2.0
    return corner, L


@dataclass
class Level:
    d: int
    H: float
    coords: np.ndarray           # (nb, 3) int64 box indices (0-based k - 1)
    start: np.ndarray            # (nb + 1,) point ranges in sorted order
    centre: np.ndarray           # (nb, 3)
    parent: np.ndarray | None = None     # (nb,) index of parent box at d-1
    neighbours: list = field(default_factory=list)
    cousins: list = field(default_factory=list)
    index: dict = field(default_factory=dict)   # coords tuple -> box id


@dataclass
class Tree:
    D: int
    L: float
    corner: np.ndarray
    perm: np.ndarray             # sorted position -> original index
    keys: np.ndarray             # sorted leaf Morton keys (uint64)
    points: np.ndarray           # sorted points
    levels: dict                 # d -> Level


def build_tree(points: np.ndarray, D: int) -> Tree:
    points = np.asarray(points, dtype=np.float64)
    n = points.shape[0]
    corner, L = root_box(points)
    m = 2 ** (D - 1)
    inv_h = m / L
    kD = np.floor((points - corner) * inv_h)
    kD = np.clip(kD, 0, m - 1).astype(np.int64)
    keys = morton3(kD[:, 0], kD[:, 1], kD[:, 2], D - 1)
    perm = np.lexsort((np.arange(n), keys))
    keys_s = keys[perm]
    pts_s = points[perm]
    kD_s = kD[perm]
    levels = {}
    for d in range(1, D + 1):
        shift = D - d
        kd = kD_s >> shift
        bk = keys_s >> np.uint64(3 * shift)
        first = np.ones(n, dtype=bool)
        first[1:] = bk[1:] != bk[:-1]
        starts = np.flatnonzero(first)
        start = np.append(starts, n).astype(np.int64)
        coords = kd[starts]
        H = L / 2 ** (d - 1)
        centre = corner + (coords + 0.5) * H
        lev = Level(d=d, H=H, coords=coords, start=start, centre=centre)
        lev.index = {tuple(c): i for i, c in enumerate(coords.tolist())}
        levels[d] = lev
    for d in range(2, D + 1):
        lev, up = levels[d], levels[d - 1]
        lev.parent = np.array([up.index[tuple(c)] for c in (lev.coords >> 1).tolist()], dtype=np.int64)
    offsets = [(dx, dy, dz) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]
    for d in range(1, D + 1):
        lev = levels[d]
        nb = lev.coords.shape[0]
        lev.neighbours = []
        lev.cousins = []
        children_of = {}
        if d >= 2:
            for j, c in enumerate(lev.coords.tolist()):
                children_of.setdefault((c[0] >> 1, c[1] >> 1, c[2] >> 1), []).append(j)
        for b in range(nb):
            kb = tuple(lev.coords[b].tolist())
            nbr = sorted(lev.index[q] for q in
                         ((kb[0] + o[0], kb[1] + o[1], kb[2] + o[2]) for o in offsets) if q in lev.index)
            lev.neighbours.append(np.array(nbr, dtype=np.int64))
            cou = []
            if d >= 2:
                pk = (kb[0] >> 1, kb[1] >> 1, kb[2] >> 1)
                nset = set(nbr)
                for o in offsets:
                    for j in children_of.get((pk[0] + o[0], pk[1] + o[1], pk[2] + o[2]), []):
                        if j not in nset:
                            cou.append(j)
            lev.cousins.append(np.array(sorted(cou), dtype=np.int64))
    return Tree(D=D, L=L, corner=corner, perm=perm, keys=keys_s, points=pts_s, levels=levels)


# ----------------------------------------------------------------------------
# Cone segments (Section 3.2) and their refinement across levels
# ----------------------------------------------------------------------------

def cone_counts(k: float, L: float, D: int, ns0: int, nc0: int) -> dict:
    """(n_s, n_C) per level: initial values at d = D, doubled d -> d-1 while k H_d > 1/2."""
    out = {D: (ns0, nc0)}
    ns, nc = ns0, nc0
    for d in range(D, 1, -1):
        H = L / 2 ** (d - 1)
        if k * H > 0.5:
            ns, nc = 2 * ns, 2 * nc
        out[d - 1] = (ns, nc)
    return out


def spherical(x: np.ndarray, y0: np.ndarray, H: float):
    """(s, theta, phi) of x about y0 for a box of side H (eqs. def_eps, defparametrizationr)."""
    dx = x - y0
    r = np.sqrt(np.sum(dx * dx, axis=-1))
    s = (math.sqrt(3.0) / 2.0) * H / r
    rho = np.sqrt(dx[..., 0] ** 2 + dx[..., 1] ** 2)
    theta = np.arctan2(rho, dx[..., 2])
    phi = np.arctan2(dx[..., 1], dx[..., 0])
    phi = np.where(phi < 0.0, phi + 2.0 * math.pi, phi)
    return s, theta, phi, r


def _axis_index(v, delta, n):
    u = v / delta
    i = np.minimum(np.floor(u), n - 1).astype(np.int64)
    i = np.maximum(i, 0)
    t = 2.0 * (u - i) - 1.0
    return i, t


def cone_of(s, theta, phi, ns: int, nc: int):
    """Cone id (i_s * nc + i_th) * 2nc + i_ph and local coordinates in [-1, 1]."""
    i_s, t_s = _axis_index(s, ETA_S / ns, ns)
    i_t, t_t = _axis_index(theta, math.pi / nc, nc)
    i_p, t_p = _axis_index(phi, math.pi / nc, 2 * nc)
    cid = (i_s * nc + i_t) * (2 * nc) + i_p
    return cid, t_s, t_t, t_p


def cone_split(cid, nc: int):
    i_p = cid % (2 * nc)
    rest = cid // (2 * nc)
    return rest // nc, rest % nc, i_p


def node_coords(cids, ns: int, nc: int, ps: int, pa: int):
    """(s, theta, phi) of the P_s x P_ang x P_ang nodes of each cone: (m, ps, pa, pa)."""
    cids = np.asarray(cids, dtype=np.int64)
    i_s, i_t, i_p = cone_split(cids, nc)
    xs, xa = cheb_nodes(ps), cheb_nodes(pa)
    ds, da = ETA_S / ns, math.pi / nc
    s = (i_s[:, None] + (1.0 + xs[None, :]) / 2.0) * ds
    th = (i_t[:, None] + (1.0 + xa[None, :]) / 2.0) * da
    ph = (i_p[:, None] + (1.0 + xa[None, :]) / 2.0) * da
    m = cids.size
    S = np.broadcast_to(s[:, :, None, None], (m, ps, pa, pa))
    TH = np.broadcast_to(th[:, None, :, None], (m, ps, pa, pa))
    PH = np.broadcast_to(ph[:, None, None, :], (m, ps, pa, pa))
    return S, TH, PH


def node_points(y0, H, cids, ns, nc, ps, pa):
    """Cartesian positions of the nodes, x(s, theta, phi; y0) of eq. (defparametrizationins)."""
    S, TH, PH = node_coords(cids, ns, nc, ps, pa)
    r = (math.sqrt(3.0) / 2.0) * H / S
    x = np.stack([r * np.sin(TH) * np.cos(PH), r * np.sin(TH) * np.sin(PH), r * np.cos(TH)], axis=-1)
    return x + np.asarray(y0, dtype=np.float64).reshape(3)


# ----------------------------------------------------------------------------
# Kernel and its analytic factor (Sections 2.2 and 3.1)
# ----------------------------------------------------------------------------

def kernel(x, y, ny, k, eta, kind=0):
    """K(x, y) = dPhi/dnu(y) - i eta Phi (eqs. GreenFunction, double_layer)."""
    if kind == 1:
        return np.ones(np.broadcast_shapes(np.shape(x)[:-1], np.shape(y)[:-1]), dtype=np.complex128)
    d = x - y
    r2 = np.sum(d * d, axis=-1)
    r = np.sqrt(r2)
    dn = np.sum(d * ny, axis=-1)
    g = np.exp(1j * k * r) / (4.0 * math.pi * r)
    return g * ((1.0 - 1j * k * r) * dn / r2 - 1j * eta)


def centred_factor(x, y0, k, kind=0):
    """exp(i k r) / (4 pi r), r = |x - y0| (eq. cent_fact with q = 1)."""
    if kind == 1:
        return np.ones(np.shape(x)[:-1], dtype=np.complex128)
    r = np.sqrt(np.sum((x - y0) ** 2, axis=-1))
    return np.exp(1j * k * r) / (4.0 * math.pi * r)


def analytic_factor(x, y, ny, y0, H, k, eta, kind=0):
    """W_c = W~2 - i k W3 - i eta W1 at target x for a source y of the box (y0, H).

    With r = |x - y0|, h = sqrt(3) H / 2, s = h / r and
    v = (x - y0)/r - (y - y0) s / h (so that x - y = r v):
      W1 = exp(i k (h/s)(|v| - 1)) / |v|                        (eq. V3)
      W3 = exp(i k (h/s)(|v| - 1)) <v, nu> / |v|^2               (eq. W2W2)
      W2 = exp(i k (h/s)(|v| - 1)) <v, nu> / |v|^3               (eq. W2W2)
      W~2 = (s / h) W2                                           (eq. w23)
    """
    if kind == 1:
        return np.ones(np.broadcast_shapes(np.shape(x)[:-1], np.shape(y)[:-1]), dtype=np.complex128)
    h = math.sqrt(3.0) / 2.0 * H
    dx = x - y0
    r = np.sqrt(np.sum(dx * dx, axis=-1))
    s = h / r
    v = dx / r[..., None] - (y - y0) * (s / h)[..., None]
    nv = np.sqrt(np.sum(v * v, axis=-1))
    vn = np.sum(v * ny, axis=-1)
    e = np.exp(1j * k * (h / s) * (nv - 1.0))
    W1 = e / nv
    W3 = e * vn / nv ** 2
    W2 = e * vn / nv ** 3
    W2t = (s / h) * W2
    return W2t - 1j * k * W3 - 1j * eta * W1


# ----------------------------------------------------------------------------
# Relevant cones (eq. RelevantCones) and Algorithm 1
# ----------------------------------------------------------------------------

@dataclass
class Plan:
    tree: Tree
    k: float
    eta: float
    ps: int
    pa: int
    counts: dict                 # d -> (ns, nc)
    cones: dict                  # d -> list over boxes of sorted cone-id arrays
    normals: np.ndarray          # sorted
    weights: np.ndarray          # sorted
    kind: int = 0


def relevant_cones(tree: Tree, counts: dict, ps: int, pa: int, far_field: bool = False) -> dict:
    """Top-down from d = 3: cones hit by cousin points, and for d > 3 also by
    the interpolation nodes of the parent's relevant cones.  With far_field,
    every level-3 cone whose radial interval starts at s = 0 (x at infinity,
    any direction) is relevant too, and so, through the node rule, is what
    those cones need below."""
    out = {}
    D = tree.D
    for d in range(3, D + 1):
        lev = tree.levels[d]
        ns, nc = counts[d]
        per_box = []
        for b in range(lev.coords.shape[0]):
            hit = set()
            if far_field and d == 3:
                hit.update(range(nc * 2 * nc))      # i_s = 0, every (i_theta, i_phi)
            y0 = lev.centre[b]
            for c in lev.cousins[b]:
                x = tree.points[lev.start[c]:lev.start[c + 1]]
                s, th, ph, _ = spherical(x, y0, lev.H)
                cid, *_ = cone_of(s, th, ph, ns, nc)
                hit.update(cid.tolist())
            if d > 3:
                up = tree.levels[d - 1]
                p = lev.parent[b]
                pc = out[d - 1][p]
                if pc.size:
                    pns, pnc = counts[d - 1]
                    X = node_points(up.centre[p], up.H, pc, pns, pnc, ps, pa).reshape(-1, 3)
                    s, th, ph, _ = spherical(X, y0, lev.H)
                    cid, *_ = cone_of(s, th, ph, ns, nc)
                    hit.update(cid.tolist())
            per_box.append(np.array(sorted(hit), dtype=np.int64))
        out[d] = per_box
    return out


def make_plan(points, normals, weights, k, eta, D, ps=3, pa=5, ns0=1, nc0=2, kind=0, far_field=False) -> Plan:
    tree = build_tree(points, D)
    counts = cone_counts(k, tree.L, D, ns0, nc0)
    cones = relevant_cones(tree, counts, ps, pa, far_field) if D >= 3 else {}
    return Plan(tree=tree, k=float(k), eta=float(eta), ps=ps, pa=pa, counts=counts, cones=cones,
                normals=np.asarray(normals, dtype=np.float64)[tree.perm],
                weights=np.asarray(weights, dtype=np.float64)[tree.perm], kind=kind)


def _interp_at(plan: Plan, d: int, b: int, coef_by_cone: dict, x: np.ndarray):
    """Interpolate box b's field F at points x (about the box centre)."""
    lev = plan.tree.levels[d]
    ns, nc = plan.counts[d]
    s, th, ph, _ = spherical(x, lev.centre[b], lev.H)
    cid, ts, tt, tp = cone_of(s, th, ph, ns, nc)
    cones = plan.cones[d][b]
    pos = np.searchsorted(cones, cid)
    if np.any(pos >= cones.size) or np.any(cones[np.minimum(pos, cones.size - 1)] != cid):
        raise AssertionError("interpolation point outside the relevant cones")
    coef = coef_by_cone[b][pos]
    return cheb_eval_3d(coef, ts, tt, tp)


def leaf_values(plan: Plan, a_sorted: np.ndarray) -> list:
    """F^{k,D} at the nodes of every relevant leaf cone (Algorithm 1, first loop)."""
    t = plan.tree
    D = t.D
    lev = t.levels[D]
    ns, nc = plan.counts[D]
    out = []
    for b in range(lev.coords.shape[0]):
        cids = plan.cones[D][b]
        lo, hi = lev.start[b], lev.start[b + 1]
        y = t.points[lo:hi]
        ny = plan.normals[lo:hi]
        X = node_points(lev.centre[b], lev.H, cids, ns, nc, plan.ps, plan.pa)   # (m, ps, pa, pa, 3)
        W = analytic_factor(X[..., None, :], y, ny, lev.centre[b], lev.H, plan.k, plan.eta, plan.kind)
        out.append(W @ a_sorted[lo:hi])
    return out


def near_field(plan: Plan, a_sorted: np.ndarray) -> np.ndarray:
    """Level-D neighbour interactions by direct summation, self excluded."""
    t = plan.tree
    lev = t.levels[t.D]
    u = np.zeros(t.points.shape[0], dtype=np.complex128)
    for b in range(lev.coords.shape[0]):
        lo, hi = lev.start[b], lev.start[b + 1]
        x = t.points[lo:hi]
        src = np.concatenate([np.arange(lev.start[j], lev.start[j + 1]) for j in lev.neighbours[b]])
        with np.errstate(divide="ignore", invalid="ignore"):
            K = kernel(x[:, None, :], t.points[src][None, :, :], plan.normals[src][None, :, :],
                       plan.k, plan.eta, plan.kind)
        K[np.arange(lo, hi)[:, None] == src[None, :]] = 0.0
        u[lo:hi] = K @ a_sorted[src]
    return u


def apply(plan: Plan, sigma: np.ndarray, stages: bool = False):
    """IFGF approximation of u_i = sum_{j != i} w_j sigma_j K(x_i, x_j).

    sigma and the result are in the caller's (original) order.  With
    stages=True also returns a dict of intermediate arrays in sorted order:
    'near', 'level_u' {d: contribution of level-d cousin interpolation},
    'F_nodes' {d: list per box of (m, ps, pa, pa) node values}.
    """
    t = plan.tree
    perm = t.perm
    a = (plan.weights * np.asarray(sigma, dtype=np.complex128)[perm])
    n = a.size
    D = t.D
    u = near_field(plan, a)
    info = {"near": u.copy(), "level_u": {}, "F_nodes": {}}
    if D >= 3:
        F_nodes = {D: leaf_values(plan, a)}
        for d in range(D, 2, -1):
            lev = t.levels[d]
            coef = [cheb_coeffs_3d(v) for v in F_nodes[d]]
            ud = np.zeros(n, dtype=np.complex128)
            if d > 3:
                up = t.levels[d - 1]
                pns, pnc = plan.counts[d - 1]
                F_up = [np.zeros((c.size, plan.ps, plan.pa, plan.pa), dtype=np.complex128)
                        for c in plan.cones[d - 1]]
            for b in range(lev.coords.shape[0]):
                # (i) cousin surface points: centred factor times the interpolant
                for c in lev.cousins[b]:
                    lo, hi = lev.start[c], lev.start[c + 1]
                    x = t.points[lo:hi]
                    val = _interp_at(plan, d, b, coef, x)
                    ud[lo:hi] += centred_factor(x, lev.centre[b], plan.k, plan.kind) * val
                # (ii) parent interpolation nodes: interpolant times K(x,y_k)/K(x,y_j)
                if d > 3:
                    p = lev.parent[b]
                    pc = plan.cones[d - 1][p]
                    if pc.size == 0:
                        continue
                    X = node_points(up.centre[p], up.H, pc, pns, pnc, plan.ps, plan.pa)
                    Xf = X.reshape(-1, 3)
                    val = _interp_at(plan, d, b, coef, Xf)
                    if plan.kind == 1:
                        ratio = 1.0
                    else:
                        rc = np.sqrt(np.sum((Xf - lev.centre[b]) ** 2, axis=-1))
                        rp = np.sqrt(np.sum((Xf - up.centre[p]) ** 2, axis=-1))
                        ratio = (rp / rc) * np.exp(1j * plan.k * (rc - rp))
                    F_up[p] += (ratio * val).reshape(F_up[p].shape)
            info["level_u"][d] = ud
            u = u + ud
            if d > 3:
                F_nodes[d - 1] = F_up
        info["F_nodes"] = F_nodes
    out = np.empty_like(u)
    out[perm] = u
    if stages:
        return out, info
    return out


def far_field(plan: Plan, sigma: np.ndarray, dirs: np.ndarray) -> np.ndarray:
    """Far-field pattern (Sec. 5, eq. FarField) from the level-3 interpolants.

    For x = R xh with R -> infinity, |x - y_B| = R - xh.y_B + O(1/R) and
    s = h / |x - y_B| -> 0, so the field of box B's sources tends to
    exp(i k R) / (4 pi R) exp(-i k xh.y_B) F_B(0, theta(xh), phi(xh)); summed
    over the level-3 boxes (which hold every source):
        u_inf(xh) = 1/(4 pi) sum_B exp(-i k xh.y_B) F_B(0, xh).
    The plan must have been made with far_field=True (the s = 0 cones are then
    relevant).  For D <= 2 there is no interpolant and the plain sum over the
    points is returned."""
    xh = np.asarray(dirs, dtype=np.float64)
    t = plan.tree
    perm = t.perm
    a = plan.weights * np.asarray(sigma, dtype=np.complex128)[perm]
    if t.D < 3:
        ph = np.exp(-1j * plan.k * (xh @ t.points.T))
        return (ph * (-1j * plan.k * (xh @ plan.normals.T) - 1j * plan.eta)) @ a / (4.0 * math.pi)
    _, info = apply(plan, sigma, stages=True)
    lev = t.levels[3]
    ns, nc = plan.counts[3]
    theta = np.arctan2(np.sqrt(xh[:, 0] ** 2 + xh[:, 1] ** 2), xh[:, 2])
    phi = np.arctan2(xh[:, 1], xh[:, 0])
    phi = np.where(phi < 0.0, phi + 2.0 * math.pi, phi)
    cid, cts, ctt, ctp = cone_of(np.zeros(xh.shape[0]), theta, phi, ns, nc)   # s = 0: i_s = 0, t_s = -1
    out = np.zeros(xh.shape[0], dtype=np.complex128)
    for b in range(lev.coords.shape[0]):
        cones = plan.cones[3][b]
        if cones.size == 0:
            continue
        coef = cheb_coeffs_3d(info["F_nodes"][3][b])
        pos = np.searchsorted(cones, cid)
        if np.any(pos >= cones.size) or np.any(cones[np.minimum(pos, cones.size - 1)] != cid):
            raise AssertionError("far-field direction outside the relevant cones (plan without far_field?)")
        val = cheb_eval_3d(coef[pos], cts, ctt, ctp)
        out += np.exp(-1j * plan.k * (xh @ lev.centre[b])) * val
    return out / (4.0 * math.pi)


def tree_pairs_count(tree: Tree):
    """Per ordered pair coverage counts: near at D plus cousins at d = D..3."""
    n = tree.points.shape[0]
    cnt = np.zeros((n, n), dtype=np.int64)
    D = tree.D
    lev = tree.levels[D]
    for b in range(lev.coords.shape[0]):
        tg = np.arange(lev.start[b], lev.start[b + 1])
        for j in lev.neighbours[b]:
            src = np.arange(lev.start[j], lev.start[j + 1])
            cnt[np.ix_(tg, src)] += 1
    for d in range(3, D + 1):
        lev = tree.levels[d]
        for b in range(lev.coords.shape[0]):
            src = np.arange(lev.start[b], lev.start[b + 1])
            for c in lev.cousins[b]:
                tg = np.arange(lev.start[c], lev.start[c + 1])
                cnt[np.ix_(tg, src)] += 1
    return cnt
