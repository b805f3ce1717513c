// Plan construction on the device: root box, Morton keys and sort, per-level
// box arrays, neighbour and cousin lists, and relevant cone segments.
//
// Paper: Section 3.4 (octree of D levels, eq. box, eq. RelevantBoxes,
// eq. NeighborsCousins, eq. RelevantCones), Section 3.5 (Morton / Z-curve
// order of boxes, then cones), Remark cone_seg_size (cone counts per level).
#include <cmath>
#include <cstring>

#include <algorithm>
#include <array>

#include "internal.h"

namespace ifgf {

namespace {

constexpr int TPB = 256;
inline unsigned nblocks(int64_t n, int tpb = TPB) { return (unsigned)((n + tpb - 1) / tpb); }

// ---------------------------------------------------------------------------
// a1: bounding box and finiteness check
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(TPB) void k_bbox(const double* __restrict__ pts, const double* __restrict__ nrm,
                                              const double* __restrict__ w, int64_t n,
                                              double* __restrict__ part, int* __restrict__ bad) {
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  int nonfinite = 0;
  for (int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x; i < n; i += (int64_t)gridDim.x * TPB) {
    for (int a = 0; a < 3; ++a) {
      double x = pts[3 * i + a];
      lo[a] = fmin(lo[a], x);
      hi[a] = fmax(hi[a], x);
      nonfinite |= !isfinite(x) || !isfinite(nrm[3 * i + a]);
    }
    nonfinite |= !isfinite(w[i]);
  }
  __shared__ double sl[3][TPB], sh[3][TPB];
  for (int a = 0; a < 3; ++a) {
    sl[a][threadIdx.x] = lo[a];
    sh[a][threadIdx.x] = hi[a];
  }
  if (nonfinite) atomicOr(bad, 1);
  __syncthreads();
  for (int st = TPB / 2; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st)
      for (int a = 0; a < 3; ++a) {
        sl[a][threadIdx.x] = fmin(sl[a][threadIdx.x], sl[a][threadIdx.x + st]);
        sh[a][threadIdx.x] = fmax(sh[a][threadIdx.x], sh[a][threadIdx.x + st]);
      }
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int a = 0; a < 3; ++a) {
      part[6 * blockIdx.x + a] = sl[a][0];
      part[6 * blockIdx.x + 3 + a] = sh[a][0];
    }
}

// a1: leaf box indices by an FP64 multiply and floor (no contraction), Morton
// key in the high word, original index in the low word.
__global__ __launch_bounds__(TPB) void k_keys(const double* __restrict__ pts, int64_t n, double c0, double c1,
                                              double c2, double inv_h, int m, uint64_t* __restrict__ out) {
#pragma clang fp contract(off)
  int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (i >= n) return;
  double cc[3] = {c0, c1, c2};
  uint32_t k[3];
  for (int a = 0; a < 3; ++a) {
    double t = floor((pts[3 * i + a] - cc[a]) * inv_h);
    t = t < 0.0 ? 0.0 : (t > (double)(m - 1) ? (double)(m - 1) : t);
    k[a] = (uint32_t)t;
  }
  uint64_t key = morton_encode(k[0], k[1], k[2]);
  out[i] = (key << 32) | (uint64_t)i;
}

__global__ __launch_bounds__(TPB) void k_unpack(const uint64_t* __restrict__ sorted, int64_t n,
                                                const double* __restrict__ pts, const double* __restrict__ nrm,
                                                const double* __restrict__ w, int* __restrict__ perm,
                                                uint32_t* __restrict__ keys, double* __restrict__ spts,
                                                double* __restrict__ snrm, double* __restrict__ sw) {
  int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (i >= n) return;
  uint64_t v = sorted[i];
  int j = (int)(v & 0xffffffffu);
  perm[i] = j;
  keys[i] = (uint32_t)(v >> 32);
  for (int a = 0; a < 3; ++a) {
    spts[3 * i + a] = pts[3 * (int64_t)j + a];
    snrm[3 * i + a] = nrm[3 * (int64_t)j + a];
  }
  sw[i] = w[j];
}

// ---------------------------------------------------------------------------
// a2: per-level boxes
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(TPB) void k_level_flags(const uint32_t* __restrict__ keys, int64_t n, int shift,
                                                     uint8_t* __restrict__ flags) {
  int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (i >= n) return;
  flags[i] = (i == 0) || ((keys[i] >> shift) != (keys[i - 1] >> shift));
}

__global__ __launch_bounds__(TPB) void k_level_boxes(const uint32_t* __restrict__ keys, const uint8_t* __restrict__ flags,
                                                     const int* __restrict__ bid, int64_t n, int shift, int nb,
                                                     double c0, double c1, double c2, double H,
                                                     int* __restrict__ start, int* __restrict__ coords,
                                                     uint32_t* __restrict__ bkey, double* __restrict__ centre,
                                                     int* __restrict__ pbox) {
#pragma clang fp contract(off)
  int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (i >= n) return;
  int b = bid[i] + flags[i] - 1;
  pbox[i] = b;
  if (i == 0) start[nb] = (int)n;
  if (!flags[i]) return;
  uint32_t k = keys[i] >> shift;
  int x, y, z;
  morton_decode(k, &x, &y, &z);
  start[b] = (int)i;
  bkey[b] = k;
  coords[3 * b + 0] = x;
  coords[3 * b + 1] = y;
  coords[3 * b + 2] = z;
  centre[3 * b + 0] = c0 + ((double)x + 0.5) * H;
  centre[3 * b + 1] = c1 + ((double)y + 0.5) * H;
  centre[3 * b + 2] = c2 + ((double)z + 0.5) * H;
}

__global__ __launch_bounds__(TPB) void k_parent(const int* __restrict__ start, int nb, const int* __restrict__ pbox_up,
                                                int* __restrict__ parent) {
  int b = blockIdx.x * TPB + threadIdx.x;
  if (b < nb) parent[b] = pbox_up[start[b]];
}

__global__ __launch_bounds__(TPB) void k_child_lo(const int* __restrict__ start, int nb, const int* __restrict__ pbox_dn,
                                                  int nb_dn, int* __restrict__ child_lo) {
  int b = blockIdx.x * TPB + threadIdx.x;
  if (b < nb) child_lo[b] = pbox_dn[start[b]];
  if (b == 0) child_lo[nb] = nb_dn;
}

__device__ __forceinline__ int find_key(const uint32_t* __restrict__ keys, int nb, uint32_t k) {
  int lo = 0, hi = nb - 1;
  while (lo <= hi) {
    int mid = (lo + hi) >> 1;
    uint32_t v = keys[mid];
    if (v == k) return mid;
    if (v < k) lo = mid + 1;
    else hi = mid - 1;
  }
  return -1;
}

// Neighbours (eq. NeighborsCousins): relevant boxes with |j - k|_inf <= 1,
// self included, in (dz, dy, dx) offset order.  off == null: count only.
__global__ __launch_bounds__(TPB) void k_neighbours(const int* __restrict__ coords, const uint32_t* __restrict__ bkey,
                                                    int nb, int side, const int* __restrict__ off,
                                                    int* __restrict__ cnt_or_idx) {
  int b = blockIdx.x * TPB + threadIdx.x;
  if (b >= nb) return;
  int x = coords[3 * b], y = coords[3 * b + 1], z = coords[3 * b + 2];
  int c = 0;
  int base = off ? off[b] : 0;
  for (int dz = -1; dz <= 1; ++dz)
    for (int dy = -1; dy <= 1; ++dy)
      for (int dx = -1; dx <= 1; ++dx) {
        int X = x + dx, Y = y + dy, Z = z + dz;
        if (X < 0 || Y < 0 || Z < 0 || X >= side || Y >= side || Z >= side) continue;
        int j = find_key(bkey, nb, morton_encode(X, Y, Z));
        if (j < 0) continue;
        if (off) cnt_or_idx[base + c] = j;
        ++c;
      }
  if (!off) cnt_or_idx[b] = c;
}

// Cousins: children of the parent's neighbours that are not neighbours.
__global__ __launch_bounds__(TPB) void k_cousins(const int* __restrict__ coords, const int* __restrict__ parent, int nb,
                                                 const int* __restrict__ pnbr_off, const int* __restrict__ pnbr,
                                                 const int* __restrict__ pchild_lo, const int* __restrict__ off,
                                                 int* __restrict__ cnt_or_idx) {
  int b = blockIdx.x * TPB + threadIdx.x;
  if (b >= nb) return;
  int x = coords[3 * b], y = coords[3 * b + 1], z = coords[3 * b + 2];
  int p = parent[b];
  int c = 0;
  int base = off ? off[b] : 0;
  for (int t = pnbr_off[p]; t < pnbr_off[p + 1]; ++t) {
    int q = pnbr[t];
    for (int j = pchild_lo[q]; j < pchild_lo[q + 1]; ++j) {
      int ddx = abs(coords[3 * j] - x), ddy = abs(coords[3 * j + 1] - y), ddz = abs(coords[3 * j + 2] - z);
      if (max(ddx, max(ddy, ddz)) <= 1) continue;
      if (off) cnt_or_idx[base + c] = j;
      ++c;
    }
  }
  if (!off) cnt_or_idx[b] = c;
}

// Sorts each box's list ascending (insertion sort; lists hold at most
// 6^3 - 3^3 boxes).  The target stage merges the lists of neighbouring
// targets, which needs a common order.
__global__ __launch_bounds__(TPB) void k_sort_segments(const int* __restrict__ off, int* __restrict__ idx, int nb) {
  int b = blockIdx.x * TPB + threadIdx.x;
  if (b >= nb) return;
  const int lo = off[b], hi = off[b + 1];
  for (int t = lo + 1; t < hi; ++t) {
    const int v = idx[t];
    int u = t - 1;
    while (u >= lo && idx[u] > v) {
      idx[u + 1] = idx[u];
      --u;
    }
    idx[u + 1] = v;
  }
}

// Pair counts for statistics: sum over boxes of npts(b) * sum_{j in list(b)} npts(j)
// (targets x sources) when `per_target` = 1, or sum_b sum_{j} npts(j) otherwise.
__global__ __launch_bounds__(TPB) void k_pair_stats(const int* __restrict__ start, int nb, const int* __restrict__ off,
                                                    const int* __restrict__ idx, int weight_by_self,
                                                    unsigned long long* __restrict__ acc) {
  int b = blockIdx.x * TPB + threadIdx.x;
  unsigned long long v = 0;
  if (b < nb) {
    long long s = 0;
    for (int t = off[b]; t < off[b + 1]; ++t) s += start[idx[t] + 1] - start[idx[t]];
    v = (unsigned long long)(weight_by_self ? s * (long long)(start[b + 1] - start[b]) : s);
  }
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  if ((threadIdx.x & 63) == 0 && v) atomicAdd(acc, v);
}

// Bitwise-equal points inside one finest-level box (equal points share a box).
__global__ __launch_bounds__(TPB) void k_duplicates(const double* __restrict__ pts, const int* __restrict__ start,
                                                    int* __restrict__ flag) {
  int b = blockIdx.x;
  int lo = start[b], hi = start[b + 1];
  for (int i = lo + threadIdx.x; i < hi; i += TPB) {
    double x = pts[3 * i], y = pts[3 * i + 1], z = pts[3 * i + 2];
    for (int j = i + 1; j < hi; ++j)
      if (pts[3 * j] == x && pts[3 * j + 1] == y && pts[3 * j + 2] == z) atomicOr(flag, 1);
  }
}

// ---------------------------------------------------------------------------
// a3: relevant cones (eq. RelevantCones)
// ---------------------------------------------------------------------------
// Cones of box B hit by the points of its cousin boxes: by symmetry of the
// cousin relation, every point x marks, for each cousin B of its own box, the
// cone of B that contains x.
template <bool F32>
__global__ __launch_bounds__(TPB) void k_mark_targets(const double* __restrict__ pts, int64_t n,
                                                      const int* __restrict__ pbox, const int* __restrict__ cou_off,
                                                      const int* __restrict__ cou, const double* __restrict__ centre,
                                                      LevelGeom g, uint8_t* __restrict__ mark) {
  int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (i >= n) return;
  const double* x = pts + 3 * i;
  int A = pbox[i];
  for (int t = cou_off[A]; t < cou_off[A + 1]; ++t) {
    int B = cou[t];
    double r;
    int cid;
    if (F32) cid = target_loc32(x, centre + 3 * B, g, &r).cid;
    else cid = target_loc64(x, centre + 3 * B, g, &r).cid;
    mark[(int64_t)B * g.ncone + cid] = 1;
  }
}

// Cones of box B hit by the interpolation nodes of its parent's relevant cones.
template <bool F32>
__global__ __launch_bounds__(TPB) void k_mark_parent_nodes(int nrel_up, int P, const int* __restrict__ rel_box_up,
                                                           const int* __restrict__ rel_cone_up,
                                                           const int* __restrict__ child_lo_up,
                                                           const int* __restrict__ coords, LevelGeom gp, LevelGeom gc,
                                                           ChebTab ct, uint8_t* __restrict__ mark) {
  int64_t t = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (t >= (int64_t)nrel_up * P) return;
  int s = (int)(t / P), node = (int)(t % P);
  int a = node / (ct.pa * ct.pa), b = (node / ct.pa) % ct.pa, c = node % ct.pa;
  int Pb = rel_box_up[s], pcid = rel_cone_up[s];
  float xf[3], rpf;
  double xd[3], rpd;
  if (F32) node_rel32(pcid, a, b, c, gp, ct, xf, &rpf);
  else node_rel64(pcid, a, b, c, gp, ct, xd, &rpd);
  for (int B = child_lo_up[Pb]; B < child_lo_up[Pb + 1]; ++B) {
    int oct = (coords[3 * B] & 1) | ((coords[3 * B + 1] & 1) << 1) | ((coords[3 * B + 2] & 1) << 2);
    int cid = F32 ? child_loc32(xf, rpf, oct, gc).loc.cid : child_loc64(xd, rpd, oct, gc).loc.cid;
    mark[(int64_t)B * gc.ncone + cid] = 1;
  }
}

// The far-field cones of a level: cone ids 0 .. nfar - 1 (radial index 0) of every box.
__global__ __launch_bounds__(TPB) void k_mark_far(int64_t nt, int nfar, int ncone, uint8_t* __restrict__ mark) {
  const int64_t t = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (t >= nt) return;
  mark[(t / nfar) * ncone + t % nfar] = 1;
}

__global__ __launch_bounds__(TPB) void k_slot_finalize(const uint8_t* __restrict__ mark, int64_t total, int ncone,
                                                       int* __restrict__ slot, int* __restrict__ slot_off,
                                                       int* __restrict__ rel_box, int* __restrict__ rel_cone) {
  int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (i >= total) return;
  int v = slot[i];
  if (i % ncone == 0) slot_off[i / ncone] = v;
  if (mark[i]) {
    rel_box[v] = (int)(i / ncone);
    rel_cone[v] = (int)(i % ncone);
  } else {
    slot[i] = -1;
  }
}

__global__ __launch_bounds__(TPB) void k_prop_stats(int nrel_up, const int* __restrict__ rel_box_up,
                                                    const int* __restrict__ child_lo_up, int P,
                                                    unsigned long long* __restrict__ acc) {
  int s = blockIdx.x * TPB + threadIdx.x;
  unsigned long long v = 0;
  if (s < nrel_up) {
    int b = rel_box_up[s];
    v = (unsigned long long)(child_lo_up[b + 1] - child_lo_up[b]) * (unsigned long long)P;
  }
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  if ((threadIdx.x & 63) == 0 && v) atomicAdd(acc, v);
}

template <typename T> T read1(const void* dptr, hipStream_t s) {
  T v;
  HIPCHK(hipMemcpyAsync(&v, dptr, sizeof(T), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  return v;
}

LevelGeom make_geom(double H, int ns, int nc) {
  LevelGeom g{};
  g.H = H;
  g.h = std::sqrt(3.0) / 2.0 * H;
  g.hf = (float)g.h;
  g.ns = ns;
  g.nc = nc;
  g.ncone = ns * nc * 2 * nc;
  g.ds = (std::sqrt(3.0) / 3.0) / ns;
  g.da = IFGF_PI / nc;
  g.inv_ds = 1.0 / g.ds;
  g.inv_da = 1.0 / g.da;
  g.dsf = (float)g.ds;
  g.daf = (float)g.da;
  g.inv_dsf = (float)g.inv_ds;
  g.inv_daf = (float)g.inv_da;
  return g;
}

}  // namespace

// Sort keys (cone id, slot) of a level's relevant cones.
__global__ __launch_bounds__(TPB) void k_cone_keys(const int* __restrict__ rel_cone, int nrel,
                                                   uint64_t* __restrict__ keys) {
  const int i = blockIdx.x * TPB + threadIdx.x;
  if (i < nrel) keys[i] = ((uint64_t)(uint32_t)rel_cone[i] << 32) | (uint32_t)i;
}

// Cone-major tiles of the upward pass into level d (one right-hand side):
// the relevant cones of level d cut into tiles of up to 8 * nw boxes of one
// cone id, ordered by families of cone ids (below).  nw_req < 0
// picks nw by the heuristic below; 0 leaves the level to the node
// formulation.  Returns the nw in use.  Callable again on a built plan (the
// autotuner re-cuts a level's tiles; the node records are built once).
int build_cone_tiles(ifgf_plan_s* p, int d, int nw_req, hipStream_t s) {
  const bool f32 = p->opt.precision == IFGF_PREC_FP32_INTERP;
  const int P = p->P;
  LevelPlan& lv = p->lev[d];
  lv.ntile = 0;
  lv.ti_nw = 0;
  if (lv.nrel == 0) return 0;
  DevBuf kb;
  kb.alloc(sizeof(uint64_t) * sort_padded_length(lv.nrel));
  k_cone_keys<<<nblocks(lv.nrel), TPB, 0, s>>>(lv.rel_cone.as<int>(), lv.nrel, kb.as<uint64_t>());
  HIPCHK(hipGetLastError());
  sort_u64(kb.as<uint64_t>(), lv.nrel, s);
  std::vector<uint64_t> keys(lv.nrel);
  HIPCHK(hipMemcpyAsync(keys.data(), kb.p, sizeof(uint64_t) * lv.nrel, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  int64_t ndistinct = 0;
  for (int64_t i = 0; i < lv.nrel; ++i)
    if (i == 0 || (keys[i] >> 32) != (keys[i - 1] >> 32)) ++ndistinct;
  const double per = (double)lv.nrel / (double)ndistinct;
  // The tiles read their node records from a table of 8 records per
  // cone id (about 42 KB at P = 144 in FP32, 60 KB in FP64); where that
  // would exceed 2.5 times the level's coefficients (few boxes per cone
  // id), only a forced CONE uses them
  const bool forced = p->opt.prop_kernel == IFGF_PROP_CONE;
  lv.ti_allowed = forced || (double)ndistinct * 8.0 * (double)ti_geo_bytes(p->opt.p_s, p->opt.p_ang, f32) <=
                                2.5 * (double)lv.nrel * P * (f32 ? sizeof(cpx<float>) : sizeof(cpx<double>));
  int nw = nw_req;
  if (nw < 0) {   // the heuristic
    nw = per >= 12.0 ? 4 : (per >= 6.0 ? 2 : 0);
    if (!lv.ti_allowed) nw = 0;
    if (forced && nw == 0) nw = 1;
  }
  if (!f32 && nw > 2) nw = 2;   // FP64 tiles: at most 16 boxes (LDS)
  if (nw == 0) return 0;
  const int cap = 8 * nw;
  // child-octant mask of every box of this level, to order the boxes of
  // one cone id so that the 8 boxes of a wave tend to share their octants
  std::vector<int> clo(lv.nb + 1), ccoords(3 * (size_t)std::max(1, p->lev[d + 1].nb)), rbox(lv.nrel);
  HIPCHK(hipMemcpy(clo.data(), lv.child_lo.p, sizeof(int) * (lv.nb + 1), hipMemcpyDeviceToHost));
  HIPCHK(hipMemcpy(ccoords.data(), p->lev[d + 1].coords.p, sizeof(int) * 3 * p->lev[d + 1].nb,
                   hipMemcpyDeviceToHost));
  HIPCHK(hipMemcpy(rbox.data(), lv.rel_box.p, sizeof(int) * lv.nrel, hipMemcpyDeviceToHost));
  std::vector<uint8_t> cmask(lv.nb, 0);
  for (int b = 0; b < lv.nb; ++b)
    for (int c = clo[b]; c < clo[b + 1]; ++c)
      cmask[b] |= (uint8_t)(1u << ((ccoords[3 * c] & 1) | ((ccoords[3 * c + 1] & 1) << 1) |
                                   ((ccoords[3 * c + 2] & 1) << 2)));
  // Tile order.  A child cone is read by the parent cones whose nodes fall
  // in it: as seen from the child, the parent's radial index s maps to about
  // s / 4 and its angular indices to about half theirs, so the 16 parent
  // cone ids (s >> 2, theta >> 1, phi >> 1) - a family - read mostly the
  // same child cones.  The families come in Morton order of those indices.
  // Within a family, the union of its cone ids' boxes is ordered by child
  // octant mask, then Morton order (the 8 rows of a wave then mostly have
  // children in the same octants: rows of a box without a child in the
  // current octant are wasted); each cone id's boxes are cut, in that
  // order, into tiles of up to cap boxes, and the family's tiles run by the
  // middle of their range in it, so that tiles of sibling cone ids over the
  // same boxes run back to back (with the XCD-aware block mapping, on one
  // XCD, where the child cones they share stay in L2).
  const LevelGeom& g = lv.geom;
  auto family_key = [&](int cid) -> uint64_t {
    const int ip = cid % (2 * g.nc), it = (cid / (2 * g.nc)) % g.nc, is = cid / (2 * g.nc * g.nc);
    return ((uint64_t)morton_encode((uint32_t)(is >> 1), (uint32_t)it, (uint32_t)ip) << 1) | (uint64_t)(is & 1);
  };
  struct ConeRange {
    uint64_t key;
    int cid;
    int64_t b, e;   // the cone id's entries of keys[]
  };
  std::vector<ConeRange> cr;
  for (int64_t i = 0; i < lv.nrel;) {
    const int cid = (int)(keys[i] >> 32);
    int64_t j = i;
    while (j < lv.nrel && (int)(keys[j] >> 32) == cid) ++j;
    cr.push_back({family_key(cid), cid, i, j});
    i = j;
  }
  std::sort(cr.begin(), cr.end(), [](const ConeRange& x, const ConeRange& y) { return x.key < y.key; });
  std::vector<int> slots;   // ti_slot: the tiles' boxes (as parent slots), tile after tile
  slots.reserve(lv.nrel);
  std::vector<std::array<int, 4>> tl;   // (cid, start, count, 0)
  std::vector<int> pos(lv.nb, -1), ub;
  struct FamTile {
    int mid;
    int cid;
    std::vector<int> sl;
  };
  std::vector<FamTile> ft;
  std::vector<std::pair<int, int>> v;
  for (size_t f0 = 0; f0 < cr.size();) {
    size_t f1 = f0;
    while (f1 < cr.size() && (cr[f1].key >> 4) == (cr[f0].key >> 4)) ++f1;
    ub.clear();
    for (size_t f = f0; f < f1; ++f)
      for (int64_t t = cr[f].b; t < cr[f].e; ++t) ub.push_back(rbox[(int)(keys[t] & 0xffffffffu)]);
    std::sort(ub.begin(), ub.end(), [&](int x, int y) { return cmask[x] != cmask[y] ? cmask[x] < cmask[y] : x < y; });
    ub.erase(std::unique(ub.begin(), ub.end()), ub.end());
    for (size_t u = 0; u < ub.size(); ++u) pos[ub[u]] = (int)u;
    ft.clear();
    for (size_t f = f0; f < f1; ++f) {
      v.clear();
      for (int64_t t = cr[f].b; t < cr[f].e; ++t) {
        const int sl = (int)(keys[t] & 0xffffffffu);
        v.push_back({pos[rbox[sl]], sl});
      }
      std::sort(v.begin(), v.end());
      for (size_t t = 0; t < v.size(); t += cap) {
        const size_t e = std::min(v.size(), t + (size_t)cap);
        FamTile x{(v[t].first + v[e - 1].first) / 2, cr[f].cid, {}};
        for (size_t u = t; u < e; ++u) x.sl.push_back(v[u].second);
        ft.push_back(std::move(x));
      }
    }
    std::stable_sort(ft.begin(), ft.end(), [](const FamTile& x, const FamTile& y) { return x.mid < y.mid; });
    for (const FamTile& x : ft) {
      tl.push_back({x.cid, (int)slots.size(), (int)x.sl.size(), 0});
      slots.insert(slots.end(), x.sl.begin(), x.sl.end());
    }
    for (int u : ub) pos[u] = -1;
    f0 = f1;
  }
  // the node records of each (cone id, octant) are computed once per
  // level; a tile's fourth entry indexes its cone id's records
  std::vector<int> qlist;
  for (const auto& t : tl) qlist.push_back(t[0]);
  std::sort(qlist.begin(), qlist.end());
  qlist.erase(std::unique(qlist.begin(), qlist.end()), qlist.end());
  std::vector<int> tiles;
  tiles.reserve(tl.size() * 4);
  for (const auto& t : tl) {
    tiles.push_back(t[0]);
    tiles.push_back(t[1]);
    tiles.push_back(t[2]);
    tiles.push_back((int)(std::lower_bound(qlist.begin(), qlist.end(), t[0]) - qlist.begin()));
  }
  if (!lv.ti_geo_built) {   // the records depend on the cone ids only, not on the tile height
    build_ti_geo(p, d, qlist, s);
    lv.ti_qlist.alloc(sizeof(int) * qlist.size());
    HIPCHK(hipMemcpy(lv.ti_qlist.p, qlist.data(), sizeof(int) * qlist.size(), hipMemcpyHostToDevice));
    lv.ti_nq = (int64_t)qlist.size();
    lv.ti_geo_built = true;
  }
  // each tile box's child per octant, in ti_slot order, so that a tile
  // reads its boxes' children with one coalesced load
  std::vector<int> tchild(8 * (size_t)lv.nrel, -1);
  for (int64_t i = 0; i < lv.nrel; ++i) {
    const int b = rbox[slots[i]];
    for (int c = clo[b]; c < clo[b + 1]; ++c)
      tchild[8 * i + ((ccoords[3 * c] & 1) | ((ccoords[3 * c + 1] & 1) << 1) | ((ccoords[3 * c + 2] & 1) << 2))] = c;
  }
  // per relevant cone, the index of its cone id's records (the batched pass reads them)
  std::vector<int> trec(lv.nrel, -1);
  for (const auto& t : tl)
    for (int i = t[1]; i < t[1] + t[2]; ++i)
      trec[slots[i]] = (int)(std::lower_bound(qlist.begin(), qlist.end(), t[0]) - qlist.begin());
  lv.ti_rec.alloc(sizeof(int) * lv.nrel);
  HIPCHK(hipMemcpy(lv.ti_rec.p, trec.data(), sizeof(int) * lv.nrel, hipMemcpyHostToDevice));
  lv.ti_nw = nw;
  lv.ntile = (int64_t)tiles.size() / 4;
  lv.ti_slot.alloc(sizeof(int) * lv.nrel);
  lv.ti_tile.alloc(sizeof(int) * tiles.size());
  lv.ti_child.alloc(sizeof(int) * tchild.size());
  HIPCHK(hipMemcpy(lv.ti_slot.p, slots.data(), sizeof(int) * lv.nrel, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(lv.ti_tile.p, tiles.data(), sizeof(int) * tiles.size(), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(lv.ti_child.p, tchild.data(), sizeof(int) * tchild.size(), hipMemcpyHostToDevice));
  return nw;
}

void build_plan(ifgf_plan_s* p, const double* pts, const double* nrm, const double* w, hipStream_t s) {
  const int64_t n = p->n;
  const bool f32 = p->opt.precision == IFGF_PREC_FP32_INTERP;

  // ---- a1: root box -------------------------------------------------------
  unsigned nbb = (unsigned)std::min<int64_t>(1024, (n + TPB - 1) / TPB);
  DevBuf part, bad;
  part.alloc(sizeof(double) * 6 * nbb);
  bad.alloc(sizeof(int) * 4);
  HIPCHK(hipMemsetAsync(bad.p, 0, sizeof(int) * 4, s));
  k_bbox<<<nbb, TPB, 0, s>>>(pts, nrm, w, n, part.as<double>(), bad.as<int>());
  HIPCHK(hipGetLastError());
  std::vector<double> hpart(6 * nbb);
  int hbad[4];
  HIPCHK(hipMemcpyAsync(hpart.data(), part.p, sizeof(double) * 6 * nbb, hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(hbad, bad.p, sizeof(int) * 4, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  part.release();
  if (hbad[0]) throw Error{IFGF_EINVAL, "non-finite point, normal or weight"};
  double lo[3], hi[3];
  for (int a = 0; a < 3; ++a) {
    lo[a] = hpart[a];
    hi[a] = hpart[3 + a];
    for (unsigned b = 1; b < nbb; ++b) {
      lo[a] = std::fmin(lo[a], hpart[6 * b + a]);
      hi[a] = std::fmax(hi[a], hpart[6 * b + 3 + a]);
    }
  }
  // Root cube (a reading of "B^1 contains all points"): bounding-box midpoint,
  // side = largest extent * (1 + 2^-20).
  double ext = 0;
  double c[3];
  for (int a = 0; a < 3; ++a) {
    c[a] = (lo[a] + hi[a]) / 2.0;
    ext = std::fmax(ext, hi[a] - lo[a]);
  }
  double L = ext * (1.0 + std::ldexp(1.0, -20));
  if (L == 0.0) L = 1.0;
  for (int a = 0; a < 3; ++a) p->corner[a] = c[a] - L / 2.0;
  p->L = L;
  if (p->opt.depth <= 0) {
    double lam = 2.0 * IFGF_PI / p->k;
    int D = 1 + (int)std::lround(std::log2(L / (p->opt.leaf_h_lambda * lam)));
    p->D = std::max(1, std::min(11, D));
  } else {
    p->D = p->opt.depth;
  }
  const int D = p->D;
  const int m = 1 << (D - 1);

  // ---- a1: Morton keys and sort --------------------------------------------
  {
    DevBuf kbuf;
    int64_t cap = sort_padded_length(n);
    kbuf.alloc(sizeof(uint64_t) * cap);
    k_keys<<<nblocks(n), TPB, 0, s>>>(pts, n, p->corner[0], p->corner[1], p->corner[2], (double)m / L, m,
                                     kbuf.as<uint64_t>());
    HIPCHK(hipGetLastError());
    sort_u64(kbuf.as<uint64_t>(), n, s);
    p->perm.alloc(sizeof(int) * n);
    p->keys.alloc(sizeof(uint32_t) * n);
    p->pts.alloc(sizeof(double) * 3 * n);
    p->nrm.alloc(sizeof(double) * 3 * n);
    p->w.alloc(sizeof(double) * n);
    k_unpack<<<nblocks(n), TPB, 0, s>>>(kbuf.as<uint64_t>(), n, pts, nrm, w, p->perm.as<int>(), p->keys.as<uint32_t>(),
                                       p->pts.as<double>(), p->nrm.as<double>(), p->w.as<double>());
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s));
  }

  // ---- a2: levels -----------------------------------------------------------
  DevBuf flags, bid;
  flags.alloc(n);
  bid.alloc(sizeof(int) * (n + 1));
  std::vector<DevBuf> bkey(D + 1);
  for (int d = 1; d <= D; ++d) {
    LevelPlan& lv = p->lev[d];
    lv.d = d;
    lv.H = L / (double)(1 << (d - 1));
    int shift = 3 * (D - d);
    k_level_flags<<<nblocks(n), TPB, 0, s>>>(p->keys.as<uint32_t>(), n, shift, flags.as<uint8_t>());
    HIPCHK(hipGetLastError());
    scan_exclusive_u8(flags.as<uint8_t>(), bid.as<int>(), n, s);
    int nb = read1<int>(bid.as<int>() + n, s);
    lv.nb = nb;
    lv.start.alloc(sizeof(int) * (nb + 1));
    lv.coords.alloc(sizeof(int) * 3 * nb);
    lv.centre.alloc(sizeof(double) * 3 * nb);
    bkey[d].alloc(sizeof(uint32_t) * nb);
    lv.pbox.alloc(sizeof(int) * n);
    k_level_boxes<<<nblocks(n), TPB, 0, s>>>(p->keys.as<uint32_t>(), flags.as<uint8_t>(), bid.as<int>(), n, shift, nb,
                                            p->corner[0], p->corner[1], p->corner[2], lv.H, lv.start.as<int>(),
                                            lv.coords.as<int>(), bkey[d].as<uint32_t>(), lv.centre.as<double>(),
                                            lv.pbox.as<int>());
    HIPCHK(hipGetLastError());
  }
  flags.release();
  bid.release();
  for (int d = 2; d <= D; ++d) {
    LevelPlan& lv = p->lev[d];
    lv.parent.alloc(sizeof(int) * lv.nb);
    k_parent<<<nblocks(lv.nb), TPB, 0, s>>>(lv.start.as<int>(), lv.nb, p->lev[d - 1].pbox.as<int>(), lv.parent.as<int>());
    HIPCHK(hipGetLastError());
  }
  for (int d = 1; d < D; ++d) {
    LevelPlan& lv = p->lev[d];
    lv.child_lo.alloc(sizeof(int) * (lv.nb + 1));
    k_child_lo<<<nblocks(lv.nb), TPB, 0, s>>>(lv.start.as<int>(), lv.nb, p->lev[d + 1].pbox.as<int>(), p->lev[d + 1].nb,
                                             lv.child_lo.as<int>());
    HIPCHK(hipGetLastError());
  }
  // neighbour lists, all levels
  for (int d = 1; d <= D; ++d) {
    LevelPlan& lv = p->lev[d];
    DevBuf cnt;
    cnt.alloc(sizeof(int) * (lv.nb + 1));
    k_neighbours<<<nblocks(lv.nb), TPB, 0, s>>>(lv.coords.as<int>(), bkey[d].as<uint32_t>(), lv.nb, 1 << (d - 1), nullptr,
                                               cnt.as<int>());
    HIPCHK(hipGetLastError());
    lv.nbr_off.alloc(sizeof(int) * (lv.nb + 1));
    scan_exclusive_i32(cnt.as<int>(), lv.nbr_off.as<int>(), lv.nb, s);
    lv.nnbr = read1<int>(lv.nbr_off.as<int>() + lv.nb, s);
    lv.nbr.alloc(sizeof(int) * std::max<int64_t>(1, lv.nnbr));
    k_neighbours<<<nblocks(lv.nb), TPB, 0, s>>>(lv.coords.as<int>(), bkey[d].as<uint32_t>(), lv.nb, 1 << (d - 1),
                                               lv.nbr_off.as<int>(), lv.nbr.as<int>());
    HIPCHK(hipGetLastError());
  }
  // cousin lists, d >= 3
  for (int d = 3; d <= D; ++d) {
    LevelPlan& lv = p->lev[d];
    LevelPlan& up = p->lev[d - 1];
    DevBuf cnt;
    cnt.alloc(sizeof(int) * (lv.nb + 1));
    k_cousins<<<nblocks(lv.nb), TPB, 0, s>>>(lv.coords.as<int>(), lv.parent.as<int>(), lv.nb, up.nbr_off.as<int>(),
                                            up.nbr.as<int>(), up.child_lo.as<int>(), nullptr, cnt.as<int>());
    HIPCHK(hipGetLastError());
    lv.cou_off.alloc(sizeof(int) * (lv.nb + 1));
    scan_exclusive_i32(cnt.as<int>(), lv.cou_off.as<int>(), lv.nb, s);
    lv.ncou = read1<int>(lv.cou_off.as<int>() + lv.nb, s);
    lv.cou.alloc(sizeof(int) * std::max<int64_t>(1, lv.ncou));
    k_cousins<<<nblocks(lv.nb), TPB, 0, s>>>(lv.coords.as<int>(), lv.parent.as<int>(), lv.nb, up.nbr_off.as<int>(),
                                            up.nbr.as<int>(), up.child_lo.as<int>(), lv.cou_off.as<int>(), lv.cou.as<int>());
    HIPCHK(hipGetLastError());
    k_sort_segments<<<nblocks(lv.nb), TPB, 0, s>>>(lv.cou_off.as<int>(), lv.cou.as<int>(), lv.nb);
    HIPCHK(hipGetLastError());
  }
  // statistics and duplicate check
  {
    DevBuf acc;
    acc.alloc(sizeof(unsigned long long) * IFGF_MAX_LEVELS);
    HIPCHK(hipMemsetAsync(acc.p, 0, acc.bytes, s));
    LevelPlan& lD = p->lev[D];
    k_pair_stats<<<nblocks(lD.nb), TPB, 0, s>>>(lD.start.as<int>(), lD.nb, lD.nbr_off.as<int>(), lD.nbr.as<int>(), 1,
                                               acc.as<unsigned long long>());
    for (int d = 3; d <= D; ++d) {
      LevelPlan& lv = p->lev[d];
      k_pair_stats<<<nblocks(lv.nb), TPB, 0, s>>>(lv.start.as<int>(), lv.nb, lv.cou_off.as<int>(), lv.cou.as<int>(), 0,
                                                 acc.as<unsigned long long>() + d);
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemsetAsync(bad.p, 0, sizeof(int), s));
    k_duplicates<<<lD.nb, TPB, 0, s>>>(p->pts.as<double>(), lD.start.as<int>(), bad.as<int>());
    HIPCHK(hipGetLastError());
    unsigned long long h[IFGF_MAX_LEVELS];
    HIPCHK(hipMemcpyAsync(h, acc.p, acc.bytes, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(hbad, bad.p, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    p->near_pairs = (int64_t)h[0];
    for (int d = 3; d <= D; ++d) p->lev[d].cousin_pairs = (int64_t)h[d];
    if (hbad[0]) throw Error{IFGF_EDUPLICATE, "two points coincide"};
  }

  // ---- cone counts per level (Remark cone_seg_size) ---------------------------
  {
    int ns = p->opt.ns0, nc = p->opt.nc0;
    p->lev[D].geom = make_geom(p->lev[D].H, ns, nc);
    for (int d = D; d >= 2; --d) {
      if (p->k * p->lev[d].H > 0.5) {
        ns *= 2;
        nc *= 2;
      }
      p->lev[d - 1].geom = make_geom(p->lev[d - 1].H, ns, nc);
    }
  }
  // Chebyshev tables
  {
    ChebTab& ct = p->cheb;
    ct.ps = p->opt.p_s;
    ct.pa = p->opt.p_ang;
    for (int i = 0; i < ct.ps; ++i) {
      ct.us[i] = 0.5 * (1.0 + std::cos((2.0 * i + 1.0) * IFGF_PI / (2.0 * ct.ps)));
      ct.usf[i] = (float)ct.us[i];
    }
    for (int i = 0; i < ct.pa; ++i) {
      ct.ua[i] = 0.5 * (1.0 + std::cos((2.0 * i + 1.0) * IFGF_PI / (2.0 * ct.pa)));
      ct.uaf[i] = (float)ct.ua[i];
    }
    auto mat = [](int nn, DevBuf& md, DevBuf& mf, hipStream_t st) {
      std::vector<double> M(nn * nn);
      std::vector<float> Mf(nn * nn);
      for (int i = 0; i < nn; ++i)
        for (int k = 0; k < nn; ++k) {
          double xk = std::cos((2.0 * k + 1.0) * IFGF_PI / (2.0 * nn));
          double Ti = std::cos(i * std::acos(xk));
          double v = (i == 0 ? 1.0 : 2.0) / nn * Ti;
          M[i * nn + k] = v;
          Mf[i * nn + k] = (float)v;
        }
      md.alloc(sizeof(double) * nn * nn);
      mf.alloc(sizeof(float) * nn * nn);
      HIPCHK(hipMemcpyAsync(md.p, M.data(), md.bytes, hipMemcpyHostToDevice, st));
      HIPCHK(hipMemcpyAsync(mf.p, Mf.data(), mf.bytes, hipMemcpyHostToDevice, st));
      HIPCHK(hipStreamSynchronize(st));
    };
    mat(ct.ps, p->Ms, p->Msf, s);
    mat(ct.pa, p->Ma, p->Maf, s);
  }
  const int P = p->P;

  // ---- a3: relevant cones, top-down from d = 3 ----------------------------------
  for (int d = 3; d <= D; ++d) {
    LevelPlan& lv = p->lev[d];
    const LevelGeom& g = lv.geom;
    int64_t total = (int64_t)lv.nb * g.ncone;
    DevBuf mark;
    mark.alloc(total);
    HIPCHK(hipMemsetAsync(mark.p, 0, total, s));
    if (f32)
      k_mark_targets<true><<<nblocks(n), TPB, 0, s>>>(p->pts.as<double>(), n, lv.pbox.as<int>(), lv.cou_off.as<int>(),
                                                     lv.cou.as<int>(), lv.centre.as<double>(), g, mark.as<uint8_t>());
    else
      k_mark_targets<false><<<nblocks(n), TPB, 0, s>>>(p->pts.as<double>(), n, lv.pbox.as<int>(), lv.cou_off.as<int>(),
                                                      lv.cou.as<int>(), lv.centre.as<double>(), g, mark.as<uint8_t>());
    HIPCHK(hipGetLastError());
    if (d == 3 && p->opt.far_field) {   // far-field cones: i_s = 0, every angular interval
      const int nfar = g.nc * 2 * g.nc;
      const int64_t nt = (int64_t)lv.nb * nfar;
      if (nt > 0) {
        k_mark_far<<<nblocks(nt), TPB, 0, s>>>(nt, nfar, g.ncone, mark.as<uint8_t>());
        HIPCHK(hipGetLastError());
      }
    }
    if (d > 3) {
      LevelPlan& up = p->lev[d - 1];
      int64_t nt = (int64_t)up.nrel * P;
      if (nt > 0) {
        if (f32)
          k_mark_parent_nodes<true><<<nblocks(nt), TPB, 0, s>>>(up.nrel, P, up.rel_box.as<int>(), up.rel_cone.as<int>(),
                                                               up.child_lo.as<int>(), lv.coords.as<int>(), up.geom, g,
                                                               p->cheb, mark.as<uint8_t>());
        else
          k_mark_parent_nodes<false><<<nblocks(nt), TPB, 0, s>>>(up.nrel, P, up.rel_box.as<int>(), up.rel_cone.as<int>(),
                                                                up.child_lo.as<int>(), lv.coords.as<int>(), up.geom, g,
                                                                p->cheb, mark.as<uint8_t>());
        HIPCHK(hipGetLastError());
      }
      DevBuf acc;
      acc.alloc(sizeof(unsigned long long));
      HIPCHK(hipMemsetAsync(acc.p, 0, acc.bytes, s));
      if (up.nrel > 0) {
        k_prop_stats<<<nblocks(up.nrel), TPB, 0, s>>>(up.nrel, up.rel_box.as<int>(), up.child_lo.as<int>(), P,
                                                     acc.as<unsigned long long>());
        HIPCHK(hipGetLastError());
      }
      lv.prop_evals = (int64_t)read1<unsigned long long>(acc.p, s);
    }
    if (total > (int64_t)0x7fffffff) throw Error{IFGF_EUNSUPPORTED, "cone map too large for this level"};
    lv.slot.alloc(sizeof(int) * (total + 1));
    scan_exclusive_u8(mark.as<uint8_t>(), lv.slot.as<int>(), total, s);
    lv.nrel = read1<int>(lv.slot.as<int>() + total, s);
    lv.slot_off.alloc(sizeof(int) * (lv.nb + 1));
    lv.rel_box.alloc(sizeof(int) * std::max(1, lv.nrel));
    lv.rel_cone.alloc(sizeof(int) * std::max(1, lv.nrel));
    k_slot_finalize<<<nblocks(total), TPB, 0, s>>>(mark.as<uint8_t>(), total, g.ncone, lv.slot.as<int>(),
                                                  lv.slot_off.as<int>(), lv.rel_box.as<int>(), lv.rel_cone.as<int>());
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(lv.slot_off.as<int>() + lv.nb, &lv.nrel, sizeof(int), hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
  }

  // ---- near-field work items at the finest level --------------------------------
  {
    LevelPlan& lD = p->lev[D];
    std::vector<int> st(lD.nb + 1);
    HIPCHK(hipMemcpy(st.data(), lD.start.p, sizeof(int) * (lD.nb + 1), hipMemcpyDeviceToHost));
    std::vector<int4> wk;
    for (int b = 0; b < lD.nb; ++b)
      for (int t = 0; t < st[b + 1] - st[b]; t += kNearChunk)
        wk.push_back(make_int4(b, t, std::min(kNearChunk, st[b + 1] - st[b] - t), 0));
    lD.n_near = (int)wk.size();
    lD.near_work.alloc(sizeof(int4) * std::max<size_t>(1, wk.size()));
    if (!wk.empty())
      HIPCHK(hipMemcpy(lD.near_work.p, wk.data(), sizeof(int4) * wk.size(), hipMemcpyHostToDevice));
  }

  // ---- leaf-factor work items at the finest level ------------------------------
  {
    LevelPlan& lD = p->lev[D];
    std::vector<int4> wk;
    if (D >= 3) {
      std::vector<int> so(lD.nb + 1);
      HIPCHK(hipMemcpy(so.data(), lD.slot_off.p, sizeof(int) * (lD.nb + 1), hipMemcpyDeviceToHost));
      const int chunk = std::max(1, kLeafChunk / P) * P;   // whole cones
      for (int b = 0; b < lD.nb; ++b) {
        const int items = (so[b + 1] - so[b]) * P;
        for (int t = 0; t < items; t += chunk) wk.push_back(make_int4(b, t, std::min(chunk, items - t), 0));
      }
    }
    lD.n_leaf = (int)wk.size();
    lD.leaf_work.alloc(sizeof(int4) * std::max<size_t>(1, wk.size()));
    if (!wk.empty())
      HIPCHK(hipMemcpy(lD.leaf_work.p, wk.data(), sizeof(int4) * wk.size(), hipMemcpyHostToDevice));
  }

  // ---- work items of the upward pass: chunks of each box's relevant cones --------
  const int CH = prop_chunk(P);
  for (int d = 3; d < D; ++d) {
    LevelPlan& lv = p->lev[d];
    std::vector<int> so(lv.nb + 1);
    HIPCHK(hipMemcpy(so.data(), lv.slot_off.p, sizeof(int) * (lv.nb + 1), hipMemcpyDeviceToHost));
    std::vector<int> wk;
    for (int b = 0; b < lv.nb; ++b)
      for (int s0 = so[b]; s0 < so[b + 1]; s0 += CH) {
        wk.push_back(b);
        wk.push_back(s0);
        wk.push_back(std::min(s0 + CH, so[b + 1]));
        wk.push_back(0);
      }
    lv.nwork = (int64_t)wk.size() / 4;
    lv.work.alloc(sizeof(int) * std::max<size_t>(4, wk.size()));
    if (!wk.empty()) HIPCHK(hipMemcpy(lv.work.p, wk.data(), sizeof(int) * wk.size(), hipMemcpyHostToDevice));
  }

  // ---- cone-major tiles of the upward pass (one RHS) ------------------------------
  // Boxes per distinct cone id decide the tile height: 32 boxes (4 waves of
  // 8) from 12 boxes per cone id on - partly filled 4-wave tiles beat fuller
  // 2-wave ones, which leave the CU at 2 waves per SIMD - 16 boxes from 6;
  // AUTO leaves sparser levels to the node formulation (forced CONE: 8).
  // ifgf_plan_autotune replaces this choice by measurement.
  if (cone_prop_supported(p))
    for (int d = 3; d < D; ++d) build_cone_tiles(p, d, -1, s);

  // ---- workspaces -------------------------------------------------------------
  size_t csz = f32 ? sizeof(cpx<float>) : sizeof(cpx<double>);
  int R = p->opt.max_rhs;
  for (int d = 3; d <= D; ++d) {
    LevelPlan& lv = p->lev[d];
    if (d == D) lv.Fn.alloc(csz * (size_t)std::max(1, lv.nrel) * P * R);
    lv.Fc.alloc(csz * (size_t)std::max(1, lv.nrel) * P * R);
  }
  p->a.alloc(csz * (size_t)n * R);
  p->uacc.alloc(csz * (size_t)n * R);
  if (p->opt.target_kernel != IFGF_TARGET_WAVE && D >= 3) p->tpart.alloc(csz * (size_t)n * (D - 2));
  p->err.alloc(sizeof(int) * 4);
  HIPCHK(hipMemsetAsync(p->err.p, 0, sizeof(int) * 4, s));
  HIPCHK(hipStreamSynchronize(s));
  build_target_pairs(p, s);   // after the error flags exist: the pair generators report missing cones there
  build_plan_up_pairs(p, s);
}

}  // namespace ifgf
