// IFGF apply on the device (paper Section 3, Algorithm 1).
//
// Stages of one apply, in launch order:
//   gather    a_j = w_j sigma_j into Morton order
//   near      level-D neighbour interactions by direct summation, self
//             excluded by index (Remark level_D_neighboring; eq. field1)
//   leaf      F^{k,D} at the interpolation nodes of every relevant leaf cone
//             (Algorithm 1, first loop): F = sum_{y in B} a_y W_c(x, y)
//   coeffs    node values -> tensor Chebyshev coefficients per cone
//   prop      for d = D..4: each node x of each relevant cone of a level-(d-1)
//             box P gets sum over children B of I[F_B](x) K(x,y_B)/K(x,y_P)
//             (Algorithm 1, parent-node update)
//   targets   for d = D..3: every point x gets, for each box B of which it is
//             a cousin point, e^{ikr}/(4 pi r) I[F_B](x) (Algorithm 1, cousin
//             interpolation), plus its near-field sum; scattered back to the
//             caller's order.
//
// The analytic factor is the combined W_c = W~2 - i k W3 - i eta W1 (eqs.
// hgn2, W2W2, w23): one field per box, valid by the linearity of eq.
// (exponential_sum_linearity) with q = 1 for each term.
//
// Interpolant evaluation: a lane that needs cone `slot` of some box reads
// that cone's P coefficients.  Lanes of a wave that need the same cone are
// served together: the wave repeatedly takes the slot of its first pending
// lane, makes it wave-uniform with readfirstlane, and every lane holding that
// slot evaluates with the uniform coefficient pointer.
#include <mutex>
#include <type_traits>

#include "internal.h"

namespace ifgf {

namespace {

constexpr int TPB = 256;
inline unsigned nblocks(int64_t n, int tpb = TPB) { return (unsigned)((n + tpb - 1) / tpb); }

template <typename T> struct Prec;
template <> struct Prec<float> {
  static constexpr bool f32 = true;
};
template <> struct Prec<double> {
  static constexpr bool f32 = false;
};

template <typename T> __device__ __forceinline__ void sincos_t(T x, T* s, T* c);
template <> __device__ __forceinline__ void sincos_t<float>(float x, float* s, float* c) { sincos_f(x, s, c); }
template <> __device__ __forceinline__ void sincos_t<double>(double x, double* s, double* c) { sincos(x, s, c); }
// The leaf and near-field phases (a few radians to a few hundred): in FP64
// the reduction and series of sincos_cw64 instead of the library call
template <typename T> __device__ __forceinline__ void sincos_phase(T x, T* s, T* c) {
  if constexpr (sizeof(T) == 8) sincos_cw64(x, s, c);
  else sincos_t<T>(x, s, c);
}

template <typename T> __device__ __forceinline__ T sqrt_t(T x);
template <> __device__ __forceinline__ float sqrt_t<float>(float x) { return sqrt_f(x); }   // hardware, ~1 ulp
template <> __device__ __forceinline__ double sqrt_t<double>(double x) { return sqrt(x); }
// 1/x: the hardware reciprocal in FP32 (about 1 ulp, as elsewhere in the FP32
// path), IEEE division in FP64.
// sqrt(x) and 1 / sqrt(x) of x > 0: in FP32 from the hardware reciprocal
// square root (one transcendental instead of a square root and a reciprocal)
template <typename T> __device__ __forceinline__ void sqrt_rsqrt(T x, T* sq, T* rs);
template <> __device__ __forceinline__ void sqrt_rsqrt<float>(float x, float* sq, float* rs) {
  const float r = __builtin_amdgcn_rsqf(x);
  *rs = r;
  *sq = x * r;
}
template <> __device__ __forceinline__ void sqrt_rsqrt<double>(double x, double* sq, double* rs) {
  sqrt_rsqrt_nr64(x, sq, rs);
}
template <typename T> __device__ __forceinline__ T rcp_t(T x);
template <> __device__ __forceinline__ float rcp_t<float>(float x) { return rcp_f(x); }
template <> __device__ __forceinline__ double rcp_t<double>(double x) { return rcp_nr64(x); }

// ---------------------------------------------------------------------------
// gather: a[i, r] = w_i sigma[perm_i, r]; points with caller index >= n_src
// (targets only) get 0 and sigma is not read there.
// ---------------------------------------------------------------------------
// Element q = (point i, right-hand side r), right-hand sides fastest.
template <typename T>
__device__ __forceinline__ void gather_one(int64_t q, const void* __restrict__ sigma, int dtype, int conj_in,
                                           const int* __restrict__ perm, const double* __restrict__ w, int64_t n,
                                           int R, cpx<T>* __restrict__ a, int64_t n_src) {
  if (q >= n * R) return;
  const int64_t i = q / R;
  const int r = (int)(q % R);
  const int64_t j = perm[i];
  if (j >= n_src) {
    a[i * R + r] = {(T)0, (T)0};
    return;
  }
  const double wi = w ? w[i] : 1.0;
  double re, im;
  if (dtype == IFGF_C128) {
    const double* s = (const double*)sigma + 2 * (j * R + r);
    re = s[0];
    im = s[1];
  } else {
    const float* s = (const float*)sigma + 2 * (j * R + r);
    re = s[0];
    im = s[1];
  }
  if (conj_in) im = -im;
  a[i * R + r] = {(T)(wi * re), (T)(wi * im)};
}

template <typename T>
__global__ __launch_bounds__(TPB) void k_gather(const void* __restrict__ sigma, int dtype, int conj_in,
                                                const int* __restrict__ perm, const double* __restrict__ w,
                                                int64_t n, int R, cpx<T>* __restrict__ a, int64_t n_src) {
  gather_one<T>((int64_t)blockIdx.x * TPB + threadIdx.x, sigma, dtype, conj_in, perm, w, n, R, a, n_src);
}

// Plans with separate targets: u[t, r] = uext[n_src + t, r] (caller order).
__global__ __launch_bounds__(TPB) void k_copy_targets(const void* __restrict__ uext, int64_t n_src, int64_t nt,
                                                      int R, int dtype, void* __restrict__ u) {
  const int64_t q = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (q >= nt * R) return;
  if (dtype == IFGF_C128)
    reinterpret_cast<double2*>(u)[q] = reinterpret_cast<const double2*>(uext)[n_src * R + q];
  else
    reinterpret_cast<float2*>(u)[q] = reinterpret_cast<const float2*>(uext)[n_src * R + q];
}

// ---------------------------------------------------------------------------
// near field: one block per finest-level box B; targets = points of B,
// sources = points of the neighbour boxes (self included, the i == j term
// excluded).  Positions relative to B's centre in precision T.  With TR the
// transposed sum is formed: output j collects v_i K(x_i, x_j), whose normal
// is the one at the output point x_j.
// ---------------------------------------------------------------------------
template <int RG> struct NearChunk { static constexpr int N = RG == 1 ? 512 : 128; };

template <typename T, int RG, int BS> struct NearSmem {
  static constexpr int NC = NearChunk<RG>::N;
  T sx[NC][3];
  T sn[NC][3];
  cpx<T> sa[NC][RG];
  int sidx[NC];
  int noff[28], nbox[27];
  cpx<T> red[BS][RG];
};

// Near field of finest-level box b, right-hand sides r0 .. r0 + RG - 1, by a
// block of BS threads.
template <typename T, bool TR, int RG, int BS>
__device__ __forceinline__ void near_box(NearSmem<T, RG, BS>& sm, int b, int toff, int tcnt, int r0,
                                         const double* __restrict__ pts,
                                         const double* __restrict__ nrm, const cpx<T>* __restrict__ a, int R,
                                         const int* __restrict__ start, const int* __restrict__ nbr_off,
                                         const int* __restrict__ nbr, const double* __restrict__ centre, double k,
                                         double eta, int kind, cpx<T>* __restrict__ uacc) {
  constexpr int NC = NearChunk<RG>::N;
  auto& sx = sm.sx;
  auto& sn = sm.sn;
  auto& sa = sm.sa;
  auto& sidx = sm.sidx;
  auto& noff = sm.noff;
  auto& nbox = sm.nbox;
  auto& red = sm.red;
  const int t0 = start[b] + toff, nt = tcnt;
  const double c0 = centre[3 * b], c1 = centre[3 * b + 1], c2 = centre[3 * b + 2];
  const int nn = nbr_off[b + 1] - nbr_off[b];
  if (threadIdx.x == 0) {
    int acc = 0;
    for (int q = 0; q < nn; ++q) {
      int j = nbr[nbr_off[b] + q];
      nbox[q] = j;
      noff[q] = acc;
      acc += start[j + 1] - start[j];
    }
    noff[nn] = acc;
  }
  __syncthreads();
  const int nsrc = noff[nn];
  // lane mapping: TP targets per pass, S = BS / TP source slices (threads
  // with sl >= S stay idle).  A pass costs about nsrc / S pair evaluations
  // per thread plus the staging of the sources (about half a pair per
  // source and block thread), so of the pass counts p from ceil(nt / BS) on
  // the one with the least p (1/S + 1/(2 BS)) is taken, TP = ceil(nt / p).
  int TP = 1, S = BS;
  {
    float best = 3.0e38f;
    const int p0 = max(1, (nt + BS - 1) / BS);
    for (int p = p0; p < p0 + 8; ++p) {
      const int tp = max(1, (nt + p - 1) / p);
      const int s = BS / tp;
      const float c = (float)p * (1.0f / (float)s + 0.5f / (float)BS);
      if (c < best) {
        best = c;
        TP = tp;
        S = s;
      }
    }
  }
  const int tl = threadIdx.x % TP, sl = threadIdx.x / TP;
  const T kk = (T)k, ee = (T)eta;
  const T inv4pi = (T)(1.0 / (4.0 * IFGF_PI));
  for (int tb = 0; tb < nt; tb += TP) {
    const int ti = tb + tl;
    const bool tv = ti < nt && sl < S;
    T x0 = 0, x1 = 0, x2 = 0, m0 = 0, m1 = 0, m2 = 0;
    if (tv) {
      x0 = (T)(pts[3 * (t0 + ti)] - c0);
      x1 = (T)(pts[3 * (t0 + ti) + 1] - c1);
      x2 = (T)(pts[3 * (t0 + ti) + 2] - c2);
      if (TR) {
        m0 = (T)nrm[3 * (t0 + ti)];
        m1 = (T)nrm[3 * (t0 + ti) + 1];
        m2 = (T)nrm[3 * (t0 + ti) + 2];
      }
    }
    cpx<T> acc[RG];
#pragma unroll
    for (int q = 0; q < RG; ++q) acc[q] = {0, 0};
    for (int cb = 0; cb < nsrc; cb += NC) {
      const int cn = min(NC, nsrc - cb);
      __syncthreads();
      for (int e = threadIdx.x; e < cn; e += BS) {
        int f = cb + e, q = 0;
        while (noff[q + 1] <= f) ++q;
        int j = start[nbox[q]] + (f - noff[q]);
        sidx[e] = j;
        sx[e][0] = (T)(pts[3 * j] - c0);
        sx[e][1] = (T)(pts[3 * j + 1] - c1);
        sx[e][2] = (T)(pts[3 * j + 2] - c2);
        sn[e][0] = (T)nrm[3 * j];
        sn[e][1] = (T)nrm[3 * j + 1];
        sn[e][2] = (T)nrm[3 * j + 2];
#pragma unroll
        for (int q2 = 0; q2 < RG; ++q2) sa[e][q2] = a[(int64_t)j * R + r0 + q2];
      }
      __syncthreads();
      if (tv) {
        const int self = t0 + ti;
        for (int e = sl; e < cn; e += S) {
          if (sidx[e] == self) continue;
          cpx<T> kv;
          if (kind == IFGF_KERNEL_CONSTANT) {
            kv = {1, 0};
          } else {
            T d0 = x0 - sx[e][0], d1 = x1 - sx[e][1], d2 = x2 - sx[e][2];
            T r2 = d0 * d0 + d1 * d1 + d2 * d2;
            T rr, ir;
            sqrt_rsqrt<T>(r2, &rr, &ir);
            // forward: <x_t - x_s, n_s>; transposed: <x_s - x_t, n_t>
            T dn = TR ? -(d0 * m0 + d1 * m1 + d2 * m2) * ir * ir
                      : (d0 * sn[e][0] + d1 * sn[e][1] + d2 * sn[e][2]) * ir * ir;
            T sn_, cs_;
            sincos_phase<T>(kk * rr, &sn_, &cs_);
            // G = e^{ikr}/(4 pi r);  K = G [ (1 - ikr) dn - i eta ]
            T g = inv4pi * ir;
            T pr = dn, pi = -(kk * rr * dn + ee);
            kv = {g * (cs_ * pr - sn_ * pi), g * (sn_ * pr + cs_ * pi)};
          }
#pragma unroll
          for (int q2 = 0; q2 < RG; ++q2) {
            const cpx<T> av = sa[e][q2];
            acc[q2].re += kv.re * av.re - kv.im * av.im;
            acc[q2].im += kv.re * av.im + kv.im * av.re;
          }
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int q2 = 0; q2 < RG; ++q2) red[threadIdx.x][q2] = acc[q2];
    __syncthreads();
    if (sl == 0 && tv) {
#pragma unroll
      for (int q2 = 0; q2 < RG; ++q2) {
        cpx<T> s2 = red[threadIdx.x][q2];
        for (int q = 1; q < S; ++q) {
          s2.re += red[threadIdx.x + q * TP][q2].re;
          s2.im += red[threadIdx.x + q * TP][q2].im;
        }
        uacc[(int64_t)(t0 + ti) * R + r0 + q2] = s2;
      }
    }
  }
}

// One block per work item (box, first target, target count): boxes with
// many points are split so that the blocks carry similar work.
template <typename T, bool TR, int RG>
__global__ __launch_bounds__(TPB) void k_near(const int4* __restrict__ work, const double* __restrict__ pts,
                                              const double* __restrict__ nrm, const cpx<T>* __restrict__ a, int R,
                                              const int* __restrict__ start, const int* __restrict__ nbr_off,
                                              const int* __restrict__ nbr, const double* __restrict__ centre,
                                              double k, double eta, int kind, cpx<T>* __restrict__ uacc) {
  __shared__ NearSmem<T, RG, TPB> sm;
  const int4 wk = work[xcd_block(blockIdx.x, gridDim.x)];
  near_box<T, TR, RG, TPB>(sm, wk.x, wk.y, wk.z, blockIdx.y * RG, pts, nrm, a, R, start, nbr_off, nbr, centre, k,
                           eta, kind, uacc);
}

// ---------------------------------------------------------------------------
// leaf factors: one block per finest-level box, items (relevant cone, node).
// W_c at node x = y0 + (h/s) e for a source y = y0 + h u:
//   v = e - s u, |v|^2 = 1 + s (s|u|^2 - 2<e,u>),
//   k r (|v| - 1) = k h (s|u|^2 - 2<e,u>) / (|v| + 1)   (bounded phase)
//   W_c = E1 [ s <v,n> / (h |v|^3) - i ( k <v,n> / |v|^2 + eta / |v| ) ]
// ---------------------------------------------------------------------------
template <int RG> struct LeafChunk { static constexpr int N = RG == 1 ? 256 : 64; };

template <typename T, int RG> struct LeafSmem {
  static constexpr int LC = LeafChunk<RG>::N;
  T su[LC][3];
  T sn[LC][3];
  T suu[LC], sun[LC];
  cpx<T> sa[LC][RG];
};

// Leaf factors of finest-level box b, right-hand sides r0 .. r0 + RG - 1, by
// a block of BS threads.
template <typename T, int PS, int PA, int RG, int BS>
__device__ __forceinline__ void leaf_box(LeafSmem<T, RG>& sm, int b, int i0, int icnt, int r0,
                                         const double* __restrict__ pts,
                                         const double* __restrict__ nrm, const cpx<T>* __restrict__ a, int R,
                                         const int* __restrict__ start, const double* __restrict__ centre,
                                         const int* __restrict__ slot_off, const int* __restrict__ rel_cone,
                                         const LevelGeom& g, const ChebTab& ct, double k, double eta, int kind,
                                         cpx<T>* __restrict__ Fn, cpx<T>* fv = nullptr) {
  constexpr int P = PS * PA * PA;
  constexpr int LC = LeafChunk<RG>::N;
  auto& su = sm.su;
  auto& sn = sm.sn;
  auto& suu = sm.suu;
  auto& sun = sm.sun;
  auto& sa = sm.sa;
  const int s0 = slot_off[b], ncn = slot_off[b + 1] - s0;
  const int p0 = start[b], np = start[b + 1] - p0;
  const double c0 = centre[3 * b], c1 = centre[3 * b + 1], c2 = centre[3 * b + 2];
  const double invh = 1.0 / g.h;
  const T kk = (T)k, ee = (T)eta, kh = (T)(k * g.h), ih = (T)invh;
  const int i1 = min(ncn * P, i0 + icnt);   // this block's (cone, node) items: i0 .. i1 - 1
  // sources of the box, relative to its centre in units of h, staged in LDS
  auto stage = [&](int cb, int cn) {
    for (int q = threadIdx.x; q < cn; q += BS) {
        int j = p0 + cb + q;
        T u0 = (T)((pts[3 * j] - c0) * invh), u1 = (T)((pts[3 * j + 1] - c1) * invh),
          u2 = (T)((pts[3 * j + 2] - c2) * invh);
        T n0 = (T)nrm[3 * j], n1 = (T)nrm[3 * j + 1], n2 = (T)nrm[3 * j + 2];
        su[q][0] = u0;
        su[q][1] = u1;
        su[q][2] = u2;
        sn[q][0] = n0;
        sn[q][1] = n1;
        sn[q][2] = n2;
        suu[q] = u0 * u0 + u1 * u1 + u2 * u2;
        sun[q] = u0 * n0 + u1 * n1 + u2 * n2;
#pragma unroll
        for (int q2 = 0; q2 < RG; ++q2) sa[q][q2] = a[(int64_t)j * R + r0 + q2];
    }
  };
  // a box's sources usually fit in one chunk: then they are staged once for
  // all passes over its (cone, node) items
  const bool once = np <= LC;
  if (once) {
    __syncthreads();
    stage(0, np);
    __syncthreads();
  }
  for (int ib = i0; ib < i1; ib += BS) {
    const int it = ib + threadIdx.x;
    const bool valid = it < i1;
    T e[3] = {0, 0, 0}, s = 0;
    if (valid) {
      int cs = it / P, node = it % P;
      int ai = node / (PA * PA), bi = (node / PA) % PA, ci = node % PA;
      int cid = rel_cone[s0 + cs];
      if constexpr (Prec<T>::f32) node_dir32(cid, ai, bi, ci, g, ct, e, &s);
      else node_dir64(cid, ai, bi, ci, g, ct, e, &s);
    }
    cpx<T> acc[RG];
#pragma unroll
    for (int q2 = 0; q2 < RG; ++q2) acc[q2] = {0, 0};
    for (int cb = 0; cb < np; cb += LC) {
      const int cn = min(LC, np - cb);
      if (!once) {
        __syncthreads();
        stage(cb, cn);
        __syncthreads();
      }
      if (valid) {
        for (int q = 0; q < cn; ++q) {
          cpx<T> W;
          if (kind == IFGF_KERNEL_CONSTANT) {
            W = {1, 0};
          } else {
            T eu = e[0] * su[q][0] + e[1] * su[q][1] + e[2] * su[q][2];
            T en = e[0] * sn[q][0] + e[1] * sn[q][1] + e[2] * sn[q][2];
            T qq = s * suu[q] - (T)2 * eu;
            T nv, inv;
            sqrt_rsqrt<T>((T)1 + s * qq, &nv, &inv);
            T ph = kh * qq * rcp_t<T>(nv + (T)1);
            T sp, cp;
            // |ph| <= k h (h: the box's half diagonal, k h = 2.7 for leaves
            // of half a wavelength): in FP32 the hardware sine and cosine,
            // absolute error about 1.5e-7 + 8.7e-8 k h
            if constexpr (Prec<T>::f32) sincos_hw(ph, &sp, &cp);
            else sincos_phase<T>(ph, &sp, &cp);
            T vn = en - s * sun[q];
            T A = vn * s * inv * inv * inv * ih;
            T B = kk * vn * inv * inv + ee * inv;
            W = {cp * A + sp * B, sp * A - cp * B};
          }
#pragma unroll
          for (int q2 = 0; q2 < RG; ++q2) {
            const cpx<T> av = sa[q][q2];
            acc[q2].re += W.re * av.re - W.im * av.im;
            acc[q2].im += W.re * av.im + W.im * av.re;
          }
        }
      }
    }
    if (valid) {
      if (fv) {   // one RHS: the node values go to LDS only (the caller turns them into coefficients)
        fv[it - i0] = acc[0];
      } else {
#pragma unroll
        for (int q2 = 0; q2 < RG; ++q2) Fn[((int64_t)s0 * P + it) * R + r0 + q2] = acc[q2];
      }
    }
  }
}

template <typename T, int PS, int PA, int BS>
__device__ __forceinline__ void lds_coeffs_store(cpx<T>* v, cpx<T>* t, int nc, const T* ms, const T* ma,
                                                 cpx<T>* __restrict__ out, int R, int r);

// One block per work item (box, first item, item count): a box's (cone,
// node) items are split into chunks of whole cones so that the blocks carry
// similar work.  With FUSE (one RHS) the block also turns its cones' node
// values into Chebyshev coefficients in LDS and writes them to Fc.
template <typename T, int PS, int PA, int RG, bool FUSE>
__global__ __launch_bounds__(TPB) void k_leaf(const int4* __restrict__ work, const double* __restrict__ pts,
                                              const double* __restrict__ nrm, const cpx<T>* __restrict__ a, int R,
                                              const int* __restrict__ start, const double* __restrict__ centre,
                                              const int* __restrict__ slot_off, const int* __restrict__ rel_cone,
                                              LevelGeom g, ChebTab ct, double k, double eta, int kind,
                                              cpx<T>* __restrict__ Fn, const T* __restrict__ Ms,
                                              const T* __restrict__ Ma, cpx<T>* __restrict__ Fc) {
  constexpr int P = PS * PA * PA;
  constexpr int NCF = FUSE ? (kLeafChunk / P > 0 ? kLeafChunk / P : 1) : 1;
  __shared__ LeafSmem<T, RG> sm;
  __shared__ cpx<T> fv[FUSE ? NCF * P : 1], ft[FUSE ? NCF * P : 1];
  __shared__ T fms[PS * PS], fma_[PA * PA];
  const int4 wk = work[xcd_block(blockIdx.x, gridDim.x)];
  if (FUSE) {
    if (threadIdx.x < PS * PS) fms[threadIdx.x] = Ms[threadIdx.x];
    if (threadIdx.x < PA * PA) fma_[threadIdx.x] = Ma[threadIdx.x];
  }
  leaf_box<T, PS, PA, RG, TPB>(sm, wk.x, wk.y, wk.z, blockIdx.y * RG, pts, nrm, a, R, start, centre, slot_off,
                               rel_cone, g, ct, k, eta, kind, Fn, FUSE ? fv : nullptr);
  if constexpr (FUSE) {
    __syncthreads();
    const int ncn = slot_off[wk.x + 1] - slot_off[wk.x];
    const int c0 = wk.y / P, nc = min(ncn * P, wk.y + wk.z) / P - c0;
    lds_coeffs_store<T, PS, PA, TPB>(fv, ft, nc, fms, fma_, Fc + ((int64_t)slot_off[wk.x] + c0) * P, 1, 0);
  }
}

// ---------------------------------------------------------------------------
// node values -> coefficients: c_ijl = sum_abc Ms[i][a] Ma[j][b] Ma[l][c] v_abc,
// coeff_cones(P) cones per block (one cone of 144 coefficients is too small
// to fill a block), three separable passes through LDS.  With TR the
// transposed map (Ms^T, Ma^T) is applied.  Fn may equal Fc (in place).
// ---------------------------------------------------------------------------
constexpr int coeff_cones(int P) { return P <= 160 ? 8 : 1; }

// The three passes over nt = (cones) x P node values in v0 (LDS), the
// matrices in ms, ma; the result to Fc (cones from c0, RHS r of R).
template <typename T, int PS, int PA>
__device__ __forceinline__ void coeffs_passes(cpx<T>* v0, cpx<T>* v1, const T* ms, const T* ma, int nt, int c0,
                                              int R, int r, cpx<T>* __restrict__ Fc) {
  constexpr int P = PS * PA * PA;
  const int t0 = threadIdx.x;
  for (int t = t0; t < nt; t += TPB) {  // over a (s)
    const int cb = t / P * P, u = t % P;
    const int i = u / (PA * PA), j = (u / PA) % PA, l = u % PA;
    cpx<T> s = {0, 0};
    for (int q = 0; q < PS; ++q) {
      cpx<T> x = v0[cb + (q * PA + j) * PA + l];
      s.re += ms[i * PS + q] * x.re;
      s.im += ms[i * PS + q] * x.im;
    }
    v1[t] = s;
  }
  __syncthreads();
  for (int t = t0; t < nt; t += TPB) {  // over b (theta)
    const int cb = t / P * P, u = t % P;
    const int i = u / (PA * PA), j = (u / PA) % PA, l = u % PA;
    cpx<T> s = {0, 0};
    for (int q = 0; q < PA; ++q) {
      cpx<T> x = v1[cb + (i * PA + q) * PA + l];
      s.re += ma[j * PA + q] * x.re;
      s.im += ma[j * PA + q] * x.im;
    }
    v0[t] = s;
  }
  __syncthreads();
  for (int t = t0; t < nt; t += TPB) {  // over c (phi)
    const int cb = t / P * P, u = t % P;
    const int i = u / (PA * PA), j = (u / PA) % PA;
    const int l = u % PA;
    cpx<T> s = {0, 0};
    for (int q = 0; q < PA; ++q) {
      cpx<T> x = v0[cb + (i * PA + j) * PA + q];
      s.re += ma[l * PA + q] * x.re;
      s.im += ma[l * PA + q] * x.im;
    }
    Fc[((int64_t)c0 * P + t) * R + r] = s;
  }
}

template <typename T, int PS, int PA, bool TR>
__global__ __launch_bounds__(TPB) void k_coeffs(const cpx<T>* __restrict__ Fn, int nrel, int R,
                                                const T* __restrict__ Ms, const T* __restrict__ Ma,
                                                cpx<T>* __restrict__ Fc) {
  constexpr int P = PS * PA * PA;
  constexpr int NC = coeff_cones(P);
  __shared__ cpx<T> v0[NC * P], v1[NC * P];
  __shared__ T ms[PS * PS], ma[PA * PA];
  const int c0 = blockIdx.x * NC, r = blockIdx.y, t0 = threadIdx.x;
  const int nc = min(NC, nrel - c0);
  const int nt = nc * P;
  if (t0 < PS * PS) ms[t0] = TR ? Ms[(t0 % PS) * PS + t0 / PS] : Ms[t0];
  if (t0 < PA * PA) ma[t0] = TR ? Ma[(t0 % PA) * PA + t0 / PA] : Ma[t0];
  for (int t = t0; t < nt; t += TPB) v0[t] = Fn[((int64_t)c0 * P + t) * R + r];
  __syncthreads();
  coeffs_passes<T, PS, PA>(v0, v1, ms, ma, nt, c0, R, r, Fc);
}

// Upward pass from a pair list, second kernel: node (s, j) of level d is the
// sum of its pair values (pairs base[s] + j * nch + t, t over the children in
// order; val in sorted order, pos[] the sorted position), then the level's
// coefficients as k_coeffs (one RHS).
template <typename T, int PS, int PA> struct UpsumSmem {
  static constexpr int P = PS * PA * PA, NC = coeff_cones(P);
  cpx<T> v0[NC * P], v1[NC * P];
  T ms[PS * PS], ma[PA * PA];
};

// The cones c0 .. c0 + NC - 1 (NC = coeff_cones(P)) of one block of TPB threads.
template <typename T, int PS, int PA>
__device__ __forceinline__ void upsum_chunk(UpsumSmem<T, PS, PA>& sm, int c0, const int* __restrict__ base,
                                            const int* __restrict__ pos, const cpx<T>* __restrict__ val, int nrel,
                                            const T* __restrict__ Ms, const T* __restrict__ Ma,
                                            cpx<T>* __restrict__ Fc) {
  constexpr int P = PS * PA * PA;
  constexpr int NC = coeff_cones(P);
  cpx<T>* v0 = sm.v0;
  const int t0 = threadIdx.x;
  const int nc = min(NC, nrel - c0);
  const int nt = nc * P;
  if (t0 < PS * PS) sm.ms[t0] = Ms[t0];
  if (t0 < PA * PA) sm.ma[t0] = Ma[t0];
  for (int t = t0; t < nt; t += TPB) {
    const int sc = c0 + t / P, j = t % P;
    const int b0 = base[sc], nch = (base[sc + 1] - b0) / P;
    const int* pp = pos + b0 + j * nch;
    cpx<T> a = {0, 0};
    for (int c = 0; c < nch; ++c) {
      const cpx<T> v = val[pp[c]];
      a.re += v.re;
      a.im += v.im;
    }
    v0[t] = a;
  }
  __syncthreads();
  coeffs_passes<T, PS, PA>(v0, sm.v1, sm.ms, sm.ma, nt, c0, 1, 0, Fc);
}

template <typename T, int PS, int PA>
__global__ __launch_bounds__(TPB) void k_upsum_coeffs(const int* __restrict__ base, const int* __restrict__ pos,
                                                      const cpx<T>* __restrict__ val, int nrel,
                                                      const T* __restrict__ Ms, const T* __restrict__ Ma,
                                                      cpx<T>* __restrict__ Fc) {
  __shared__ UpsumSmem<T, PS, PA> sm;
  upsum_chunk<T, PS, PA>(sm, xcd_block(blockIdx.x, gridDim.x) * coeff_cones(PS * PA * PA), base, pos, val, nrel, Ms,
                         Ma, Fc);
}

// Node values -> coefficients for RG right-hand sides at once (layout
// [slot][P][R]): one block per (cone, RHS group); the P x RG tile is read and
// written in rows of RG consecutive values.
template <typename T, int PS, int PA, int RG>
__global__ __launch_bounds__(TPB) void k_coeffs_rg(const cpx<T>* __restrict__ Fn, int R, const T* __restrict__ Ms,
                                                   const T* __restrict__ Ma, cpx<T>* __restrict__ Fc) {
  constexpr int P = PS * PA * PA;
  constexpr int N = P * RG;
  __shared__ cpx<T> v0[N], v1[N];
  __shared__ T ms[PS * PS], ma[PA * PA];
  const int sl = blockIdx.x, r0 = blockIdx.y * RG;
  const int t = threadIdx.x;
  if (t < PS * PS) ms[t] = Ms[t];
  if (t < PA * PA) ma[t] = Ma[t];
  const cpx<T>* src = Fn + (int64_t)sl * P * R + r0;
  for (int q = t; q < N; q += TPB) v0[q] = src[(int64_t)(q / RG) * R + q % RG];
  __syncthreads();
  for (int q = t; q < N; q += TPB) {   // over a (s)
    const int j = q / RG, rr = q % RG, i = j / (PA * PA), jj = (j / PA) % PA, l = j % PA;
    cpx<T> acc = {0, 0};
    for (int k = 0; k < PS; ++k) {
      const cpx<T> x = v0[((k * PA + jj) * PA + l) * RG + rr];
      acc.re += ms[i * PS + k] * x.re;
      acc.im += ms[i * PS + k] * x.im;
    }
    v1[q] = acc;
  }
  __syncthreads();
  for (int q = t; q < N; q += TPB) {   // over b (theta)
    const int j = q / RG, rr = q % RG, i = j / (PA * PA), jj = (j / PA) % PA, l = j % PA;
    cpx<T> acc = {0, 0};
    for (int k = 0; k < PA; ++k) {
      const cpx<T> x = v1[((i * PA + k) * PA + l) * RG + rr];
      acc.re += ma[jj * PA + k] * x.re;
      acc.im += ma[jj * PA + k] * x.im;
    }
    v0[q] = acc;
  }
  __syncthreads();
  cpx<T>* dst = Fc + (int64_t)sl * P * R + r0;
  for (int q = t; q < N; q += TPB) {   // over c (phi)
    const int j = q / RG, rr = q % RG, i = j / (PA * PA), jj = (j / PA) % PA, l = j % PA;
    cpx<T> acc = {0, 0};
    for (int k = 0; k < PA; ++k) {
      const cpx<T> x = v0[((i * PA + jj) * PA + k) * RG + rr];
      acc.re += ma[l * PA + k] * x.re;
      acc.im += ma[l * PA + k] * x.im;
    }
    dst[(int64_t)j * R + rr] = acc;
  }
}

// ---------------------------------------------------------------------------
// Interpolant evaluation with wave-uniform coefficients.
// ---------------------------------------------------------------------------
// sum_ijl C_ijl T_i(ts) T_j(tt) T_l(tp) with C in LDS (interleaved re, im).
// T_0 = 1, so every partial sum starts from its T_0 term.
template <typename T, int PS, int PA>
__device__ __forceinline__ cpx<T> contract_lds(const T* C, const T* Ts, const T* Tt, const T* Tp) {
  cpx<T> acc;
#pragma unroll
  for (int i = 0; i < PS; ++i) {
    cpx<T> h;
#pragma unroll
    for (int j = 0; j < PA; ++j) {
      const int q0 = (i * PA + j) * PA;
      cpx<T> g = {C[2 * q0], C[2 * q0 + 1]};
#pragma unroll
      for (int l = 1; l < PA; ++l) {
        g.re += C[2 * (q0 + l)] * Tp[l];
        g.im += C[2 * (q0 + l) + 1] * Tp[l];
      }
      if (j == 0) {
        h = g;
      } else {
        h.re += g.re * Tt[j];
        h.im += g.im * Tt[j];
      }
    }
    if (i == 0) {
      acc = h;
    } else {
      acc.re += h.re * Ts[i];
      acc.im += h.im * Ts[i];
    }
  }
  return acc;
}

// For every lane with slot >= 0, evaluates the interpolant of cone `slot` of
// F (coefficient layout [slot][P][R], right-hand side r) at (ts, tt, tp).
// All 64 lanes of the wave must call it together (lanes without work pass
// slot = -1).  The wave serves one slot at a time: its lanes copy that cone's
// P coefficients into the wave's LDS buffer `wbuf` (2P values, coalesced
// reads issued together) and the lanes holding the slot contract against
// it with wave-uniform LDS reads.  LDS operations of a wave complete in
// order, so the copy is visible to the reads that follow it.
template <typename T, int PS, int PA>
__device__ __forceinline__ cpx<T> eval_uniform(const cpx<T>* __restrict__ F, int slot, int R, int r, T ts, T tt,
                                               T tp, T* wbuf) {
  constexpr int P = PS * PA * PA;
  constexpr int NCP = (P + 63) / 64;
  T Ts[PS], Tt[PA], Tp[PA];
  cheb_T<T, PS>(ts, Ts);
  cheb_T<T, PA>(tt, Tt);
  cheb_T<T, PA>(tp, Tp);
  cpx<T> out = {0, 0};
  const int lane = threadIdx.x & 63;
  cpx<T>* wb = reinterpret_cast<cpx<T>*>(wbuf);
  uint64_t pending = __ballot(slot >= 0);
  while (pending) {
    const int lead = first_lane(pending);
    const int su = __builtin_amdgcn_readfirstlane(__shfl(slot, lead, 64));
    const bool mine = slot == su;
    pending &= ~__ballot(mine);
    const cpx<T>* src = F + (int64_t)su * P * R + r;
    cpx<T> v[NCP];
    if (R == 1) {
#pragma unroll
      for (int j = 0; j < NCP; ++j)
        if (lane + 64 * j < P) v[j] = src[lane + 64 * j];
    } else {
#pragma unroll
      for (int j = 0; j < NCP; ++j)
        if (lane + 64 * j < P) v[j] = src[(int64_t)(lane + 64 * j) * R];
    }
#pragma unroll
    for (int j = 0; j < NCP; ++j)
      if (lane + 64 * j < P) wb[lane + 64 * j] = v[j];
    __builtin_amdgcn_wave_barrier();
    if (mine) out = contract_lds<T, PS, PA>(wbuf, Ts, Tt, Tp);
    __builtin_amdgcn_wave_barrier();
  }
  return out;
}

#include "row_stage1.inc"

// Minimum of v over the 16 lanes of each row.
__device__ __forceinline__ int row_min16(int v) {
  v = min(v, __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, true));    // quad_perm [1,0,3,2]
  v = min(v, __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, true));    // quad_perm [2,3,0,1]
  v = min(v, __builtin_amdgcn_mov_dpp(v, 0x141, 0xF, 0xF, true));   // row_half_mirror
  v = min(v, __builtin_amdgcn_mov_dpp(v, 0x140, 0xF, 0xF, true));   // row_mirror
  return v;
}

// Lane nl (0..15) of a row loads its share of one cone's 2P values.  FP32:
// float 64 m + 4 nl + e into register 4 m + e; FP64: double 32 m + 2 nl + e
// into register 2 m + e.  Registers past the cone stay 0.
template <int P, int NREG>
__device__ __forceinline__ void row_load_cone(const double* __restrict__ src, int nl, double (&c)[NREG]) {
#pragma unroll
  for (int m = 0; m < NREG / 2; ++m) {
    const int off = 32 * m + 2 * nl;
    double2 v = make_double2(0.0, 0.0);
    if (off + 2 <= 2 * P) v = *reinterpret_cast<const double2*>(src + off);
    c[2 * m] = v.x;
    c[2 * m + 1] = v.y;
  }
}

template <int P, int NREG>
__device__ __forceinline__ void row_load_cone(const float* __restrict__ src, int nl, float (&c)[NREG]) {
#pragma unroll
  for (int m = 0; m < NREG / 4; ++m) {
    const int off = 64 * m + 4 * nl;
    if constexpr (P % 2 == 0) {   // cone base 16-byte aligned
      float4 v = {0, 0, 0, 0};
      if (off + 4 <= 2 * P) v = *reinterpret_cast<const float4*>(src + off);
      c[4 * m] = v.x;
      c[4 * m + 1] = v.y;
      c[4 * m + 2] = v.z;
      c[4 * m + 3] = v.w;
    } else {                      // 8-byte aligned
      float2 a = {0, 0}, b = {0, 0};
      if (off + 2 <= 2 * P) a = *reinterpret_cast<const float2*>(src + off);
      if (off + 4 <= 2 * P) b = *reinterpret_cast<const float2*>(src + off + 2);
      c[4 * m] = a.x;
      c[4 * m + 1] = a.y;
      c[4 * m + 2] = b.x;
      c[4 * m + 3] = b.y;
    }
  }
}


// Radial indices per row-stage pass: the whole cone where a stage for the
// order is generated, else pairs of radial indices with the (2, P_ang) stage
// (the cone's coefficients of two consecutive radial indices are contiguous);
// 0 if neither exists.
template <typename T, int PS, int PA> constexpr int row_chunk() {
  if constexpr (RowStage1<T, PS, PA>::ok) return PS;
  else if constexpr (PS % 2 == 0 && RowStage1<T, 2, PA>::ok) return 2;
  else return 0;
}
template <typename T, int PS, int PA> constexpr bool rows_ok() { return row_chunk<T, PS, PA>() > 0; }

// The interpolant of one cone (2P values at `cone`, held across the row's 16
// lanes pass by pass) at this lane's Chebyshev values: sum_a Ts[a] sum_b Tt[b]
// sum_c C[a][b][c] Tp[c], the c sum by DPP broadcast (RowStage1).  All lanes
// of the row call it with the same cone.
// One row-stage pass: for the CS radial indices whose coefficients start at
// `chunk`, h[a] = sum_b Tt[b] sum_c C[a][b][c] Tp[c].
template <typename T, int CS, int PA>
__device__ __forceinline__ void row_pass(const T* __restrict__ chunk, int nl, const T (&Tt)[PA], const T (&Tp)[PA],
                                         T (&h_re)[CS], T (&h_im)[CS]) {
  using S1 = RowStage1<T, CS, PA>;
  constexpr int NREG = S1::NREG;
  T c[NREG];
  row_load_cone<CS * PA * PA, NREG>(chunk, nl, c);
  T D[2 * CS * PA];
  S1::run(c, Tp, D);
#pragma unroll
  for (int a = 0; a < CS; ++a) {
    h_re[a] = D[2 * a * PA];
    h_im[a] = D[2 * a * PA + 1];
#pragma unroll
    for (int b = 1; b < PA; ++b) {
      h_re[a] += D[2 * (a * PA + b)] * Tt[b];
      h_im[a] += D[2 * (a * PA + b) + 1] * Tt[b];
    }
  }
}

// The interpolant of one cone (2P values at `cone`, held across the row's 16
// lanes pass by pass) at this lane's Chebyshev values: sum_a Ts[a] sum_b Tt[b]
// sum_c C[a][b][c] Tp[c], the c sum by DPP broadcast (RowStage1).  All lanes
// of the row call it with the same cone.
template <typename T, int PS, int PA>
__device__ __forceinline__ void row_contract(const T* __restrict__ cone, int nl, const T (&Ts)[PS], const T (&Tt)[PA],
                                             const T (&Tp)[PA], T& v_re, T& v_im) {
  constexpr int CS = row_chunk<T, PS, PA>();
  T h_re[CS], h_im[CS];
  row_pass<T, CS, PA>(cone, nl, Tt, Tp, h_re, h_im);
  v_re = h_re[0];
  v_im = h_im[0];
#pragma unroll
  for (int a = 1; a < CS; ++a) {
    v_re += h_re[a] * Ts[a];
    v_im += h_im[a] * Ts[a];
  }
  if constexpr (CS < PS) {   // the further radial chunks, one pass each
    constexpr int PC = CS * PA * PA;
#pragma unroll 1
    for (int h = 1; h < PS / CS; ++h) {
      row_pass<T, CS, PA>(cone + (int64_t)h * 2 * PC, nl, Tt, Tp, h_re, h_im);
#pragma unroll
      for (int a = 0; a < CS; ++a) {
        T ta = Ts[0];
#pragma unroll
        for (int m = 1; m < PS; ++m)
          if (m == h * CS + a) ta = Ts[m];
        v_re += h_re[a] * ta;
        v_im += h_im[a] * ta;
      }
    }
  }
}

// For every lane with slot >= 0, the interpolant of cone `slot` of F (one
// right-hand side, layout [slot][P]) at (ts, tt, tp), by rows: each row of
// 16 lanes loads one cone across its lanes and contracts with the
// coefficients broadcast by DPP (RowStage1); lanes of the row that need
// another cone take a further round.  All 64 lanes of the wave call it
// together (lanes without work pass slot = -1).
template <typename T, int PS, int PA>
__device__ __forceinline__ cpx<T> eval_rows(const cpx<T>* __restrict__ Fc, int slot, T ts, T tt, T tp) {
  constexpr int P = PS * PA * PA;
  constexpr int NONE = 0x7fffffff;
  const T* F = reinterpret_cast<const T*>(Fc);
  const int nl = threadIdx.x & 15;
  T Ts[PS], Tt[PA], Tp[PA];
  cheb_T<T, PS>(ts, Ts);
  cheb_T<T, PA>(tt, Tt);
  cheb_T<T, PA>(tp, Tp);
  cpx<T> out = {0, 0};
  bool pend = slot >= 0;
  while (__ballot(pend)) {
    const int su = row_min16(pend ? slot : NONE);
    T v_re, v_im;
    row_contract<T, PS, PA>(F + (int64_t)(su == NONE ? 0 : su) * (2 * P), nl, Ts, Tt, Tp, v_re, v_im);
    if (pend && slot == su) {
      out = {v_re, v_im};
      pend = false;
    }
  }
  return out;
}

// ---------------------------------------------------------------------------
// upward pass d -> d-1 (Algorithm 1, parent-node update), fused with the
// node-value -> coefficient transform of level d-1.
//
// One block per work item = (parent box P, up to PropShape::CH consecutive
// relevant cones of P).  For each child B of P the block
//   A. locates every node of its cones in B's cone segments (slot, local
//      coordinates, ratio K(x,y_B)/K(x,y_P)),
//   B. buckets the nodes by child slot in LDS (hash table + counting sort),
//   C. evaluates the child interpolants in bucket order, so that the lanes of
//      a wave mostly share one slot and read its coefficients once, and
//      accumulates ratio * value into the node's LDS accumulator.
// Finally the node values of the chunk are turned into Chebyshev
// coefficients in LDS and written to level d-1.
// ---------------------------------------------------------------------------
// Chunking of the upward pass: CH cones of P = P_s P_ang^2 nodes per block
// of BS threads, chosen so that CH * P (nearly) fills whole passes.
template <int P> struct PropShape;
template <> struct PropShape<75> { static constexpr int CH = 10, BS = 256; };    // 750 nodes, 3 x 256
template <> struct PropShape<144> { static constexpr int CH = 4, BS = 192; };    // 576 nodes, 3 x 192
template <> struct PropShape<512> { static constexpr int CH = 1, BS = 256; };    // 512 nodes, 2 x 256

template <typename T> struct PropGeomT;
template <> struct PropGeomT<float> { using P = PropF; };
template <> struct PropGeomT<double> { using P = Prop64; };

__device__ __forceinline__ uint32_t hash_slot(int slot, int bits) {
  return ((uint32_t)slot * 2654435761u) >> (32 - bits);
}

// In-LDS exclusive scan of n counts, in place.
template <int BS>
__device__ __forceinline__ void block_scan_inplace(int* a, int n, int* wsum) {
  const int per = (n + BS - 1) / BS;
  const int base = threadIdx.x * per;
  const int cnt = max(0, min(per, n - base));
  int tot = 0;
  for (int i = 0; i < cnt; ++i) tot += a[base + i];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  int x = tot;
  for (int off = 1; off < 64; off <<= 1) {
    int y = __shfl_up(x, off, 64);
    if (lane >= off) x += y;
  }
  if (lane == 63) wsum[wid] = x;
  __syncthreads();
  int run = x - tot;
  for (int w = 0; w < wid; ++w) run += wsum[w];
  for (int i = 0; i < cnt; ++i) {
    int v = a[base + i];
    a[base + i] = run;
    run += v;
  }
  __syncthreads();
}

// Chebyshev transform of nc cones of node values in LDS (in: v, scratch: t),
// written to global coefficients out[((cone) * P + j) * R + r].
template <typename T, int PS, int PA, int BS>
__device__ __forceinline__ void lds_coeffs_store(cpx<T>* v, cpx<T>* t, int nc, const T* ms, const T* ma,
                                                 cpx<T>* __restrict__ out, int R, int r) {
  constexpr int P = PS * PA * PA;
  const int tot = nc * P;
  for (int q = threadIdx.x; q < tot; q += BS) {
    const int c = q / P, j = q % P, i = j / (PA * PA), jj = (j / PA) % PA, l = j % PA;
    cpx<T> acc = {0, 0};
    for (int k = 0; k < PS; ++k) {
      cpx<T> x = v[c * P + (k * PA + jj) * PA + l];
      acc.re += ms[i * PS + k] * x.re;
      acc.im += ms[i * PS + k] * x.im;
    }
    t[q] = acc;
  }
  __syncthreads();
  for (int q = threadIdx.x; q < tot; q += BS) {
    const int c = q / P, j = q % P, i = j / (PA * PA), jj = (j / PA) % PA, l = j % PA;
    cpx<T> acc = {0, 0};
    for (int k = 0; k < PA; ++k) {
      cpx<T> x = t[c * P + (i * PA + k) * PA + l];
      acc.re += ma[jj * PA + k] * x.re;
      acc.im += ma[jj * PA + k] * x.im;
    }
    v[q] = acc;
  }
  __syncthreads();
  for (int q = threadIdx.x; q < tot; q += BS) {
    const int c = q / P, j = q % P, i = j / (PA * PA), jj = (j / PA) % PA, l = j % PA;
    cpx<T> acc = {0, 0};
    for (int k = 0; k < PA; ++k) {
      cpx<T> x = v[c * P + (i * PA + jj) * PA + k];
      acc.re += ma[l * PA + k] * x.re;
      acc.im += ma[l * PA + k] * x.im;
    }
    out[((int64_t)c * P + j) * R + r] = acc;
  }
}

// CB: the per-wave coefficient buffer of the LDS-staged evaluation (not
// needed by a single right-hand side with a row stage).
template <typename T, int PS, int PA, int BS_ = PropShape<PS * PA * PA>::BS, bool CB = true> struct PropSmem {
  static constexpr int P = PS * PA * PA;
  static constexpr int BS = BS_;
  static constexpr int NN = PropShape<P>::CH * P;
  static constexpr int HB = NN <= 256 ? 8 : (NN <= 512 ? 9 : (NN <= 1024 ? 10 : 11));   // 2^HB >= NN
  static constexpr int HT = 1 << HB;
  static_assert(HT >= NN, "the hash table must be able to hold every node");
  cpx<T> acc[NN], tmp[NN];
  T st[NN][3];            // local coordinates in the child cone
  int skey[NN];
  short sord[NN];
  int hkey[HT], hoff[HT];
  int wsum[BS / 64];
  T ms[PS * PS], ma[PA * PA];
  __align__(16) T cbuf[CB ? BS / 64 : 1][CB ? 2 * P : 4];
  // per cone of the item, (sin, cos) of its PA polar and PA azimuthal node
  // angles, and its PS node radii h / s
  T ang[PropShape<P>::CH][2 * PA][2];
  T rad[PropShape<P>::CH][PS];
};

// One work item wk = (parent box, first slot, end slot) of the upward pass,
// right-hand side r, by a block of BS threads (PropShape::BS in the
// standalone kernel).  ONE: a single right-hand side (R = 1 at compile time,
// contiguous cones).
template <typename T, int PS, int PA, bool ONE, int BS_ = PropShape<PS * PA * PA>::BS, bool CB = true>
__device__ __forceinline__ void prop_item(PropSmem<T, PS, PA, BS_, CB>& sm, int4 wk, int r, const int* __restrict__ rel_cone_up,
                                          const int* __restrict__ child_lo_up, const int* __restrict__ coords,
                                          const int* __restrict__ slot_c, const cpx<T>* __restrict__ Fc_c,
                                          const LevelGeom& gp, const LevelGeom& gc, const ChebTab& ct,
                                          const T* __restrict__ Ms, const T* __restrict__ Ma, double k, int kind,
                                          int R_, cpx<T>* __restrict__ Fc_up, int* __restrict__ err) {
  using S = PropSmem<T, PS, PA, BS_, CB>;
  constexpr int P = S::P;
  constexpr int BS = S::BS;
  constexpr int NN = S::NN;
  constexpr int HB = S::HB;
  constexpr int HT = S::HT;
  const int R = ONE ? 1 : R_;
  auto& acc = sm.acc;
  auto& tmp = sm.tmp;
  auto& st = sm.st;
  auto& skey = sm.skey;
  auto& sord = sm.sord;
  auto& hkey = sm.hkey;
  auto& hoff = sm.hoff;
  auto& wsum = sm.wsum;
  auto& ms = sm.ms;
  auto& ma = sm.ma;
  auto& cbuf = sm.cbuf;
  const int Pb = wk.x, s0 = wk.y, ncn = wk.z - wk.y;
  const int nn = ncn * P;
  if (threadIdx.x < PS * PS) ms[threadIdx.x] = Ms[threadIdx.x];
  if (threadIdx.x < PA * PA) ma[threadIdx.x] = Ma[threadIdx.x];
  // node angles and radii of the item's cones (the terms of node_rel32 / node_rel64)
  for (int t = threadIdx.x; t < ncn * (2 * PA + PS); t += BS) {
    const int c = t / (2 * PA + PS), j = t % (2 * PA + PS);
    int is, it, ip;
    cone_split(rel_cone_up[s0 + c], gp.nc, &is, &it, &ip);
    if constexpr (Prec<T>::f32) {
      if (j < PA)
        sincos_f(((float)it + ct.uaf[j]) * gp.daf, &sm.ang[c][j][0], &sm.ang[c][j][1]);
      else if (j < 2 * PA)
        sincos_f(((float)ip + ct.uaf[j - PA]) * gp.daf, &sm.ang[c][j][0], &sm.ang[c][j][1]);
      else
        sm.rad[c][j - 2 * PA] = gp.hf * rcp_f(((float)is + ct.usf[j - 2 * PA]) * gp.dsf);
    } else {
      if (j < PA)
        sincos(((double)it + ct.ua[j]) * gp.da, &sm.ang[c][j][0], &sm.ang[c][j][1]);
      else if (j < 2 * PA)
        sincos(((double)ip + ct.ua[j - PA]) * gp.da, &sm.ang[c][j][0], &sm.ang[c][j][1]);
      else
        sm.rad[c][j - 2 * PA] = gp.h / (((double)is + ct.us[j - 2 * PA]) * gp.ds);
    }
  }
  for (int q = threadIdx.x; q < nn; q += BS) acc[q] = {0, 0};
  for (int h = threadIdx.x; h < HT; h += BS) {
    hkey[h] = -1;
    hoff[h] = 0;
  }
  __syncthreads();

  const int B0 = child_lo_up[Pb], B1 = child_lo_up[Pb + 1];
  for (int B = B0; B < B1; ++B) {
    const int oct = (coords[3 * B] & 1) | ((coords[3 * B + 1] & 1) << 1) | ((coords[3 * B + 2] & 1) << 2);
    // A: locate each node in B's cones; count bucket sizes
    for (int q = threadIdx.x; q < nn; q += BS) {
      const int c = q / P, node = q % P;
      const int ai = node / (PA * PA), bi = (node / PA) % PA, ci = node % PA;
      T x[3], rp;
      typename PropGeomT<T>::P pr;
      {   // the node relative to the parent centre (node_rel32 / node_rel64) from the tabulated terms
        const T st = sm.ang[c][bi][0], ctt = sm.ang[c][bi][1];
        const T sp = sm.ang[c][PA + ci][0], cp = sm.ang[c][PA + ci][1];
        const T e0 = st * cp, e1 = st * sp;
        rp = sm.rad[c][ai];
        x[0] = rp * e0;
        x[1] = rp * e1;
        x[2] = rp * ctt;
      }
      if constexpr (Prec<T>::f32)
        pr = child_loc32(x, rp, oct, gc);
      else
        pr = child_loc64(x, rp, oct, gc);
      const int sl = slot_c[(int64_t)B * gc.ncone + pr.loc.cid];
      if (sl < 0) atomicOr(err, 2);
      st[q][0] = pr.loc.ts;
      st[q][1] = pr.loc.tt;
      st[q][2] = pr.loc.tp;
      tmp[q] = {pr.rp_over_rc, pr.dr};
      skey[q] = sl;
      const int hk = sl >= 0 ? sl : 0x7ffffffe;   // never the empty marker -1
      uint32_t h = hash_slot(hk, HB);
      while (true) {
        int prev = atomicCAS(&hkey[h], -1, hk);
        if (prev == -1 || prev == hk) break;
        h = (h + 1) & (HT - 1);
      }
      atomicAdd(&hoff[h], 1);
    }
    __syncthreads();
    block_scan_inplace<BS>(hoff, HT, wsum);
    // B: counting sort of the nodes by slot
    for (int q = threadIdx.x; q < nn; q += BS) {
      const int sl = skey[q];
      const int hk = sl >= 0 ? sl : 0x7ffffffe;
      uint32_t h = hash_slot(hk, HB);
      while (hkey[h] != hk) h = (h + 1) & (HT - 1);
      const int pos = atomicAdd(&hoff[h], 1);
      sord[pos] = (short)q;
    }
    __syncthreads();
    for (int h = threadIdx.x; h < HT; h += BS) {   // the table is free again; cleared for the next child
      hkey[h] = -1;
      hoff[h] = 0;
    }
    // C: evaluate in bucket order
    for (int qb = 0; qb < nn; qb += BS) {
      const int qq = qb + threadIdx.x;
      int n = -1, sl = -1;
      if (qq < nn) {
        n = sord[qq];
        sl = skey[n];
      }
      T ts = 0, tt = 0, tp = 0;
      if (n >= 0) {
        ts = st[n][0];
        tt = st[n][1];
        tp = st[n][2];
      }
      cpx<T> v;
      if constexpr (ONE && rows_ok<T, PS, PA>())
        v = eval_rows<T, PS, PA>(Fc_c, sl, ts, tt, tp);
      else if constexpr (CB)
        v = eval_uniform<T, PS, PA>(Fc_c, sl, R, r, ts, tt, tp, cbuf[threadIdx.x >> 6]);
      if (n >= 0 && sl >= 0) {
        T rr = tmp[n].re, dr = tmp[n].im;
        T c_, s_;
        if (kind == IFGF_KERNEL_CONSTANT) {
          c_ = 1;
          s_ = 0;
          rr = 1;
        } else {
          sincos_t<T>((T)k * dr, &s_, &c_);
        }
        const T rre = rr * c_, rim = rr * s_;
        acc[n].re += rre * v.re - rim * v.im;
        acc[n].im += rre * v.im + rim * v.re;
      }
    }
    __syncthreads();
  }
  lds_coeffs_store<T, PS, PA, BS>(acc, tmp, ncn, ms, ma, Fc_up + (int64_t)s0 * P * R, R, r);
}

template <typename T, int PS, int PA, bool ONE>
__global__ __launch_bounds__(PropShape<PS * PA * PA>::BS) __attribute__((amdgpu_waves_per_eu(3))) void k_prop(
    const int4* __restrict__ work, const int* __restrict__ rel_cone_up, const int* __restrict__ child_lo_up,
    const int* __restrict__ coords, const int* __restrict__ slot_c, const cpx<T>* __restrict__ Fc_c, LevelGeom gp,
    LevelGeom gc, ChebTab ct, const T* __restrict__ Ms, const T* __restrict__ Ma, double k, int kind, int R,
    cpx<T>* __restrict__ Fc_up, int* __restrict__ err) {
  constexpr bool CB = !(ONE && rows_ok<T, PS, PA>());
  __shared__ PropSmem<T, PS, PA, PropShape<PS * PA * PA>::BS, CB> sm;
  prop_item<T, PS, PA, ONE, PropShape<PS * PA * PA>::BS, CB>(sm, work[xcd_block(blockIdx.x, gridDim.x)], ONE ? 0 : blockIdx.y, rel_cone_up,
                            child_lo_up, coords, slot_c, Fc_c, gp, gc, ct, Ms, Ma, k, kind, R, Fc_up, err);
}

// ---------------------------------------------------------------------------
// cousin targets for a range of levels + near-field sum, scattered to the
// caller's order.
// ---------------------------------------------------------------------------
template <typename T> struct TLevel {
  const int IFGF_GAS* pbox;
  const int IFGF_GAS* cou_off;
  const int IFGF_GAS* cou;
  const double IFGF_GAS* centre;
  const int IFGF_GAS* slot;
  const cpx<T> IFGF_GAS* Fc;
  LevelGeom g;
};
template <typename T> struct TLevels {
  TLevel<T> lv[IFGF_MAX_LEVELS];
};

// Cousin targets of point i0 (Morton order) for levels dlo..dhi, right-hand
// side r, plus its near-field value; scattered to the caller's order.  Every
// lane of the wave calls it (i0 >= n: no point); wbuf is the wave's staging
// buffer of 2P values.
template <typename T, int PS, int PA>
__device__ __forceinline__ void target_point(T* wbuf, int64_t i0, int r, const double* __restrict__ pts, int64_t n,
                                             const int* __restrict__ perm, const cpx<T>* __restrict__ uacc,
                                             int use_near, const TLevels<T>& L, int dlo, int dhi, double k, int kind,
                                             int R, int dtype, int conj_out, const double* __restrict__ wout,
                                             void* __restrict__ u, int* __restrict__ err) {
  const bool valid = i0 < n;
  const int64_t i = valid ? i0 : n - 1;      // lanes past the end follow the last point and store nothing
  const double* x = pts + 3 * i;
  double acc_re = 0, acc_im = 0;
  if (use_near) {
    cpx<T> v = uacc[i * R + r];
    acc_re = v.re;
    acc_im = v.im;
  }
  const double inv4pi = 1.0 / (4.0 * IFGF_PI);
  for (int d = dhi; d >= dlo; --d) {
    const TLevel<T>& lv = L.lv[d];
    const int A = lv.pbox[i];
    cpx<T> lacc = {0, 0};
    // The lanes of a wave may belong to different boxes with different
    // cousin counts; the loop runs to the wave's largest count so that every
    // lane takes part in each coefficient staging of eval_uniform.
    const int c0 = lv.cou_off[A], cnt = lv.cou_off[A + 1] - c0;
    int cmax = cnt;
    for (int off = 32; off > 0; off >>= 1) cmax = max(cmax, __shfl_xor(cmax, off, 64));
    for (int t = 0; t < cmax; ++t) {
      const bool has = valid && t < cnt;
      const int B = lv.cou[c0 + min(t, max(cnt - 1, 0))];
      double rr;
      T ts = 0, tt = 0, tp = 0, e_re = 0, e_im = 0;
      int sl = -1;
      if (cnt > 0) {
        int cid;
        if constexpr (Prec<T>::f32) {
          LocF loc = target_loc32(x, gen(lv.centre) + 3 * B, lv.g, &rr);
          cid = loc.cid;
          ts = loc.ts;
          tt = loc.tt;
          tp = loc.tp;
          float c, s;
          expi_reduced32(k * rr, &c, &s);
          float g = (float)inv4pi / (float)rr;
          e_re = g * c;
          e_im = g * s;
        } else {
          Loc loc = target_loc64(x, gen(lv.centre) + 3 * B, lv.g, &rr);
          cid = loc.cid;
          ts = loc.ts;
          tt = loc.tt;
          tp = loc.tp;
          double c, s;
          sincos(k * rr, &s, &c);
          double g = inv4pi / rr;
          e_re = g * c;
          e_im = g * s;
        }
        if (kind == IFGF_KERNEL_CONSTANT) {
          e_re = 1;
          e_im = 0;
        }
        sl = lv.slot[(int64_t)B * lv.g.ncone + cid];
        if (sl < 0 && has) atomicOr(err, 4);
      }
      if (!has) sl = -1;
      cpx<T> v = eval_uniform<T, PS, PA>(gen(lv.Fc), sl, R, r, ts, tt, tp, wbuf);
      if (has) {
        lacc.re += e_re * v.re - e_im * v.im;
        lacc.im += e_re * v.im + e_im * v.re;
      }
    }
    acc_re += lacc.re;
    acc_im += lacc.im;
  }
  if (wout) {
    acc_re *= wout[i];
    acc_im *= wout[i];
  }
  if (conj_out) acc_im = -acc_im;
  if (!valid) return;
  const int64_t o = (int64_t)perm[i] * R + r;
  if (dtype == IFGF_C128) {
    ((double*)u)[2 * o] = acc_re;
    ((double*)u)[2 * o + 1] = acc_im;
  } else {
    ((float*)u)[2 * o] = (float)acc_re;
    ((float*)u)[2 * o + 1] = (float)acc_im;
  }
}

template <typename T, int PS, int PA>
__global__ __launch_bounds__(TPB) void k_targets(const double* __restrict__ pts, int64_t n, const int* __restrict__ perm,
                                                 const cpx<T>* __restrict__ uacc, int use_near, TLevels<T> L,
                                                 int dlo, int dhi, double k, int kind, int R, int dtype, int conj_out,
                                                 const double* __restrict__ wout, void* __restrict__ u,
                                                 int* __restrict__ err) {
  constexpr int P = PS * PA * PA;
  __shared__ __align__(16) T cbuf[TPB / 64][2 * P];
  const int64_t i0 = (int64_t)xcd_block(blockIdx.x, gridDim.x) * TPB + threadIdx.x;
  target_point<T, PS, PA>(cbuf[threadIdx.x >> 6], i0, blockIdx.y, pts, n, perm, uacc, use_near, L, dlo, dhi, k, kind,
                          R, dtype, conj_out, wout, u, err);
}

// ---------------------------------------------------------------------------
// Cousin targets, FP32, one right-hand side: row-broadcast formulation.
//
// A wave takes 64 consecutive (Morton-order) targets at one level d; a row of
// 16 lanes holds 16 neighbouring targets.  Each row walks the merged,
// ascending cousin lists of its lanes: at each step the row takes the
// smallest cousin box B still pending in any of its lanes, and the lanes
// whose list holds B evaluate B's interpolant at their target.  Such targets
// are close together and mostly fall in one cone of B; the row loads that
// cone's 2P coefficients across its 16 lanes (one float4 per lane per 64
// floats) and every lane contracts against them with the coefficients
// broadcast from their lanes by DPP (RowStage1), so four rows of a wave serve
// four cones at once and no coefficient passes through LDS.  Lanes whose
// cone differs from the row's current one wait for a further round.  Each
// lane sums its cousins in ascending box order: deterministic.  The level's
// sum goes to part[d - dlo][i]; k_targets_sum adds the levels.
// ---------------------------------------------------------------------------
// Sum over the cousins at level d of the lane's target x (valid: the lane
// holds a target; i: its Morton index, any in-range index when !valid).
// Every lane of the wave must call it together with the same level.
template <typename T, int PS, int PA>
__device__ __forceinline__ void rows_level(const TLevel<T>& lv, const double (&x)[3], bool valid, int64_t i,
                                           double k, int kind, int* __restrict__ err, T& acc_re, T& acc_im) {
  constexpr int P = PS * PA * PA;
  constexpr int NONE = 0x7fffffff;
  int ptr = 0, end = 0;
  if (valid) {
    const int A = lv.pbox[i];
    ptr = lv.cou_off[A];
    end = lv.cou_off[A + 1];
  }
  int nxt = ptr < end ? lv.cou[ptr] : NONE;
  const int nl = threadIdx.x & 15;
  const T* F = reinterpret_cast<const T*>(gen(lv.Fc));
  acc_re = 0;
  acc_im = 0;
  while (true) {
    const int B = row_min16(nxt);
    if (__ballot(B != NONE) == 0) break;
    int sl = NONE;
    T ts = 0, tt = 0, tp = 0, e_re = 0, e_im = 0;
    if (nxt == B && B != NONE) {
      double rr;
      int cid;
      if constexpr (Prec<T>::f32) {
        const LocF loc = target_loc32(x, gen(lv.centre) + 3 * B, lv.g, &rr);
        cid = loc.cid;
        ts = loc.ts;
        tt = loc.tt;
        tp = loc.tp;
        if (kind == IFGF_KERNEL_CONSTANT) {
          e_re = 1;
          e_im = 0;
        } else {
          float c, s;
          expi_reduced32(k * rr, &c, &s);
          const float g = (float)(1.0 / (4.0 * IFGF_PI)) / (float)rr;
          e_re = g * c;
          e_im = g * s;
        }
      } else {
        const Loc loc = target_loc64(x, gen(lv.centre) + 3 * B, lv.g, &rr);
        cid = loc.cid;
        ts = loc.ts;
        tt = loc.tt;
        tp = loc.tp;
        if (kind == IFGF_KERNEL_CONSTANT) {
          e_re = 1;
          e_im = 0;
        } else {
          double c, s;
          sincos(k * rr, &s, &c);
          const double g = (1.0 / (4.0 * IFGF_PI)) / rr;
          e_re = g * c;
          e_im = g * s;
        }
      }
      const int s0 = lv.slot[(int64_t)B * lv.g.ncone + cid];
      if (s0 < 0)
        atomicOr(err, 4);
      else
        sl = s0;
      ++ptr;
      nxt = ptr < end ? lv.cou[ptr] : NONE;
    }
    T Ts[PS], Tt[PA], Tp[PA];
    cheb_T<T, PS>(ts, Ts);
    cheb_T<T, PA>(tt, Tt);
    cheb_T<T, PA>(tp, Tp);
    bool pend = sl != NONE;
    while (__ballot(pend)) {
      const int su = row_min16(pend ? sl : NONE);
      T v_re, v_im;
      row_contract<T, PS, PA>(F + (int64_t)(su == NONE ? 0 : su) * (2 * P), nl, Ts, Tt, Tp, v_re, v_im);
      if (pend && sl == su) {
        acc_re += e_re * v_re - e_im * v_im;
        acc_im += e_re * v_im + e_im * v_re;
        pend = false;
      }
    }
  }
}

template <typename T, int PS, int PA>
__global__ __launch_bounds__(TPB) void k_targets_rows(const double* __restrict__ pts, int64_t n, TLevels<T> L,
                                                      int dlo, double k, int kind, cpx<T>* __restrict__ part,
                                                      int* __restrict__ err) {
  const int nchunk = (int)gridDim.x;
  const int lin = xcd_block((int)(blockIdx.y * gridDim.x + blockIdx.x), (int)(gridDim.x * gridDim.y));
  const int d = dlo + lin / nchunk;
  const int64_t i0 = (int64_t)(lin % nchunk) * TPB + threadIdx.x;
  const bool valid = i0 < n;
  const int64_t i = valid ? i0 : n - 1;
  const double x[3] = {pts[3 * i], pts[3 * i + 1], pts[3 * i + 2]};
  T acc_re, acc_im;
  rows_level<T, PS, PA>(L.lv[d], x, valid, i, k, kind, err, acc_re, acc_im);
  if (valid) part[(int64_t)(d - dlo) * n + i] = {acc_re, acc_im};
}

// u = near field + the level sums of k_targets_rows (levels from the finest
// down, as target_point adds them), scattered to the caller's order; one
// right-hand side.
template <typename T>
__global__ __launch_bounds__(TPB) void k_targets_sum(int64_t n, const int* __restrict__ perm,
                                                     const cpx<T>* __restrict__ uacc, int use_near,
                                                     const cpx<T>* __restrict__ part, int nlev, int dtype,
                                                     void* __restrict__ u) {
  const int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (i >= n) return;
  double re = 0, im = 0;
  if (use_near) {
    re = uacc[i].re;
    im = uacc[i].im;
  }
  for (int l = nlev - 1; l >= 0; --l) {
    const cpx<T> v = part[(int64_t)l * n + i];
    re += v.re;
    im += v.im;
  }
  const int64_t o = perm[i];
  if (dtype == IFGF_C128) {
    ((double*)u)[2 * o] = re;
    ((double*)u)[2 * o + 1] = im;
  } else {
    ((float*)u)[2 * o] = (float)re;
    ((float*)u)[2 * o + 1] = (float)im;
  }
}

// ---------------------------------------------------------------------------
// Cousin targets from plan-time pair lists (one RHS, orders with a row stage).
// The plan lists, per level, every (target, cousin box) pair with its cone
// slot, local coordinates and centred factor e^{ikr}/(4 pi r) (the same
// expressions as the row-broadcast formulation), sorted by slot, i.e. by
// (box, cone).  Pass one: each row of 16 lanes takes 16 consecutive pairs,
// which mostly share one cone, loads that cone across the row once and
// contracts by DPP broadcast (the row stage), and writes each pair's value.
// Pass two: each target sums its pairs' values, the levels from the finest
// down, in a fixed order.
// ---------------------------------------------------------------------------
template <typename T> struct Vec4;
template <> struct Vec4<float> { using type = float4; };
template <> struct Vec4<double> { using type = double4; };

template <typename T> struct PLevel {
  int64_t np;
  const int* slot;
  const typename Vec4<T>::type* loc;
  const T* fim;
  cpx<T>* val;
  const int* off;
  const int* pos;
  const cpx<T>* Fc;
};
template <typename T> struct PLevels {
  PLevel<T> lv[IFGF_MAX_LEVELS];
};

// One thread per target: its cousin pairs at level lv, in cousin order.
template <typename T>
__global__ __launch_bounds__(TPB) void k_pair_gen(const double* __restrict__ pts, int64_t n, TLevel<T> lv,
                                                  const int* __restrict__ off, double k, int kind,
                                                  uint64_t* __restrict__ keys, typename Vec4<T>::type* __restrict__ tloc,
                                                  T* __restrict__ tfim, int* __restrict__ err) {
  const int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (i >= n) return;
  const int A = lv.pbox[i];
  const int c0 = lv.cou_off[A], cnt = lv.cou_off[A + 1] - c0;
  const int64_t o = off[i];
  const double x[3] = {pts[3 * i], pts[3 * i + 1], pts[3 * i + 2]};
  for (int t = 0; t < cnt; ++t) {
    const int B = lv.cou[c0 + t];
    double rr;
    int cid;
    T ts, tt, tp, e_re, e_im;
    if constexpr (Prec<T>::f32) {
      const LocF loc = target_loc32(x, gen(lv.centre) + 3 * B, lv.g, &rr);
      cid = loc.cid;
      ts = loc.ts;
      tt = loc.tt;
      tp = loc.tp;
      if (kind == IFGF_KERNEL_CONSTANT) {
        e_re = 1;
        e_im = 0;
      } else {
        float c, sn;
        expi_reduced32(k * rr, &c, &sn);
        const float g = (float)(1.0 / (4.0 * IFGF_PI)) / (float)rr;
        e_re = g * c;
        e_im = g * sn;
      }
    } else {
      const Loc loc = target_loc64(x, gen(lv.centre) + 3 * B, lv.g, &rr);
      cid = loc.cid;
      ts = loc.ts;
      tt = loc.tt;
      tp = loc.tp;
      if (kind == IFGF_KERNEL_CONSTANT) {
        e_re = 1;
        e_im = 0;
      } else {
        double c, sn;
        sincos(k * rr, &sn, &c);
        const double g = (1.0 / (4.0 * IFGF_PI)) / rr;
        e_re = g * c;
        e_im = g * sn;
      }
    }
    int sl = lv.slot[(int64_t)B * lv.g.ncone + cid];
    if (sl < 0) {
      atomicOr(err, 4);
      sl = 0;
      e_re = e_im = 0;
    }
    keys[o + t] = ((uint64_t)(uint32_t)sl << 32) | (uint64_t)(uint32_t)(o + t);
    tloc[o + t] = {ts, tt, tp, e_re};
    tfim[o + t] = e_im;
  }
}

// Sorted position q holds original pair orig = low word of its key.
template <typename T>
__global__ __launch_bounds__(TPB) void k_pair_place(const uint64_t* __restrict__ keys, int64_t np,
                                                    const typename Vec4<T>::type* __restrict__ tloc,
                                                    const T* __restrict__ tfim, int* __restrict__ slot,
                                                    typename Vec4<T>::type* __restrict__ loc, T* __restrict__ fim,
                                                    int* __restrict__ pos) {
  const int64_t q = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (q >= np) return;
  const uint64_t key = keys[q];
  const int64_t orig = (int64_t)(uint32_t)key;
  slot[q] = (int)(key >> 32);
  loc[q] = tloc[orig];
  fim[q] = tfim[orig];
  pos[orig] = (int)q;
}

// ---------------------------------------------------------------------------
// Upward pass d+1 -> d from a pair list (sparse levels, one RHS; Algorithm 1,
// parent interpolation nodes).  Where few boxes share a cone id the
// cone-major tiles run nearly empty, and the node formulation re-locates and
// re-buckets every node at every apply.  The plan instead locates once every
// (parent node, child box) pair - child cone slot, local coordinates, factor
// K(x, y_child) / K(x, y_parent) - and sorts the pairs by slot; an apply then
// evaluates them with pairs_block (the rows of 16 lanes mostly share one
// cone) and k_upsum_coeffs adds each node's pairs in child order and turns
// the node values into coefficients.
// ---------------------------------------------------------------------------
// pairs of relevant cone s: P per child of its box
__global__ __launch_bounds__(TPB) void k_upair_count(int nrel, const int* __restrict__ rel_box,
                                                     const int* __restrict__ child_lo, int P, int* __restrict__ cnt) {
  const int64_t sc = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (sc >= nrel) return;
  const int b = rel_box[sc];
  cnt[sc] = P * (child_lo[b + 1] - child_lo[b]);
}

// One thread per parent node (s, j): its pairs with the children of s's box,
// in child order, at base[s] + j * nch + t (key: slot, then that index).
template <typename T, int PS, int PA>
__global__ __launch_bounds__(TPB) void k_upair_gen(int nrel, const int* __restrict__ rel_box,
                                                   const int* __restrict__ rel_cone, const int* __restrict__ child_lo,
                                                   const int* __restrict__ coords, const int* __restrict__ slot_c,
                                                   const int* __restrict__ base, LevelGeom gp, LevelGeom gc,
                                                   ChebTab ct, double k, int kind, uint64_t* __restrict__ keys,
                                                   typename Vec4<T>::type* __restrict__ tloc, T* __restrict__ tfim,
                                                   int* __restrict__ err) {
  constexpr int P = PS * PA * PA;
  const int64_t t = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (t >= (int64_t)nrel * P) return;
  const int sc = (int)(t / P), node = (int)(t % P);
  const int ai = node / (PA * PA), bi = (node / PA) % PA, ci = node % PA;
  const int Pb = rel_box[sc];
  T x[3], rp;
  if constexpr (Prec<T>::f32) node_rel32(rel_cone[sc], ai, bi, ci, gp, ct, x, &rp);
  else node_rel64(rel_cone[sc], ai, bi, ci, gp, ct, x, &rp);
  const int B0 = child_lo[Pb], nch = child_lo[Pb + 1] - B0;
  const int64_t o0 = base[sc] + (int64_t)node * nch;
  for (int c = 0; c < nch; ++c) {
    const int B = B0 + c;
    const int oct = (coords[3 * B] & 1) | ((coords[3 * B + 1] & 1) << 1) | ((coords[3 * B + 2] & 1) << 2);
    typename PropGeomT<T>::P pr;
    if constexpr (Prec<T>::f32) pr = child_loc32(x, rp, oct, gc);
    else pr = child_loc64(x, rp, oct, gc);
    int sl = slot_c[(int64_t)B * gc.ncone + pr.loc.cid];
    T rr = pr.rp_over_rc, c_, s_;
    if (kind == IFGF_KERNEL_CONSTANT) {
      c_ = 1;
      s_ = 0;
      rr = 1;
    } else {
      sincos_t<T>((T)k * pr.dr, &s_, &c_);
    }
    T rre = rr * c_, rim = rr * s_;
    if (sl < 0) {   // a missing child cone: flagged, the pair adds nothing
      atomicOr(err, 2);
      sl = 0;
      rre = rim = 0;
    }
    const int64_t o = o0 + c;
    keys[o] = ((uint64_t)(uint32_t)sl << 32) | (uint64_t)(uint32_t)o;
    tloc[o] = {pr.loc.ts, pr.loc.tt, pr.loc.tp, rre};
    tfim[o] = rim;
  }
}

// parent node s * P + j of every sorted pair (for the transposed pass)
__global__ __launch_bounds__(TPB) void k_upair_node(int nrel, int P, const int* __restrict__ base,
                                                    const int* __restrict__ pos, int* __restrict__ node) {
  const int64_t t = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (t >= (int64_t)nrel * P) return;
  const int sc = (int)(t / P), j = (int)(t % P);
  const int b0 = base[sc], nch = (base[sc + 1] - b0) / P;
  for (int c = 0; c < nch; ++c) node[pos[b0 + j * nch + c]] = (int)t;
}

// Pass one for the TPB pairs q0 .. q0 + TPB - 1 of a level (one per thread).
template <typename T, int PS, int PA>
__device__ __forceinline__ void pairs_block(const PLevel<T>& lv, int64_t q0) {
  constexpr int P = PS * PA * PA;
  constexpr int NONE = 0x7fffffff;
  const int64_t q = q0 + threadIdx.x;
  const bool valid = q < lv.np;
  const int sl = valid ? lv.slot[q] : NONE;
  typename Vec4<T>::type lc = {0, 0, 0, 0};
  T fim = 0;
  if (valid) {
    lc = lv.loc[q];
    fim = lv.fim[q];
  }
  T Ts[PS], Tt[PA], Tp[PA];
  cheb_T<T, PS>(lc.x, Ts);
  cheb_T<T, PA>(lc.y, Tt);
  cheb_T<T, PA>(lc.z, Tp);
  const int nl = threadIdx.x & 15;
  const T* F = reinterpret_cast<const T*>(lv.Fc);
  T o_re = 0, o_im = 0;
  bool pend = valid;
  while (__ballot(pend)) {
    const int su = row_min16(pend ? sl : NONE);
    T v_re, v_im;
    row_contract<T, PS, PA>(F + (int64_t)(su == NONE ? 0 : su) * (2 * P), nl, Ts, Tt, Tp, v_re, v_im);
    if (pend && sl == su) {
      o_re = lc.w * v_re - fim * v_im;
      o_im = lc.w * v_im + fim * v_re;
      pend = false;
    }
  }
  if (valid) lv.val[q] = {o_re, o_im};
}

// Upward pass from a pair list, first kernel: the value of every pair.
template <typename T, int PS, int PA>
__global__ __launch_bounds__(TPB) __attribute__((amdgpu_waves_per_eu(3))) void k_upairs(PLevel<T> lv) {
  const int64_t q0 = (int64_t)xcd_block(blockIdx.x, gridDim.x) * TPB;
  if (q0 >= lv.np) return;   // block-uniform
  pairs_block<T, PS, PA>(lv, q0);
}

// Pass one: the value of every pair of level dlo + blockIdx.y.
template <typename T, int PS, int PA>
__global__ __launch_bounds__(TPB) __attribute__((amdgpu_waves_per_eu(3))) void k_targets_pairs(PLevels<T> L, int dlo) {
  const PLevel<T>& lv = L.lv[dlo + blockIdx.y];
  const int64_t q0 = (int64_t)xcd_block(blockIdx.x, gridDim.x) * TPB;
  if (q0 >= lv.np) return;   // block-uniform
  pairs_block<T, PS, PA>(lv, q0);
}

// Pass two: u = near field + per level (finest first) the sum of the
// target's pair values, scattered to the caller's order.  16 lanes per
// target: lane j adds pairs j, j + 16, ... of the target's list at a level
// (coalesced reads of the position list), then a fixed butterfly adds the 16
// partial sums.  The order is fixed (every call gives the same sums), not
// the row formulation's sequential one (the two agree to rounding).
template <typename T>
__device__ __forceinline__ void pairsum16(int64_t tid, int64_t n, const int* __restrict__ perm,
                                          const cpx<T>* __restrict__ uacc, int use_near, const PLevels<T>& L,
                                          int dlo, int dhi, int dtype, void* __restrict__ u) {
  const int64_t i0 = tid >> 4;
  const int j = threadIdx.x & 15;
  const bool valid = i0 < n;
  const int64_t i = valid ? i0 : n - 1;   // every lane takes part in the butterfly
  double re = 0, im = 0;
  for (int d = dhi; d >= dlo; --d) {
    const PLevel<T>& lv = L.lv[d];
    T lre = 0, lim = 0;
    const int t1 = lv.off[i + 1];
    for (int t = lv.off[i] + j; t < t1; t += 16) {
      const cpx<T> v = lv.val[lv.pos[t]];
      lre += v.re;
      lim += v.im;
    }
#pragma unroll
    for (int m = 8; m > 0; m >>= 1) {
      lre += __shfl_xor(lre, m, 16);
      lim += __shfl_xor(lim, m, 16);
    }
    re += lre;
    im += lim;
  }
  if (!valid || j != 0) return;
  if (use_near) {
    re += uacc[i].re;
    im += uacc[i].im;
  }
  const int64_t o = perm[i];
  if (dtype == IFGF_C128) {
    ((double*)u)[2 * o] = re;
    ((double*)u)[2 * o + 1] = im;
  } else {
    ((float*)u)[2 * o] = (float)re;
    ((float*)u)[2 * o + 1] = (float)im;
  }
}

template <typename T>
__global__ __launch_bounds__(TPB) void k_targets_pairsum(int64_t n, const int* __restrict__ perm,
                                                         const cpx<T>* __restrict__ uacc, int use_near,
                                                         PLevels<T> L, int dlo, int dhi, int dtype,
                                                         void* __restrict__ u) {
  pairsum16<T>((int64_t)blockIdx.x * TPB + threadIdx.x, n, perm, uacc, use_near, L, dlo, dhi, dtype, u);
}

// Per row of 16 consecutive sorted pairs, the cone slots it meets (1 + the
// slot changes inside the row): the passes of the row stage.
__global__ __launch_bounds__(TPB) void k_pair_rows(const int* __restrict__ slot, int64_t np,
                                                   unsigned long long* __restrict__ acc) {
  const int64_t r = (int64_t)blockIdx.x * TPB + threadIdx.x;
  unsigned long long v = 0;
  if (r * 16 < np) {
    const int64_t q0 = r * 16, q1 = min(np, q0 + 16);
    v = 1;
    for (int64_t q = q0 + 1; q < q1; ++q) v += slot[q] != slot[q - 1] ? 1 : 0;
  }
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  if ((threadIdx.x & 63) == 0 && v) atomicAdd(acc, v);
}

// per target, the number of its cousin pairs at a level
__global__ __launch_bounds__(TPB) void k_pair_count(const int* __restrict__ pbox, const int* __restrict__ cou_off,
                                                    int64_t n, int* __restrict__ cnt) {
  const int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (i < n) cnt[i] = cou_off[pbox[i] + 1] - cou_off[pbox[i]];
}

// ---------------------------------------------------------------------------
// Batched right-hand sides on MFMA (FP32 mode, nrhs a multiple of 16).
//
// For the 64 evaluations held by a wave (one per lane: a target and a cousin
// box, or a parent node and a child), the interpolants of one cone for 16
// right-hand sides form the product
//     OUT[row][e] = sum_k C[k][row] B[k][e],
// rows = 16 RHS x (re, im) in two 16-row tiles, k = basis index, and
// B[k][e] = T_a(ts_e) T_b(tt_e) T_c(tp_e) for evaluations whose cone is the
// current one (0 otherwise).  It runs on v_mfma_f32_16x16x4_f32 with the
// evaluations as four 16-column blocks and the basis index ordered (b, c, a)
// so that the radial index a fills the instruction's 4-wide K step: each
// lane's B operand is then T_a(ts) T_b(tt) T_c(tp) with its own a and
// compile-time b, c.  Lane layouts: A[i][k] from lane 16k + i, B[k][j] from
// lane 16k + j, D[4q + v][j] in lane 16q + j, element v.
// ---------------------------------------------------------------------------
typedef float floatx4 __attribute__((ext_vector_type(4)));
constexpr int MF_RG = 16;   // right-hand sides per pass

template <int PS, int PA> struct MfRec {
  static constexpr int NR = PS + 2 * PA + 3;   // Ts, Tt, Tp, slot (as int), factor (re, im)
};

template <int PS, int PA>
__device__ __forceinline__ void mfma_cone(const float* __restrict__ Cb, int R, int g, const float (&wq)[4][PA],
                                          const float (&tq)[4][PA], floatx4 (&acc)[2][4]) {
  const int l = threadIdx.x & 63;
  const int h = min(l >> 4, PS - 1);
  const int i = l & 15;
#pragma unroll
  for (int bb = 0; bb < PA; ++bb) {
#pragma unroll
    for (int c = 0; c < PA; ++c) {
      const int64_t j = (h * PA + bb) * PA + c;
      const float a0 = Cb[(j * R + g * MF_RG) * 2 + i];
      const float a1 = Cb[(j * R + g * MF_RG) * 2 + 16 + i];
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const float bv = wq[b][bb] * tq[b][c];
        acc[0][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, bv, acc[0][b], 0, 0, 0);
        acc[1][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, bv, acc[1][b], 0, 0, 0);
      }
    }
  }
}

// One evaluation per lane (all 64 lanes call; slot < 0 = none): adds
// f_e * I_e[rhs] into tot for the evaluations and RHS this lane holds:
// tot[b][2 rt + p] is RHS 8 rt + 2 (lane >> 4) + p of evaluation 16 b + (lane & 15).
template <int PS, int PA>
__device__ __forceinline__ void wave_eval_mfma(const cpx<float>* __restrict__ F, int R, int g, int slot, float ts,
                                               float tt, float tp, float fre, float fim, float* rec,
                                               cpx<float> (&tot)[4][4]) {
  constexpr int P = PS * PA * PA;
  constexpr int NR = MfRec<PS, PA>::NR;
  const int l = threadIdx.x & 63;
  float* my = rec + l * NR;
  cheb_T<float, PS>(ts, my);
  cheb_T<float, PA>(tt, my + PS);
  cheb_T<float, PA>(tp, my + PS + PA);
  my[PS + 2 * PA] = __int_as_float(slot);
  my[PS + 2 * PA + 1] = fre;
  my[PS + 2 * PA + 2] = fim;
  __builtin_amdgcn_wave_barrier();
  const int h = l >> 4;
  floatx4 acc[2][4];
#pragma unroll
  for (int rt = 0; rt < 2; ++rt)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[rt][b] = (floatx4){0.f, 0.f, 0.f, 0.f};
  uint64_t pending = __ballot(slot >= 0);
  while (pending) {
    const int lead = first_lane(pending);
    const int su = __builtin_amdgcn_readfirstlane(__shfl(slot, lead, 64));
    pending &= ~__ballot(slot == su);
    float wq[4][PA], tq[4][PA];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const float* re = rec + (16 * b + (l & 15)) * NR;
      const bool m = __float_as_int(re[PS + 2 * PA]) == su && h < PS;
      const float ta = m ? re[min(h, PS - 1)] : 0.f;
#pragma unroll
      for (int bb = 0; bb < PA; ++bb) wq[b][bb] = ta * re[PS + bb];
#pragma unroll
      for (int c = 0; c < PA; ++c) tq[b][c] = re[PS + PA + c];
    }
    mfma_cone<PS, PA>(reinterpret_cast<const float*>(F + (int64_t)su * P * R), R, g, wq, tq, acc);
  }
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const float* re = rec + (16 * b + (l & 15)) * NR;
    const float er = re[PS + 2 * PA + 1], ei = re[PS + 2 * PA + 2];
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
      for (int p2 = 0; p2 < 2; ++p2) {
        const float vr = acc[rt][b][2 * p2], vi = acc[rt][b][2 * p2 + 1];
        tot[b][2 * rt + p2].re += er * vr - ei * vi;
        tot[b][2 * rt + p2].im += er * vi + ei * vr;
      }
  }
  (void)h;
  __builtin_amdgcn_wave_barrier();
}

// Cousin targets (levels dlo..dhi) for RHS group blockIdx.y, plus the near
// field, scattered to the caller's order.  Same traversal as k_targets.
template <int PS, int PA>
__global__ __launch_bounds__(TPB) void k_targets_mfma(const double* __restrict__ pts, int64_t n,
                                                      const int* __restrict__ perm, const cpx<float>* __restrict__ uacc,
                                                      int use_near, TLevels<float> L, int dlo, int dhi, double k,
                                                      int kind, int R, int dtype, void* __restrict__ u,
                                                      int* __restrict__ err) {
  constexpr int NR = MfRec<PS, PA>::NR;
  __shared__ float rec[TPB / 64][64 * NR];
  const int g = blockIdx.y;
  const int l = threadIdx.x & 63;
  const int64_t i0 = (int64_t)xcd_block(blockIdx.x, gridDim.x) * TPB + threadIdx.x;
  const bool valid = i0 < n;
  const int64_t i = valid ? i0 : n - 1;
  const double* x = pts + 3 * i;
  cpx<float> tot[4][4];
#pragma unroll
  for (int b = 0; b < 4; ++b)
#pragma unroll
    for (int q = 0; q < 4; ++q) tot[b][q] = {0.f, 0.f};
  const double inv4pi = 1.0 / (4.0 * IFGF_PI);
  for (int d = dhi; d >= dlo; --d) {
    const TLevel<float>& lv = L.lv[d];
    const int A = lv.pbox[i];
    const int c0 = lv.cou_off[A], cnt = lv.cou_off[A + 1] - c0;
    int cmax = cnt;
    for (int off = 32; off > 0; off >>= 1) cmax = max(cmax, __shfl_xor(cmax, off, 64));
    for (int t = 0; t < cmax; ++t) {
      const bool has = valid && t < cnt;
      const int B = lv.cou[c0 + min(t, max(cnt - 1, 0))];
      float ts = 0, tt = 0, tp = 0, e_re = 0, e_im = 0;
      int sl = -1;
      if (cnt > 0) {
        double rr;
        LocF loc = target_loc32(x, gen(lv.centre) + 3 * B, lv.g, &rr);
        ts = loc.ts;
        tt = loc.tt;
        tp = loc.tp;
        float c, s;
        expi_reduced32(k * rr, &c, &s);
        float gf = (float)inv4pi / (float)rr;
        e_re = gf * c;
        e_im = gf * s;
        if (kind == IFGF_KERNEL_CONSTANT) {
          e_re = 1;
          e_im = 0;
        }
        sl = lv.slot[(int64_t)B * lv.g.ncone + loc.cid];
        if (sl < 0 && has) atomicOr(err, 4);
      }
      if (!has) {
        sl = -1;
        e_re = e_im = 0;
      }
      wave_eval_mfma<PS, PA>(gen(lv.Fc), R, g, sl, ts, tt, tp, e_re, e_im, rec[threadIdx.x >> 6], tot);
    }
  }
  // lane l holds RHS 8 rt + 2 (l >> 4) + p of target 16 b + (l & 15) of its wave
  const int64_t wbase = i0 - l;
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const int64_t ti = wbase + 16 * b + (l & 15);
    if (ti >= n) continue;
    const int64_t po = perm[ti];
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
      for (int p2 = 0; p2 < 2; ++p2) {
        const int rr = g * MF_RG + 8 * rt + 2 * (l >> 4) + p2;
        double re = tot[b][2 * rt + p2].re, im = tot[b][2 * rt + p2].im;
        if (use_near) {
          const cpx<float> v = uacc[ti * R + rr];
          re += v.re;
          im += v.im;
        }
        const int64_t o = po * R + rr;
        if (dtype == IFGF_C128) {
          ((double*)u)[2 * o] = re;
          ((double*)u)[2 * o + 1] = im;
        } else {
          ((float*)u)[2 * o] = (float)re;
          ((float*)u)[2 * o + 1] = (float)im;
        }
      }
  }
}

// Pair-list cousin targets for RHS group g (FP32, nrhs a multiple of
// 16): a wave takes 64 consecutive pairs of level dlo + blockIdx.y, which
// mostly share one cone, and evaluates them for the group's 16 right-hand
// sides on MFMA (wave_eval_mfma: one pass per distinct cone); the values,
// times each pair's centred factor, go to val[pair][16].
template <int PS, int PA>
__global__ __launch_bounds__(TPB) void k_targets_pairs_rg(PLevels<float> L, int dlo, int R, int g) {
  constexpr int NR = MfRec<PS, PA>::NR;
  __shared__ float rec[TPB / 64][64 * NR];
  const PLevel<float>& lv = L.lv[dlo + blockIdx.y];
  const int64_t q0 = (int64_t)xcd_block(blockIdx.x, gridDim.x) * TPB;
  if (q0 >= lv.np) return;   // block-uniform
  const int l = threadIdx.x & 63;
  const int64_t qw = q0 + (threadIdx.x & ~63);
  const int64_t q = qw + l;
  const bool valid = q < lv.np;
  int sl = -1;
  float4 lc = {0.f, 0.f, 0.f, 0.f};
  float fim = 0.f;
  if (valid) {
    sl = lv.slot[q];
    lc = lv.loc[q];
    fim = lv.fim[q];
  }
  cpx<float> tot[4][4];
#pragma unroll
  for (int b = 0; b < 4; ++b)
#pragma unroll
    for (int c = 0; c < 4; ++c) tot[b][c] = {0.f, 0.f};
  wave_eval_mfma<PS, PA>(lv.Fc, R, g, sl, lc.x, lc.y, lc.z, lc.w, fim, rec[threadIdx.x >> 6], tot);
  // lane l holds RHS 8 rt + 2 (l >> 4) + p of pair 16 b + (l & 15) of its wave
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const int64_t e = qw + 16 * b + (l & 15);
    if (e >= lv.np) continue;
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
      for (int p2 = 0; p2 < 2; ++p2) lv.val[e * MF_RG + 8 * rt + 2 * (l >> 4) + p2] = tot[b][2 * rt + p2];
  }
}

// u[:, group g] = near field + per level (finest first) the sum of the
// target's pair values in cousin order.
__global__ __launch_bounds__(TPB) void k_targets_pairsum_rg(int64_t n, const int* __restrict__ perm,
                                                            const cpx<float>* __restrict__ uacc, int use_near,
                                                            PLevels<float> L, int dlo, int dhi, int R, int g,
                                                            int dtype, void* __restrict__ u) {
  // 16 lanes per target, lane r = RHS g * 16 + r: a pair's 16 values are one
  // 128-byte row read by the 16 lanes together; each lane adds its RHS over
  // the target's pairs in cousin order
  const int64_t tid = (int64_t)blockIdx.x * TPB + threadIdx.x;
  const int64_t i = tid / MF_RG;
  const int r = (int)(tid % MF_RG);
  if (i >= n) return;
  double re = 0.0, im = 0.0;
  if (use_near) {
    const cpx<float> v = uacc[i * R + g * MF_RG + r];
    re = v.re;
    im = v.im;
  }
  for (int d = dhi; d >= dlo; --d) {
    const PLevel<float>& lv = L.lv[d];
    float lre = 0.f, lim = 0.f;
    const int t1 = lv.off[i + 1];
    for (int t = lv.off[i]; t < t1; ++t) {
      const cpx<float> v = lv.val[(int64_t)lv.pos[t] * MF_RG + r];
      lre += v.re;
      lim += v.im;
    }
    re += lre;
    im += lim;
  }
  const int64_t o = (int64_t)perm[i] * R + g * MF_RG + r;
  if (dtype == IFGF_C128) {
    ((double*)u)[2 * o] = re;
    ((double*)u)[2 * o + 1] = im;
  } else {
    ((float*)u)[2 * o] = (float)re;
    ((float*)u)[2 * o + 1] = (float)im;
  }
}

// Upward pass for RHS group blockIdx.y with the nodes grouped by child cone:
// one work-group per parent slot.  For each child, the P node geometries are
// computed once and grouped by child cone; the waves then evaluate, per
// group, OUT[row][e] = sum_k C[row][k] B[k][e] with rows = 16 RHS (one tile
// for re, one for im) of the child cone's coefficients and columns = 16
// nodes of the group, so that no column of an MFMA tile belongs to another
// cone.  ratio * OUT is added to the node values in LDS (one writer per
// (node, RHS) per child: deterministic); they are turned into coefficients
// in place and written to level d-1.
template <int PS, int PA> struct TiGeo;

template <int PS, int PA> struct BcSmem {
  static constexpr int P = PS * PA * PA;
  static constexpr int NBAS = PS + 2 * PA;
  static constexpr int BAS_LD = NBAS | 1;
  cpx<float> acc[P][MF_RG + 1];   // node values for the 16 RHS of the group (padded row)
  float bas[P][BAS_LD];
  float rat[P][2];
  int cid[P];
  short order[P];
  int gstart[P + 1], gcid[P];
  short tstart[P + 1];          // group g: column tiles tstart[g] .. tstart[g+1]-1
  short tgrp[P + P / 16 + 1];   // group of each column tile
  int ngroup;
  float ms[PS * PS], ma[PA * PA];
  float ang[2 * PA][2];   // (sin, cos) of the parent cone's PA polar and PA azimuthal node angles
  float rad[PS];          // and its node radii h / s
};

template <int PS, int PA>
__global__ __launch_bounds__(TPB) __attribute__((amdgpu_waves_per_eu(4))) void k_prop_mfma_cone(const int* __restrict__ rel_box_up,
                                                        const int* __restrict__ rel_cone_up,
                                                        const int* __restrict__ child_lo_up,
                                                        const int* __restrict__ coords, const int* __restrict__ slot_c,
                                                        const cpx<float>* __restrict__ Fc_c, LevelGeom gp,
                                                        LevelGeom gc, ChebTab ct, const float* __restrict__ Ms,
                                                        const float* __restrict__ Ma, double k, int kind, int R,
                                                        const TiGeo<PS, PA>* __restrict__ recs,
                                                        const int* __restrict__ rec_of, cpx<float>* __restrict__ Fc_up,
                                                        int* __restrict__ err) {
  using S = BcSmem<PS, PA>;
  constexpr int P = S::P;
  constexpr int NWV = TPB / 64;
  __shared__ S sm;
  const int sp = xcd_block(blockIdx.x, gridDim.x);
  const int g = blockIdx.y;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int li = lane & 15, la = lane >> 4;
  const int Pb = rel_box_up[sp], q = rel_cone_up[sp];
  for (int t = threadIdx.x; t < P * (MF_RG + 1); t += TPB) sm.acc[t / (MF_RG + 1)][t % (MF_RG + 1)] = {0.f, 0.f};
  if (threadIdx.x < PS * PS) sm.ms[threadIdx.x] = Ms[threadIdx.x];
  if (threadIdx.x < PA * PA) sm.ma[threadIdx.x] = Ma[threadIdx.x];
  if (threadIdx.x < 2 * PA + PS) {   // the terms of node_rel32 for cone id q
    const int j = threadIdx.x;
    int is, it, ip;
    cone_split(q, gp.nc, &is, &it, &ip);
    if (j < PA)
      sincos_f(((float)it + ct.uaf[j]) * gp.daf, &sm.ang[j][0], &sm.ang[j][1]);
    else if (j < 2 * PA)
      sincos_f(((float)ip + ct.uaf[j - PA]) * gp.daf, &sm.ang[j][0], &sm.ang[j][1]);
    else
      sm.rad[j - 2 * PA] = gp.hf * rcp_f(((float)is + ct.usf[j - 2 * PA]) * gp.dsf);
  }
  const int B0 = child_lo_up[Pb], B1 = child_lo_up[Pb + 1];
  // the plan's node records of the cone id, where the level has them
  const int rec = rec_of ? rec_of[sp] : -1;   // block-uniform
  for (int B = B0; B < B1; ++B) {
    const int oct = (coords[3 * B] & 1) | ((coords[3 * B + 1] & 1) << 1) | ((coords[3 * B + 2] & 1) << 2);
    __syncthreads();   // previous child's groups and geometry no longer read; the node terms written
    if (rec >= 0) {   // geometry and groups from the record of (cone id, octant)
      const TiGeo<PS, PA>& G = recs[(int64_t)rec * 8 + oct];
      const int ngr = G.ngroup;
      for (int e = threadIdx.x; e < P; e += TPB) {
        const int n = G.node[e];
        const float4 lc = G.loc[e];
        const float2 rt = G.rat[e];
        sm.order[e] = (short)n;
        cheb_T<float, PS>(lc.x, &sm.bas[n][0]);
        cheb_T<float, PA>(lc.y, &sm.bas[n][PS]);
        cheb_T<float, PA>(lc.z, &sm.bas[n][PS + PA]);
        sm.rat[n][0] = rt.x;
        sm.rat[n][1] = rt.y;
      }
      for (int t = threadIdx.x; t <= ngr; t += TPB) {
        sm.gstart[t] = G.gstart[t];
        sm.tstart[t] = G.tstart[t];
        if (t < ngr) sm.gcid[t] = G.gcid[t];
      }
      const int nt = G.tstart[ngr];
      for (int t = threadIdx.x; t < nt; t += TPB) sm.tgrp[t] = G.tgrp[t];
      if (threadIdx.x == 0) sm.ngroup = ngr;
    } else {
      for (int n = threadIdx.x; n < P; n += TPB) {
        float x[3], rp;
        {   // node_rel32 from the tabulated terms
          const int bi = (n / PA) % PA, ci = n % PA;
          const float st = sm.ang[bi][0], ctt = sm.ang[bi][1], sp_ = sm.ang[PA + ci][0], cp = sm.ang[PA + ci][1];
          const float e0 = st * cp, e1 = st * sp_;
          rp = sm.rad[n / (PA * PA)];
          x[0] = rp * e0;
          x[1] = rp * e1;
          x[2] = rp * ctt;
        }
        const PropF pr = child_loc32(x, rp, oct, gc);
        sm.cid[n] = pr.loc.cid;
        cheb_T<float, PS>(pr.loc.ts, &sm.bas[n][0]);
        cheb_T<float, PA>(pr.loc.tt, &sm.bas[n][PS]);
        cheb_T<float, PA>(pr.loc.tp, &sm.bas[n][PS + PA]);
        float c_ = 1.f, s_ = 0.f, rr = 1.f;
        if (kind != IFGF_KERNEL_CONSTANT) {
          sincos_f((float)k * pr.dr, &s_, &c_);
          rr = pr.rp_over_rc;
        }
        sm.rat[n][0] = rr * c_;
        sm.rat[n][1] = rr * s_;
      }
      __syncthreads();
      if (wv == 0) {   // group the nodes by child cone
        constexpr int NPL = (P + 63) / 64;
        int cv[NPL];
        bool pend[NPL];
#pragma unroll
        for (int m = 0; m < NPL; ++m) {
          const int n = lane + 64 * m;
          pend[m] = n < P;
          cv[m] = pend[m] ? sm.cid[n] : 0;
        }
        int pos = 0, ng = 0;
        while (true) {
          int lead = -1, su = 0;
#pragma unroll
          for (int m = 0; m < NPL && lead < 0; ++m) {
            const uint64_t b = __ballot(pend[m]);
            if (b) {
              lead = first_lane(b);
              su = __builtin_amdgcn_readfirstlane(__shfl(cv[m], lead, 64));
            }
          }
          if (lead < 0) break;
          if (lane == 0) {
            sm.gstart[ng] = pos;
            sm.gcid[ng] = su;
          }
#pragma unroll
          for (int m = 0; m < NPL; ++m) {
            const bool hit = pend[m] && cv[m] == su;
            const uint64_t b = __ballot(hit);
            if (hit) sm.order[pos + __popcll(b & ((1ull << lane) - 1))] = (short)(lane + 64 * m);
            pos += __popcll(b);
            pend[m] = pend[m] && !hit;
          }
          ++ng;
        }
        if (lane == 0) {
          sm.gstart[ng] = pos;
          sm.ngroup = ng;
        }
      }
      __syncthreads();
      if (threadIdx.x == 0) {   // column tiles of the groups
        int tp = 0;
        for (int gi = 0; gi < sm.ngroup; ++gi) {
          sm.tstart[gi] = (short)tp;
          const int nt = (sm.gstart[gi + 1] - sm.gstart[gi] + 15) >> 4;
          for (int t = 0; t < nt; ++t) sm.tgrp[tp + t] = (short)gi;
          tp += nt;
        }
        sm.tstart[sm.ngroup] = (short)tp;
      }
    }
    __syncthreads();
    // the groups' column tiles, in order, split evenly over the waves; a
    // wave loads a group's A operand (the child cone's coefficients for the
    // 16 RHS, re and im) when its run of tiles enters the group
    const int ngt = sm.tstart[sm.ngroup];
    const int u0 = wv * ngt / NWV, u1 = (wv + 1) * ngt / NWV;
    int gcur = -1, sl = -1;
    float are[PA * PA], aim[PA * PA];
    for (int u = u0; u < u1; ++u) {
      const int gi = sm.tgrp[u];
      const int n0 = sm.gstart[gi], n1 = sm.gstart[gi + 1];
      if (gi != gcur) {   // wave-uniform
        gcur = gi;
        sl = slot_c[(int64_t)B * gc.ncone + sm.gcid[gi]];
        if (sl < 0) {
          if (lane == 0) atomicOr(err, 2);
        } else {   // A rows: RHS g*16 + li of coefficient (la, b, c) of the child cone
          const cpx<float>* Cs = Fc_c + ((int64_t)sl * P + (la < PS ? la : 0) * PA * PA) * R + g * MF_RG + li;
#pragma unroll
          for (int t = 0; t < PA * PA; ++t) {
            const cpx<float> av = la < PS ? Cs[(int64_t)t * R] : cpx<float>{0.f, 0.f};
            are[t] = av.re;
            aim[t] = av.im;
          }
        }
      }
      if (sl < 0) continue;
      {
        const int c0 = n0 + 16 * (u - sm.tstart[gi]);
        const int e = c0 + li;
        const int n = e < n1 ? sm.order[e] : -1;
        float ta = 0.f, tt[PA], tp[PA];
        if (n >= 0) {
          ta = la < PS ? sm.bas[n][min(la, PS - 1)] : 0.f;
#pragma unroll
          for (int b = 0; b < PA; ++b) tt[b] = sm.bas[n][PS + b];
#pragma unroll
          for (int c = 0; c < PA; ++c) tp[c] = sm.bas[n][PS + PA + c];
        } else {
#pragma unroll
          for (int b = 0; b < PA; ++b) tt[b] = tp[b] = 0.f;
        }
        floatx4 d0 = {0.f, 0.f, 0.f, 0.f}, d1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int b = 0; b < PA; ++b) {
          const float w = ta * tt[b];
#pragma unroll
          for (int c = 0; c < PA; ++c) {
            const float bv = w * tp[c];
            d0 = __builtin_amdgcn_mfma_f32_16x16x4f32(are[b * PA + c], bv, d0, 0, 0, 0);
            d1 = __builtin_amdgcn_mfma_f32_16x16x4f32(aim[b * PA + c], bv, d1, 0, 0, 0);
          }
        }
        // lane 16 r + j: RHS 4r..4r+3 of column j
        if (e < n1) {
          const float er = sm.rat[n][0], ei = sm.rat[n][1];
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const float vr = d0[v], vi = d1[v];
            sm.acc[n][4 * la + v].re += er * vr - ei * vi;
            sm.acc[n][4 * la + v].im += er * vi + ei * vr;
          }
        }
      }
    }
  }
  // node values -> coefficients, in place, one line of one RHS per thread and pass
  __syncthreads();
  for (int t = threadIdx.x; t < PA * PA * MF_RG; t += TPB) {   // over a (s)
    const int bc = t / MF_RG, r = t % MF_RG;
    cpx<float> v[PS], w[PS];
#pragma unroll
    for (int a = 0; a < PS; ++a) v[a] = sm.acc[a * PA * PA + bc][r];
#pragma unroll
    for (int i = 0; i < PS; ++i) {
      w[i] = {0.f, 0.f};
#pragma unroll
      for (int a = 0; a < PS; ++a) {
        w[i].re += sm.ms[i * PS + a] * v[a].re;
        w[i].im += sm.ms[i * PS + a] * v[a].im;
      }
    }
#pragma unroll
    for (int i = 0; i < PS; ++i) sm.acc[i * PA * PA + bc][r] = w[i];
  }
  __syncthreads();
  for (int t = threadIdx.x; t < PS * PA * MF_RG; t += TPB) {   // over b (theta)
    const int ic = t / MF_RG, r = t % MF_RG, i = ic / PA, c = ic % PA;
    cpx<float> v[PA], w[PA];
#pragma unroll
    for (int b = 0; b < PA; ++b) v[b] = sm.acc[(i * PA + b) * PA + c][r];
#pragma unroll
    for (int j = 0; j < PA; ++j) {
      w[j] = {0.f, 0.f};
#pragma unroll
      for (int b = 0; b < PA; ++b) {
        w[j].re += sm.ma[j * PA + b] * v[b].re;
        w[j].im += sm.ma[j * PA + b] * v[b].im;
      }
    }
#pragma unroll
    for (int j = 0; j < PA; ++j) sm.acc[(i * PA + j) * PA + c][r] = w[j];
  }
  __syncthreads();
  for (int t = threadIdx.x; t < PS * PA * MF_RG; t += TPB) {   // over c (phi)
    const int ij = t / MF_RG, r = t % MF_RG;
    cpx<float> v[PA], w[PA];
#pragma unroll
    for (int c = 0; c < PA; ++c) v[c] = sm.acc[ij * PA + c][r];
#pragma unroll
    for (int l = 0; l < PA; ++l) {
      w[l] = {0.f, 0.f};
#pragma unroll
      for (int c = 0; c < PA; ++c) {
        w[l].re += sm.ma[l * PA + c] * v[c].re;
        w[l].im += sm.ma[l * PA + c] * v[c].im;
      }
    }
#pragma unroll
    for (int l = 0; l < PA; ++l) sm.acc[ij * PA + l][r] = w[l];
  }
  __syncthreads();
  for (int t = threadIdx.x; t < P * MF_RG; t += TPB) {
    const int n = t / MF_RG, r = t % MF_RG;
    Fc_up[((int64_t)sp * P + n) * R + g * MF_RG + r] = sm.acc[n][r];
  }
}

// ---------------------------------------------------------------------------
// Cone-major upward pass on MFMA (FP32, one right-hand side).
//
// Every box of a level has the same size, so the position of parent node
// (a, b, c) of parent cone id q relative to the centre of the child in
// octant o - hence its child cone, local coordinates and the ratio
// K(x, y_B)/K(x, y_P) - depends on (q, o, node) only, not on the box; the
// plan computes these node records once per (q, o), grouped by child cone
// (k_ti_geo).  A work item is one cone id q and up to 8 NW parent boxes
// holding it.  For each octant the block copies q's records into LDS; the
// boxes that have a child in octant o are packed into row blocks of 8, and
// the (row block, column tile) units are split evenly over the waves.  A
// unit evaluates the child interpolants of 8 boxes at 16 nodes of a group
// as the product
//     OUT[row][e] = sum_k C[row][k] B[k][e],
// rows = 8 boxes x (re, im) of the child cone's coefficients, columns = 16
// nodes of the group, B[k][e] = T_a(ts_e) T_b(tt_e) T_c(tp_e), on
// v_mfma_f32_16x16x4_f32 with the basis index ordered (b, c, a) so that a
// fills the 4-wide K step.  The wave adds ratio * OUT to the boxes' node
// values in LDS (each (box, node) has one writer per octant, octants in
// order: deterministic).  After the 8 octants the node values are turned
// into coefficients in place and written to the parent level.
//
// Latency hiding: the records of the next octant with children are in LDS
// before the current octant's MFMA phase (two buffers), so that a wave's
// A-operand pipeline runs on from its last segment in one octant into its
// first in the next.
// ---------------------------------------------------------------------------
// A run of a wave's work units with the same row block and group: octant
// k (0: current, 1: next; SEG_NONE / SEG_UNKNOWN: none, or not known yet),
// row block r, group g, units u .. ue-1.
constexpr int SEG_NONE = -1, SEG_UNKNOWN = -2;
struct Seg {
  int k, r, g, u, ue;
};

// The nodes of parent cone id q in the frame of the child in octant o,
// grouped by child cone, in group order.  The same for every box of a level:
// the plan computes one per (cone id, octant) of the cone-major tiles.
template <int PS, int PA> struct alignas(16) TiGeo {
  static constexpr int P = PS * PA * PA;
  float4 loc[P];               // (ts, tt, tp, -): local coordinates in the node's child cone
  float2 rat[P];               // ratio K(x, y_B) / K(x, y_P)
  short node[P];               // node index
  short gstart[P + 1];         // group g: entries gstart[g] .. gstart[g+1]-1
  short tstart[P + 1];         // group g: column tiles tstart[g] .. tstart[g+1]-1 (16 entries each)
  short tgrp[P + P / 16 + 1];  // group of each column tile
  int gcid[P];                 // child cone id of group g
  int ngroup;
};

// One TiGeo record per work-group: (cone id qlist[b / 8], octant b % 8), node
// n on thread n; geometry, grouping by child cone (wave 0), then the records
// in group order.
template <int PS, int PA>
__global__ __launch_bounds__(256) void k_ti_geo(const int* __restrict__ qlist, LevelGeom gp, LevelGeom gc,
                                                ChebTab ct, double k, int kind, TiGeo<PS, PA>* __restrict__ out) {
  using Geo = TiGeo<PS, PA>;
  constexpr int P = Geo::P;
  static_assert(P <= 256, "one node per thread");
  __shared__ Geo G;
  __shared__ int cid[P];
  __shared__ short rank[P];
  const int q = qlist[blockIdx.x >> 3], o = blockIdx.x & 7;
  const int n = threadIdx.x, lane = n & 63, wv = n >> 6;
  float4 loc = make_float4(0.f, 0.f, 0.f, 0.f);
  float2 rat = make_float2(0.f, 0.f);
  if (n < P) {
    float x[3], rp;   // node relative to the parent centre
    node_rel32(q, n / (PA * PA), (n / PA) % PA, n % PA, gp, ct, x, &rp);
    const PropF pr = child_loc32(x, rp, o, gc);
    cid[n] = pr.loc.cid;
    loc = make_float4(pr.loc.ts, pr.loc.tt, pr.loc.tp, 0.f);
    float c_ = 1.f, s_ = 0.f, rr = 1.f;
    if (kind != IFGF_KERNEL_CONSTANT) {
      sincos_f((float)k * pr.dr, &s_, &c_);
      rr = pr.rp_over_rc;
    }
    rat = make_float2(rr * c_, rr * s_);
  }
  __syncthreads();
  if (wv == 0) {   // groups in order of first appearance; ranks within them
    constexpr int NPL = (P + 63) / 64;   // nodes per lane
    int cv[NPL];
    bool pend[NPL];
#pragma unroll
    for (int m = 0; m < NPL; ++m) {
      const int nn = lane + 64 * m;
      pend[m] = nn < P;
      cv[m] = pend[m] ? cid[nn] : 0;
    }
    int pos = 0, g = 0, tpos = 0;
    while (true) {
      int lead = -1, su = 0;
#pragma unroll
      for (int m = 0; m < NPL && lead < 0; ++m) {
        const uint64_t b = __ballot(pend[m]);
        if (b) {
          lead = first_lane(b);
          su = __builtin_amdgcn_readfirstlane(__shfl(cv[m], lead, 64));
        }
      }
      if (lead < 0) break;
      if (lane == 0) {
        G.gstart[g] = (short)pos;
        G.tstart[g] = (short)tpos;
        G.gcid[g] = su;
      }
      const int pos0 = pos;
#pragma unroll
      for (int m = 0; m < NPL; ++m) {
        const bool hit = pend[m] && cv[m] == su;
        const uint64_t b = __ballot(hit);
        if (hit) rank[lane + 64 * m] = (short)(pos + __popcll(b & ((1ull << lane) - 1)));
        pos += __popcll(b);
        pend[m] = pend[m] && !hit;
      }
      const int nt = (pos - pos0 + 15) >> 4;   // at most ceil(P / 16) <= 64 column tiles
      if (lane < nt) G.tgrp[tpos + lane] = (short)g;
      tpos += nt;
      ++g;
    }
    if (lane == 0) {
      G.gstart[g] = (short)pos;
      G.tstart[g] = (short)tpos;
      G.ngroup = g;
    }
  }
  __syncthreads();
  if (n < P) {
    const int r = rank[n];
    G.loc[r] = loc;
    G.rat[r] = rat;
    G.node[r] = (short)n;
  }
  __syncthreads();
  const uint4* src = reinterpret_cast<const uint4*>(&G);
  uint4* dst = reinterpret_cast<uint4*>(out + blockIdx.x);
  for (int i = threadIdx.x; i < (int)(sizeof(Geo) / 16); i += 256) dst[i] = src[i];
}

template <int PS, int PA, int NW> struct TiSmem {
  static constexpr int P = PS * PA * PA;
  static constexpr int NB = 8 * NW;
  // Row stride padded so that lanes reading different boxes fall in
  // different LDS banks; columns P and P + 1 of row NB take unused updates.
  static constexpr int ACC_LD = P + 4;
  using Geo = TiGeo<PS, PA>;
  cpx<float> acc[NB + 1][ACC_LD];  // node values of the tile's boxes; row NB takes unused updates
  Geo geo[2];
  int child[NB][8];            // child box per (box, octant), -1 if none
  signed char olist[8][NB];    // per octant: the tile's boxes with a child there, ascending
  int ocnt[8];
  int pslot[NB];               // parent slot of each box
  float ms[PS * PS], ma[PA * PA];
};

// One tile tl = (cone id, first index into ti_slot, boxes, index of the cone
// id's records in ti_geo) by a block of 64 NW threads; ti_child[8 i + o] is
// the child in octant o of the box of ti_slot[i] (-1 if none), ti_geo[8 j + o]
// the node records of octant o of the tile's cone id.
template <int PS, int PA, int NW>
__device__ __forceinline__ void prop_ti_tile(TiSmem<PS, PA, NW>& sm, int4 tl, const int* __restrict__ ti_slot,
                                             const int* __restrict__ ti_child,
                                             const TiGeo<PS, PA>* __restrict__ ti_geo, const int* __restrict__ slot_c,
                                             const cpx<float>* __restrict__ Fc_c, const LevelGeom& gp,
                                             const LevelGeom& gc, const ChebTab& ct, const float* __restrict__ Ms,
                                             const float* __restrict__ Ma, double k, int kind,
                                             cpx<float>* __restrict__ Fc_up, int* __restrict__ err) {
  using S = TiSmem<PS, PA, NW>;
  constexpr int P = S::P;
  constexpr int NB = S::NB;
  constexpr int BS = 64 * NW;
  const int nb = tl.z;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;

  // ---- set-up: boxes, their children by octant -----------------------------------
  if (threadIdx.x < PS * PS) sm.ms[threadIdx.x] = Ms[threadIdx.x];
  if (threadIdx.x < PA * PA) sm.ma[threadIdx.x] = Ma[threadIdx.x];
  for (int t = threadIdx.x; t < NB * 8; t += BS)
    sm.child[t >> 3][t & 7] = (t >> 3) < nb ? ti_child[(int64_t)(tl.y + (t >> 3)) * 8 + (t & 7)] : -1;
  if (threadIdx.x < nb) sm.pslot[threadIdx.x] = ti_slot[tl.y + threadIdx.x];
  for (int t = threadIdx.x; t < NB * S::ACC_LD; t += BS) sm.acc[t / S::ACC_LD][t % S::ACC_LD] = {0.f, 0.f};
  __syncthreads();
  // per octant, the boxes that have a child in it (MFMA rows are packed with
  // them): every wave forms the octant mask, wave 0 writes the lists
  static_assert(NB <= 64, "one lane per box");
  int anychild = 0;
#pragma unroll
  for (int o = 0; o < 8; ++o) {
    const bool has = lane < nb && sm.child[lane < nb ? lane : 0][o] >= 0;
    const uint64_t b = __ballot(has);
    anychild |= b ? 1 << o : 0;
    if (wv == 0) {
      if (has) sm.olist[o][__popcll(b & ((1ull << lane) - 1))] = (signed char)lane;
      if (lane == 0) sm.ocnt[o] = __popcll(b);
    }
  }
  auto next_oct = [&](int o) -> int {  // next octant with children after o, -1 if none
    const int m = o < 0 ? anychild : anychild & ~((2 << o) - 1);
    return m ? __builtin_ctz(m) : -1;
  };

  // ---- an octant's node records, from the plan's table ---------------------------
  auto fetch = [&](typename S::Geo& dst, int oo) {
    const uint4* src = reinterpret_cast<const uint4*>(ti_geo + (int64_t)tl.w * 8 + oo);
    uint4* d = reinterpret_cast<uint4*>(&dst);
    for (int i = threadIdx.x; i < (int)(sizeof(typename S::Geo) / 16); i += BS) d[i] = src[i];
  };

  // this lane's A rows and B columns; in each octant, the wave's 8 rows are
  // entries 8 wv .. 8 wv + 7 of that octant's box list
  const int li = lane & 15;       // A row (box, re/im) and B / OUT column
  const int la = lane >> 4;       // index within the 4-wide K step: the radial index a
  const int reim = li & 1;

  // Where a row is 16-byte aligned (P = 144) the two lanes of a box (re row,
  // im row; neighbours) each load every other 16-byte chunk of the cone's
  // slab - 2 coefficients, re and im - and swap the halves the other one
  // needs (DPP between neighbouring lanes): 9 loads and 36 registers per row
  // and group, so that this group's operand and the next group's loads in
  // flight stay within what the vector-memory counter tracks and within 3
  // waves per SIMD.
  constexpr bool QUAD = (PA * PA) % 4 == 0;
  constexpr int NRAW = QUAD ? PA * PA / 4 : PA * PA;
  using Raw = typename std::conditional<QUAD, float4, float2>::type;
  auto load_raw = [&](int sl, Raw(&dst)[NRAW]) {
    if (sl >= 0 && la < PS) {
      const cpx<float>* row = Fc_c + (int64_t)sl * P + la * PA * PA;
      if constexpr (QUAD) {
        const float4* src = reinterpret_cast<const float4*>(row) + reim;   // chunks 2u + reim
#pragma unroll
        for (int u = 0; u < NRAW; ++u) dst[u] = src[2 * u];
      } else {
#pragma unroll
        for (int u = 0; u < NRAW; ++u) dst[u] = reinterpret_cast<const float2*>(row)[u];
      }
    } else {
#pragma unroll
      for (int u = 0; u < NRAW; ++u) {
        if constexpr (QUAD) dst[u] = make_float4(0.f, 0.f, 0.f, 0.f);
        else dst[u] = make_float2(0.f, 0.f);
      }
    }
  };
  auto unpack = [&](const Raw(&raw)[NRAW], float(&dst)[PA * PA]) {
#pragma unroll
    for (int u = 0; u < NRAW; ++u) {
      if constexpr (QUAD) {
        // lane re holds (re, im) of coefficients 4u, 4u+1; lane im those of 4u+2, 4u+3
        const float4 v = raw[u];
        const float s0 = reim ? v.x : v.y, s1 = reim ? v.z : v.w;
        const float r0 = __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(s0), 0xB1, 0xF, 0xF, false));
        const float r1 = __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(s1), 0xB1, 0xF, 0xF, false));
        dst[4 * u + 0] = reim ? r0 : v.x;
        dst[4 * u + 1] = reim ? r1 : v.z;
        dst[4 * u + 2] = reim ? v.y : r0;
        dst[4 * u + 3] = reim ? v.w : r1;
      } else {
        dst[u] = reim ? raw[u].y : raw[u].x;
      }
    }
  };
  // the child box of this lane's A row in octant o, -1 if none
  auto row_child = [&](int o) -> int {
    const int le = wv * 8 + (li >> 1);
    return (o >= 0 && le < sm.ocnt[o]) ? sm.child[sm.olist[o][le]][o] : -1;
  };

  // ---- octants ----------------------------------------------------------------------
  int o = next_oct(-1);   // block-uniform; -1 only if no box of the tile has a child
  int cb = 0;             // record buffer of octant o
  if (o >= 0) fetch(sm.geo[0], o);
  // A-operand pipeline state carried from one octant to the next: when
  // primed, av holds the operand of segment cur, the wave's first in the
  // octant, and s_nxt the slot of segment nxt (SEG_UNKNOWN: in an octant
  // whose groups were not known yet).
  bool primed = false;
  float av[PA * PA];
  Raw rn[NRAW];
  Seg cur{SEG_NONE, 0, 0, 0, 0}, nxt{SEG_NONE, 0, 0, 0, 0};
  int s_cur = -1, s_nxt = -1, b_cur = -1, b_nxt = -1;
  while (o >= 0) {
    const int o1 = next_oct(o);
    typename S::Geo& G = sm.geo[cb];
    typename S::Geo& G1 = sm.geo[cb ^ 1];
    __syncthreads();   // G's records visible; G1 no longer read (previous octant's MFMA phase done)
    if (o1 >= 0) fetch(G1, o1);
    __syncthreads();   // G1's records visible

    // ---- child interpolants on MFMA ------------------------------------------------
    // Work units are (row block r: 8 boxes of the octant's list, column tile
    // t of the groups), r-major; wave wv takes the units [wv U / NW,
    // (wv + 1) U / NW), so every wave has about the same share whatever the
    // octant's box count.  A run of units with the same (r, group) is a
    // segment and needs one A operand (the 8 boxes' coefficients of the
    // group's child cone).  A wave's segments continue into octant o1, whose
    // groups are known: while a segment is evaluated, the A operand of the
    // next one and the slot of the one after are in flight, across the
    // octant boundary too.  Units are disjoint in (box, node), so the waves'
    // LDS accumulations within an octant never meet.
    const int no = sm.ocnt[o], T = G.tstart[G.ngroup];
    const int U = ((no + 7) >> 3) * T, u0 = wv * U / NW, u1 = (wv + 1) * U / NW;
    const int no1 = o1 >= 0 ? sm.ocnt[o1] : 0, T1 = o1 >= 0 ? G1.tstart[G1.ngroup] : 0;
    const int U1 = ((no1 + 7) >> 3) * T1, v0 = wv * U1 / NW, v1 = (wv + 1) * U1 / NW;
    auto decode = [&](int kk, int u) -> Seg {   // the segment of unit u of octant o (kk = 0) or o1 (kk = 1)
      const int TT = kk ? T1 : T, ue = kk ? v1 : u1;
      const typename S::Geo& GG = kk ? G1 : G;
      const int r = u / TT, g = GG.tgrp[u - r * TT];
      return Seg{kk, r, g, u, min(ue, r * TT + GG.tstart[g + 1])};
    };
    auto after = [&](const Seg& sg) -> Seg {   // the next segment of this wave's stream
      if (sg.k == 0) {
        if (sg.ue < u1) return decode(0, sg.ue);
        if (v0 < v1) return decode(1, v0);
        return Seg{o1 >= 0 ? SEG_UNKNOWN : SEG_NONE, 0, 0, 0, 0};
      }
      if (sg.k == 1 && sg.ue < v1) return decode(1, sg.ue);
      return Seg{sg.k == SEG_NONE ? SEG_NONE : SEG_UNKNOWN, 0, 0, 0, 0};
    };
    // slot of a segment's cone for this lane's A row (bc: the row's child box, -1 if none)
    auto slot_of = [&](const Seg& sg, int& bc) -> int {
      bc = -1;
      if (sg.k < 0) return -1;
      const int oo = sg.k ? o1 : o;
      const int le = sg.r * 8 + (li >> 1);
      if (le < sm.ocnt[oo]) bc = sm.child[sm.olist[oo][le]][oo];
      return bc >= 0 ? slot_c[(int64_t)bc * gc.ncone + (sg.k ? G1 : G).gcid[sg.g]] : -1;
    };
    if (!primed) {
      cur = u0 < u1 ? decode(0, u0) : (v0 < v1 ? decode(1, v0) : Seg{o1 >= 0 ? SEG_UNKNOWN : SEG_NONE, 0, 0, 0, 0});
      nxt = after(cur);
      s_cur = slot_of(cur, b_cur);
      s_nxt = slot_of(nxt, b_nxt);
      load_raw(s_cur, rn);
      unpack(rn, av);
    } else if (nxt.k == SEG_UNKNOWN) {   // known now that its octant is this one or o1
      nxt = after(cur);
      s_nxt = slot_of(nxt, b_nxt);
    }
    // The accumulation of a column tile is deferred to the next tile's
    // iteration (the first time: zeros to the spare row), so that it can run
    // under that tile's MFMAs.  A column past its group gets a zero basis;
    // its entries, and rows past the octant's list, go to row NB, the b entry
    // to column P + 1 there, so that the two entries of a lane never
    // coincide and both can be read before either is written.
    floatx4 dq = {0.f, 0.f, 0.f, 0.f};
    float2 qr = make_float2(0.f, 0.f);
    int qn = 0, qa = NB, qb = NB;
    auto flush = [&]() {
      cpx<float>& ua = sm.acc[qa][qn];
      cpx<float>& ub = sm.acc[qb][qb == NB ? P + 1 : qn];
      cpx<float> va = ua, vb = ub;
      va.re += qr.x * dq[0] - qr.y * dq[1];
      va.im += qr.x * dq[1] + qr.y * dq[0];
      vb.re += qr.x * dq[2] - qr.y * dq[3];
      vb.im += qr.x * dq[3] + qr.y * dq[2];
      ua = va;
      ub = vb;
    };
    while (cur.k == 0) {   // wave-uniform
      const Seg nn = after(nxt);
      int b_nn;
      const int s_nn = slot_of(nn, b_nn);
      load_raw(s_nxt, rn);
      if (b_cur >= 0 && s_cur < 0) atomicOr(err, 2);
      const int g = cur.g, t0 = cur.r * T + G.tstart[g];
      const int n0 = G.gstart[g], n1 = G.gstart[g + 1];
      // lane 16 r + j holds rows 4r..4r+3 = boxes 2r, 2r+1 (re, im) of column j
      const int e2a = cur.r * 8 + 2 * la, e2b = e2a + 1;
      const int bxa = e2a < no ? (int)sm.olist[o][e2a] : NB, bxb = e2b < no ? (int)sm.olist[o][e2b] : NB;
      for (int u = cur.u; u < cur.ue; ++u) {
        const int e = n0 + 16 * (u - t0) + li;
        const bool ok = e < n1;
        const int ee = ok ? e : n0;
        const float4 lc = G.loc[ee];
        const float2 rt = G.rat[ee];
        const int n = G.node[ee];
        float ts[PS], tt[PA], tp[PA];
        cheb_T<float, PS>(lc.x, ts);
        cheb_T<float, PA>(lc.y, tt);
        cheb_T<float, PA>(lc.z, tp);
        float ta = ts[0];
#pragma unroll
        for (int a = 1; a < PS; ++a) ta = la == a ? ts[a] : ta;
        ta = (ok && la < PS) ? ta : 0.f;
        flush();   // the previous tile's
        floatx4 d = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int b = 0; b < PA; ++b) {
          const float w = ta * tt[b];
#pragma unroll
          for (int c = 0; c < PA; ++c) d = __builtin_amdgcn_mfma_f32_16x16x4f32(av[b * PA + c], w * tp[c], d, 0, 0, 0);
        }
        dq = d;
        qr = rt;
        qn = n;
        qa = ok ? bxa : NB;
        qb = ok ? bxb : NB;
      }
      unpack(rn, av);
      cur = nxt;
      nxt = nn;
      s_cur = s_nxt;
      s_nxt = s_nn;
      b_cur = b_nxt;
      b_nxt = b_nn;
    }
    flush();
    primed = cur.k == 1;   // av holds the operand of cur, a segment of octant o1
    if (cur.k == 1) cur.k = 0;   // octant o1 becomes the current one
    if (nxt.k == 1) nxt.k = 0;
    o = o1;
    cb ^= 1;
  }
  __syncthreads();

  // ---- node values -> coefficients, in place, then to the parent level -------------
  for (int t = threadIdx.x; t < nb * PA * PA; t += BS) {   // over a (s)
    const int bx = t / (PA * PA), r = t % (PA * PA);
    cpx<float> v[PS], w[PS];
#pragma unroll
    for (int a = 0; a < PS; ++a) v[a] = sm.acc[bx][a * PA * PA + r];
#pragma unroll
    for (int i = 0; i < PS; ++i) {
      w[i] = {0.f, 0.f};
#pragma unroll
      for (int a = 0; a < PS; ++a) {
        w[i].re += sm.ms[i * PS + a] * v[a].re;
        w[i].im += sm.ms[i * PS + a] * v[a].im;
      }
    }
#pragma unroll
    for (int i = 0; i < PS; ++i) sm.acc[bx][i * PA * PA + r] = w[i];
  }
  __syncthreads();
  for (int t = threadIdx.x; t < nb * PS * PA; t += BS) {   // over b (theta)
    const int bx = t / (PS * PA), i = (t / PA) % PS, c = t % PA;
    cpx<float> v[PA], w[PA];
#pragma unroll
    for (int b = 0; b < PA; ++b) v[b] = sm.acc[bx][(i * PA + b) * PA + c];
#pragma unroll
    for (int j = 0; j < PA; ++j) {
      w[j] = {0.f, 0.f};
#pragma unroll
      for (int b = 0; b < PA; ++b) {
        w[j].re += sm.ma[j * PA + b] * v[b].re;
        w[j].im += sm.ma[j * PA + b] * v[b].im;
      }
    }
#pragma unroll
    for (int j = 0; j < PA; ++j) sm.acc[bx][(i * PA + j) * PA + c] = w[j];
  }
  __syncthreads();
  for (int t = threadIdx.x; t < nb * PS * PA; t += BS) {   // over c (phi)
    const int bx = t / (PS * PA), i = (t / PA) % PS, j = t % PA;
    cpx<float> v[PA], w[PA];
#pragma unroll
    for (int c = 0; c < PA; ++c) v[c] = sm.acc[bx][(i * PA + j) * PA + c];
#pragma unroll
    for (int l = 0; l < PA; ++l) {
      w[l] = {0.f, 0.f};
#pragma unroll
      for (int c = 0; c < PA; ++c) {
        w[l].re += sm.ma[l * PA + c] * v[c].re;
        w[l].im += sm.ma[l * PA + c] * v[c].im;
      }
    }
#pragma unroll
    for (int l = 0; l < PA; ++l) sm.acc[bx][(i * PA + j) * PA + l] = w[l];
  }
  __syncthreads();
  for (int t = threadIdx.x; t < nb * P; t += BS) {
    const int bx = t / P, jn = t % P;
    Fc_up[(int64_t)sm.pslot[bx] * P + jn] = sm.acc[bx][jn];
  }
}

template <int PS, int PA, int NW>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(3))) void k_prop_ti(
    const int4* __restrict__ tiles, const int* __restrict__ ti_slot, const int* __restrict__ ti_child,
    const TiGeo<PS, PA>* __restrict__ ti_geo, const int* __restrict__ slot_c, const cpx<float>* __restrict__ Fc_c,
    LevelGeom gp, LevelGeom gc, ChebTab ct, const float* __restrict__ Ms, const float* __restrict__ Ma, double k,
    int kind, cpx<float>* __restrict__ Fc_up, int* __restrict__ err) {
  __shared__ TiSmem<PS, PA, NW> sm;
  prop_ti_tile<PS, PA, NW>(sm, tiles[xcd_block(blockIdx.x, gridDim.x)], ti_slot, ti_child, ti_geo, slot_c, Fc_c, gp,
                           gc, ct, Ms, Ma, k, kind, Fc_up, err);
}

// ---------------------------------------------------------------------------
// Cone-major upward pass in FP64 on v_mfma_f64_16x16x4_f64 (one right-hand
// side): the scheme of prop_ti_tile with complex double coefficients and node
// values.  Tiles hold up to 8 NW boxes (NW <= 2).  The nodes' local
// coordinates (ts, tt, tp) are kept in LDS and each lane forms the Chebyshev
// basis of its column, which keeps a 2-wave block under 49 KB of LDS.  The A
// operand: the two lanes of a box (re row, im row; neighbours) each load every
// other complex coefficient of the cone's slab and swap the halves the other
// one needs (64-bit DPP between neighbouring lanes).
// ---------------------------------------------------------------------------
typedef double doublex4 __attribute__((ext_vector_type(4)));

// FP64 node records of one (cone id, octant), in group order (as TiGeo).
template <int PS, int PA> struct alignas(16) TiGeo64 {
  static constexpr int P = PS * PA * PA;
  double crd[P][3];            // (ts, tt, tp): local coordinates in the node's child cone
  double rat[P][2];            // ratio K(x, y_B) / K(x, y_P)
  short node[P];               // node index
  short gstart[P + 1];         // group g: entries gstart[g] .. gstart[g+1]-1
  short tstart[P + 1];         // group g: column tiles tstart[g] .. tstart[g+1]-1
  short tgrp[P + P / 16 + 1];  // group of each column tile
  int gcid[P];                 // child cone id of group g
  int ngroup;
};

// One TiGeo64 record per work-group: (cone id qlist[b / 8], octant b % 8), node
// n on thread n (the scheme of k_ti_geo in FP64).
template <int PS, int PA>
__global__ __launch_bounds__(256) void k_ti_geo64(const int* __restrict__ qlist, LevelGeom gp, LevelGeom gc,
                                                  ChebTab ct, double k, int kind, TiGeo64<PS, PA>* __restrict__ out) {
  using Geo = TiGeo64<PS, PA>;
  constexpr int P = Geo::P;
  static_assert(P <= 256, "one node per thread");
  __shared__ Geo G;
  __shared__ int cid[P];
  __shared__ short rank[P];
  const int q = qlist[blockIdx.x >> 3], o = blockIdx.x & 7;
  const int n = threadIdx.x, lane = n & 63, wv = n >> 6;
  double ts = 0, tt = 0, tp = 0, r0 = 0, r1 = 0;
  if (n < P) {
    double x[3], rp;   // node relative to the parent centre
    node_rel64(q, n / (PA * PA), (n / PA) % PA, n % PA, gp, ct, x, &rp);
    const Prop64 pr = child_loc64(x, rp, o, gc);
    cid[n] = pr.loc.cid;
    ts = pr.loc.ts;
    tt = pr.loc.tt;
    tp = pr.loc.tp;
    double c_ = 1.0, s_ = 0.0, rr = 1.0;
    if (kind != IFGF_KERNEL_CONSTANT) {
      sincos(k * pr.dr, &s_, &c_);
      rr = pr.rp_over_rc;
    }
    r0 = rr * c_;
    r1 = rr * s_;
  }
  __syncthreads();
  if (wv == 0) {   // groups in order of first appearance; ranks within them
    constexpr int NPL = (P + 63) / 64;
    int cv[NPL];
    bool pend[NPL];
#pragma unroll
    for (int m = 0; m < NPL; ++m) {
      const int nn = lane + 64 * m;
      pend[m] = nn < P;
      cv[m] = pend[m] ? cid[nn] : 0;
    }
    int pos = 0, g = 0, tpos = 0;
    while (true) {
      int lead = -1, su = 0;
#pragma unroll
      for (int m = 0; m < NPL && lead < 0; ++m) {
        const uint64_t b = __ballot(pend[m]);
        if (b) {
          lead = first_lane(b);
          su = __builtin_amdgcn_readfirstlane(__shfl(cv[m], lead, 64));
        }
      }
      if (lead < 0) break;
      if (lane == 0) {
        G.gstart[g] = (short)pos;
        G.tstart[g] = (short)tpos;
        G.gcid[g] = su;
      }
      const int pos0 = pos;
#pragma unroll
      for (int m = 0; m < NPL; ++m) {
        const bool hit = pend[m] && cv[m] == su;
        const uint64_t b = __ballot(hit);
        if (hit) rank[lane + 64 * m] = (short)(pos + __popcll(b & ((1ull << lane) - 1)));
        pos += __popcll(b);
        pend[m] = pend[m] && !hit;
      }
      const int nt = (pos - pos0 + 15) >> 4;
      if (lane < nt) G.tgrp[tpos + lane] = (short)g;
      tpos += nt;
      ++g;
    }
    if (lane == 0) {
      G.gstart[g] = (short)pos;
      G.tstart[g] = (short)tpos;
      G.ngroup = g;
    }
  }
  __syncthreads();
  if (n < P) {
    const int r = rank[n];
    G.crd[r][0] = ts;
    G.crd[r][1] = tt;
    G.crd[r][2] = tp;
    G.rat[r][0] = r0;
    G.rat[r][1] = r1;
    G.node[r] = (short)n;
  }
  __syncthreads();
  const uint4* src = reinterpret_cast<const uint4*>(&G);
  uint4* dst = reinterpret_cast<uint4*>(out + blockIdx.x);
  for (int i = threadIdx.x; i < (int)(sizeof(Geo) / 16); i += 256) dst[i] = src[i];
}

template <int PS, int PA, int NW> struct Ti64Smem {
  static constexpr int P = PS * PA * PA;
  static constexpr int NB = 8 * NW;
  static constexpr int ACC_LD = P + 1;
  cpx<double> acc[NB + 1][ACC_LD];  // node values of the tile's boxes; row NB takes unused updates
  TiGeo64<PS, PA> geo;              // the current octant's node records
  int child[NB][8];
  signed char olist[8][NB];
  int ocnt[8];
  int pslot[NB];
  double ms[PS * PS], ma[PA * PA];
};

__device__ __forceinline__ double swap_lane_pair(double v) {
  const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
  const int lo = __builtin_amdgcn_mov_dpp((int)(unsigned)b, 0xB1, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(unsigned)(b >> 32), 0xB1, 0xF, 0xF, false);
  return __builtin_bit_cast(double, (unsigned long long)(unsigned)lo | ((unsigned long long)(unsigned)hi << 32));
}

template <int PS, int PA, int NW>
__device__ __forceinline__ void prop_ti64_tile(Ti64Smem<PS, PA, NW>& sm, int4 tl, const int* __restrict__ ti_slot,
                                               const int* __restrict__ ti_child,
                                               const TiGeo64<PS, PA>* __restrict__ ti_geo,
                                               const int* __restrict__ slot_c, const cpx<double>* __restrict__ Fc_c,
                                               const LevelGeom& gp, const LevelGeom& gc, const ChebTab& ct,
                                               const double* __restrict__ Ms, const double* __restrict__ Ma,
                                               double k, int kind, cpx<double>* __restrict__ Fc_up,
                                               int* __restrict__ err) {
  using S = Ti64Smem<PS, PA, NW>;
  constexpr int P = S::P;
  constexpr int NB = S::NB;
  constexpr int BS = 64 * NW;
  const int nb = tl.z;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;

  // ---- set-up: boxes, their children by octant ----------------------------------
  if (threadIdx.x < PS * PS) sm.ms[threadIdx.x] = Ms[threadIdx.x];
  if (threadIdx.x < PA * PA) sm.ma[threadIdx.x] = Ma[threadIdx.x];
  for (int t = threadIdx.x; t < NB * 8; t += BS)   // each box's children by octant, from the plan
    sm.child[t >> 3][t & 7] = (t >> 3) < nb ? ti_child[(int64_t)(tl.y + (t >> 3)) * 8 + (t & 7)] : -1;
  if (threadIdx.x < nb) sm.pslot[threadIdx.x] = ti_slot[tl.y + threadIdx.x];
  for (int t = threadIdx.x; t < NB * S::ACC_LD; t += BS) sm.acc[t / S::ACC_LD][t % S::ACC_LD] = {0.0, 0.0};
  __syncthreads();
  // per octant, the boxes that have a child in it: every wave forms the
  // octant mask, wave 0 writes the lists (read after the next barrier)
  static_assert(NB <= 64, "one lane per box");
  int anychild = 0;
#pragma unroll
  for (int o = 0; o < 8; ++o) {
    const bool has = lane < nb && sm.child[lane < nb ? lane : 0][o] >= 0;
    const uint64_t b = __ballot(has);
    anychild |= b ? 1 << o : 0;
    if (wv == 0) {
      if (has) sm.olist[o][__popcll(b & ((1ull << lane) - 1))] = (signed char)lane;
      if (lane == 0) sm.ocnt[o] = __popcll(b);
    }
  }
  const int li = lane & 15;       // A row (box, re/im) and B / OUT column
  const int la = lane >> 4;       // index within the 4-wide K step: the radial index a
  const int reim = li & 1;

  for (int o = 0; o < 8; ++o) {
    if (!((anychild >> o) & 1)) continue;   // block-uniform
    // ---- the octant's node records, from the plan's table --------------------------
    {
      const uint4* src = reinterpret_cast<const uint4*>(ti_geo + (int64_t)tl.w * 8 + o);
      uint4* d = reinterpret_cast<uint4*>(&sm.geo);
      for (int i = threadIdx.x; i < (int)(sizeof(TiGeo64<PS, PA>) / 16); i += BS) d[i] = src[i];
    }
    __syncthreads();
    const TiGeo64<PS, PA>& G = sm.geo;
    // ---- child interpolants on MFMA ------------------------------------------------
    // Work units (row block r: 8 boxes of the octant's list, column tile t of
    // the groups), r-major, split evenly over the waves; a run of units with
    // the same (r, group) is a segment with one A operand, loaded one segment
    // ahead.  Units are disjoint in (box, node).
    const int ng = G.ngroup;
    const int no = sm.ocnt[o];
    const int T = G.tstart[ng];
    const int U = ((no + 7) >> 3) * T;
    const int u0 = wv * U / NW, u1 = (wv + 1) * U / NW;
    struct Seg64 {
      int r, g, ue;   // r < 0: none
    };
    auto seg_at = [&](int u) -> Seg64 {
      if (u >= u1) return Seg64{-1, 0, u1};
      const int r = u / T, g = G.tgrp[u - r * T];
      return Seg64{r, g, min(u1, r * T + G.tstart[g + 1])};
    };
    auto child_of = [&](const Seg64& sg) -> int {   // the child box of this lane's A row
      const int le = sg.r * 8 + (li >> 1);
      return (sg.r >= 0 && le < no) ? sm.child[sm.olist[o][le]][o] : -1;
    };
    auto slot_of = [&](const Seg64& sg, int Bc) -> int {
      return Bc >= 0 ? slot_c[(int64_t)Bc * gc.ncone + G.gcid[sg.g]] : -1;
    };
    constexpr bool PAIR = (PA * PA) % 2 == 0;
    constexpr int NRAW = PAIR ? PA * PA / 2 : PA * PA;
    auto load_raw = [&](int sl, double2(&dst)[NRAW]) {
      if (sl >= 0 && la < PS) {
        const double2* row = reinterpret_cast<const double2*>(Fc_c + (int64_t)sl * P + la * PA * PA);
#pragma unroll
        for (int u = 0; u < NRAW; ++u) dst[u] = PAIR ? row[2 * u + reim] : row[u];
      } else {
#pragma unroll
        for (int u = 0; u < NRAW; ++u) dst[u] = make_double2(0.0, 0.0);
      }
    };
    auto unpack = [&](const double2(&raw)[NRAW], double(&dst)[PA * PA]) {
#pragma unroll
      for (int u = 0; u < NRAW; ++u) {
        if constexpr (PAIR) {
          // lane re holds coefficient 2u, lane im coefficient 2u + 1 (re, im each)
          const double2 v = raw[u];
          const double r = swap_lane_pair(reim ? v.x : v.y);
          dst[2 * u] = reim ? r : v.x;
          dst[2 * u + 1] = reim ? v.y : r;
        } else {
          dst[u] = reim ? raw[u].y : raw[u].x;
        }
      }
    };
    // The f64 MFMA spreads a lane's four outputs over the rows: element v of
    // lane 16 r + j is row 4 v + r, i.e. box 2 v + (r >> 1), part r & 1, of
    // column j.  Lanes r and r ^ 1 (16 apart) exchange their values, and
    // each lane then adds two boxes: r even elements 0, 1 (boxes r >> 1,
    // 2 + (r >> 1)), r odd elements 2, 3 (boxes 4 + (r >> 1), 6 + (r >> 1)).
    // A tile's accumulation is deferred to the next tile's iteration; unused
    // entries go to row NB (the b entry to column P there).
    const bool odd = la & 1;
    doublex4 dq = {0.0, 0.0, 0.0, 0.0};
    double2 qr = make_double2(0.0, 0.0);
    int qn = 0, qa = NB, qb = NB;
    auto xchg = [](double v) {
      const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
      const int lo = __shfl_xor((int)(unsigned)b, 16, 64), hi = __shfl_xor((int)(unsigned)(b >> 32), 16, 64);
      return __builtin_bit_cast(double, (unsigned long long)(unsigned)lo | ((unsigned long long)(unsigned)hi << 32));
    };
    auto flush = [&]() {
      const double o0 = xchg(dq[0]), o1 = xchg(dq[1]), o2 = xchg(dq[2]), o3 = xchg(dq[3]);
      const double m0 = odd ? dq[2] : dq[0], m1 = odd ? dq[3] : dq[1];
      const double t0 = odd ? o2 : o0, t1 = odd ? o3 : o1;
      const double re0 = odd ? t0 : m0, im0 = odd ? m0 : t0, re1 = odd ? t1 : m1, im1 = odd ? m1 : t1;
      const double er = qr.x, ei = qr.y;
      cpx<double>& ua = sm.acc[qa][qn];
      cpx<double>& ub = sm.acc[qb][qb == NB ? P : qn];
      cpx<double> va = ua, vb = ub;
      va.re += er * re0 - ei * im0;
      va.im += er * im0 + ei * re0;
      vb.re += er * re1 - ei * im1;
      vb.im += er * im1 + ei * re1;
      ua = va;
      ub = vb;
    };
    double av[PA * PA];
    double2 rn[NRAW];
    Seg64 cur = seg_at(u0);
    Seg64 nxt = seg_at(cur.ue);
    int b_cur = child_of(cur), b_nxt = child_of(nxt);
    int s_cur = slot_of(cur, b_cur), s_nxt = slot_of(nxt, b_nxt);
    if (u0 < u1) {
      load_raw(s_cur, rn);
      unpack(rn, av);
    }
    for (int u = u0; u < u1;) {   // wave-uniform
      const Seg64 nn = seg_at(nxt.ue);
      const int b_nn = child_of(nn);
      const int s_nn = slot_of(nn, b_nn);
      load_raw(s_nxt, rn);
      if (b_cur >= 0 && s_cur < 0) atomicOr(err, 2);
      const int g = cur.g, t0 = cur.r * T + G.tstart[g];
      const int n0 = G.gstart[g], n1 = G.gstart[g + 1];
      const int e2a = cur.r * 8 + (odd ? 4 : 0) + (la >> 1), e2b = e2a + 2;
      const int bxa = e2a < no ? (int)sm.olist[o][e2a] : NB, bxb = e2b < no ? (int)sm.olist[o][e2b] : NB;
      for (; u < cur.ue; ++u) {
        const int e = n0 + 16 * (u - t0) + li;
        const bool ok = e < n1;
        const int ee = ok ? e : n0;
        const int n = G.node[ee];
        const double2 rt = make_double2(G.rat[ee][0], G.rat[ee][1]);
        double Ts[PS], Tt[PA], Tp[PA];
        cheb_T<double, PS>(G.crd[ee][0], Ts);
        cheb_T<double, PA>(G.crd[ee][1], Tt);
        cheb_T<double, PA>(G.crd[ee][2], Tp);
        double ta = 0.0;
#pragma unroll
        for (int a = 0; a < PS; ++a)
          if (la == a) ta = Ts[a];
        if (!ok) ta = 0.0;
        flush();   // the previous tile's (the first time: zeros to the spare row)
        doublex4 d = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int b = 0; b < PA; ++b) {
          const double w = ta * Tt[b];
#pragma unroll
          for (int c = 0; c < PA; ++c) d = __builtin_amdgcn_mfma_f64_16x16x4f64(av[b * PA + c], w * Tp[c], d, 0, 0, 0);
        }
        dq = d;
        qr = rt;
        qn = n;
        qa = ok ? bxa : NB;
        qb = ok ? bxb : NB;
      }
      unpack(rn, av);
      cur = nxt;
      nxt = nn;
      s_cur = s_nxt;
      s_nxt = s_nn;
      b_cur = b_nxt;
      b_nxt = b_nn;
    }
    flush();
    __syncthreads();
  }

  // ---- node values -> coefficients, in place, then to the parent level -------------
  for (int t = threadIdx.x; t < nb * PA * PA; t += BS) {   // over a (s)
    const int bx = t / (PA * PA), r = t % (PA * PA);
    cpx<double> v[PS], w[PS];
#pragma unroll
    for (int a = 0; a < PS; ++a) v[a] = sm.acc[bx][a * PA * PA + r];
#pragma unroll
    for (int i = 0; i < PS; ++i) {
      w[i] = {0.0, 0.0};
#pragma unroll
      for (int a = 0; a < PS; ++a) {
        w[i].re += sm.ms[i * PS + a] * v[a].re;
        w[i].im += sm.ms[i * PS + a] * v[a].im;
      }
    }
#pragma unroll
    for (int i = 0; i < PS; ++i) sm.acc[bx][i * PA * PA + r] = w[i];
  }
  __syncthreads();
  for (int t = threadIdx.x; t < nb * PS * PA; t += BS) {   // over b (theta)
    const int bx = t / (PS * PA), i = (t / PA) % PS, c = t % PA;
    cpx<double> v[PA], w[PA];
#pragma unroll
    for (int b = 0; b < PA; ++b) v[b] = sm.acc[bx][(i * PA + b) * PA + c];
#pragma unroll
    for (int j = 0; j < PA; ++j) {
      w[j] = {0.0, 0.0};
#pragma unroll
      for (int b = 0; b < PA; ++b) {
        w[j].re += sm.ma[j * PA + b] * v[b].re;
        w[j].im += sm.ma[j * PA + b] * v[b].im;
      }
    }
#pragma unroll
    for (int j = 0; j < PA; ++j) sm.acc[bx][(i * PA + j) * PA + c] = w[j];
  }
  __syncthreads();
  for (int t = threadIdx.x; t < nb * PS * PA; t += BS) {   // over c (phi)
    const int bx = t / (PS * PA), i = (t / PA) % PS, j = t % PA;
    cpx<double> v[PA], w[PA];
#pragma unroll
    for (int c = 0; c < PA; ++c) v[c] = sm.acc[bx][(i * PA + j) * PA + c];
#pragma unroll
    for (int l = 0; l < PA; ++l) {
      w[l] = {0.0, 0.0};
#pragma unroll
      for (int c = 0; c < PA; ++c) {
        w[l].re += sm.ma[l * PA + c] * v[c].re;
        w[l].im += sm.ma[l * PA + c] * v[c].im;
      }
    }
#pragma unroll
    for (int l = 0; l < PA; ++l) sm.acc[bx][(i * PA + j) * PA + l] = w[l];
  }
  __syncthreads();
  for (int t = threadIdx.x; t < nb * P; t += BS) {
    const int bx = t / P, jn = t % P;
    Fc_up[(int64_t)sm.pslot[bx] * P + jn] = sm.acc[bx][jn];
  }
}

template <int PS, int PA, int NW>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(2))) void k_prop_ti64(
    const int4* __restrict__ tiles, const int* __restrict__ ti_slot, const int* __restrict__ ti_child,
    const TiGeo64<PS, PA>* __restrict__ ti_geo, const int* __restrict__ slot_c, const cpx<double>* __restrict__ Fc_c,
    LevelGeom gp, LevelGeom gc, ChebTab ct, const double* __restrict__ Ms, const double* __restrict__ Ma, double k,
    int kind, cpx<double>* __restrict__ Fc_up, int* __restrict__ err) {
  __shared__ Ti64Smem<PS, PA, NW> sm;
  prop_ti64_tile<PS, PA, NW>(sm, tiles[xcd_block(blockIdx.x, gridDim.x)], ti_slot, ti_child, ti_geo, slot_c, Fc_c, gp,
                             gc, ct, Ms, Ma, k, kind, Fc_up, err);
}

// ---------------------------------------------------------------------------
// Transposed apply.  The forward operator is
//   u = N a + sum_d T_d c_d,  c_D = X L a,  c_{d-1} = X P_d c_d,
// (N near field, L leaf factors, X node values -> coefficients, P_d upward
// pass, T_d cousin-target interpolation, a = w sigma).  Its exact transpose
//   g = N^T v + L^T X^T chat_D,  chat_3 = T_3^T v,
//   chat_d = T_d^T v + P_d^T X^T chat_{d-1}   (d = 4..D),  out = w g,
// is formed stage by stage.  T^T and P^T scatter into coefficient space: the
// lanes of a wave that hit the same cone sum their contributions in LDS and
// add them with one coalesced atomic add per coefficient.
// ---------------------------------------------------------------------------
template <typename T> __device__ __forceinline__ void atomic_add_t(T* p, T v);
template <> __device__ __forceinline__ void atomic_add_t<float>(float* p, float v) { unsafeAtomicAdd(p, v); }
template <> __device__ __forceinline__ void atomic_add_t<double>(double* p, double v) { unsafeAtomicAdd(p, v); }

template <typename T, int PS, int PA> struct AntShape {
  static constexpr int P = PS * PA * PA;
  static constexpr int NF = 2 + PS + 2 * PA;   // weight (re, im) and the three Chebyshev vectors
  static constexpr int NCP = (P + 63) / 64;
};

// For every lane with slot >= 0: G[slot] += wt * (T_a(ts) T_b(tt) T_c(tp))_abc
// (layout [slot][P][R], right-hand side r).  All 64 lanes of the wave call it
// together; fbuf is the wave's LDS buffer of 64 * NF values.
template <typename T, int PS, int PA>
__device__ __forceinline__ void anterp_uniform(cpx<T>* __restrict__ G, int slot, int R, int r, T ts, T tt, T tp,
                                               cpx<T> wt, T* fbuf) {
  using S = AntShape<T, PS, PA>;
  constexpr int P = S::P, NF = S::NF, NCP = S::NCP;
  const int lane = threadIdx.x & 63;
  T* f = fbuf + lane * NF;
  f[0] = wt.re;
  f[1] = wt.im;
  cheb_T<T, PS>(ts, f + 2);
  cheb_T<T, PA>(tt, f + 2 + PS);
  cheb_T<T, PA>(tp, f + 2 + PS + PA);
  int ia[NCP], ib[NCP], ic[NCP];
#pragma unroll
  for (int m = 0; m < NCP; ++m) {
    const int j = min(lane + 64 * m, P - 1);
    ia[m] = 2 + j / (PA * PA);
    ib[m] = 2 + PS + (j / PA) % PA;
    ic[m] = 2 + PS + PA + j % PA;
  }
  __builtin_amdgcn_wave_barrier();
  uint64_t pending = __ballot(slot >= 0);
  while (pending) {
    const int lead = first_lane(pending);
    const int su = __builtin_amdgcn_readfirstlane(__shfl(slot, lead, 64));
    uint64_t grp = __ballot(slot == su);
    pending &= ~grp;
    cpx<T> acc[NCP];
#pragma unroll
    for (int m = 0; m < NCP; ++m) acc[m] = {0, 0};
    while (grp) {
      const int q = first_lane(grp);
      grp &= grp - 1;
      const T* fq = fbuf + q * NF;
      const T wre = fq[0], wim = fq[1];
#pragma unroll
      for (int m = 0; m < NCP; ++m) {
        const T b = fq[ia[m]] * fq[ib[m]] * fq[ic[m]];
        acc[m].re += wre * b;
        acc[m].im += wim * b;
      }
    }
    cpx<T>* dst = G + (int64_t)su * P * R + r;
#pragma unroll
    for (int m = 0; m < NCP; ++m) {
      const int j = lane + 64 * m;
      if (j < P) {
        atomic_add_t<T>(&dst[(int64_t)j * R].re, acc[m].re);
        atomic_add_t<T>(&dst[(int64_t)j * R].im, acc[m].im);
      }
    }
  }
  __builtin_amdgcn_wave_barrier();
}

template <typename T>
__global__ __launch_bounds__(TPB) void k_fill_zero(cpx<T>* __restrict__ x, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (i < n) x[i] = {0, 0};
}

// T_d^T for the levels dlo..dhi: every target x with value v (gathered,
// T precision) scatters v e^{ikr}/(4 pi r) basis(x) into the coefficient
// adjoint of the cone of each box of which it is a cousin point.
template <typename T> struct ALevel {
  const int* pbox;
  const int* cou_off;
  const int* cou;
  const double* centre;
  const int* slot;
  cpx<T>* G;
  LevelGeom g;
};
template <typename T> struct ALevels {
  ALevel<T> lv[IFGF_MAX_LEVELS];
};

template <typename T, int PS, int PA>
__global__ __launch_bounds__(TPB) void k_adj_targets(const double* __restrict__ pts, int64_t n,
                                                     const cpx<T>* __restrict__ vs, ALevels<T> L, int dlo, int dhi,
                                                     double k, int kind, int R, int* __restrict__ err) {
  using S = AntShape<T, PS, PA>;
  __shared__ T fbuf[TPB / 64][64 * S::NF];
  const int r = blockIdx.y;
  const int64_t i0 = (int64_t)xcd_block(blockIdx.x, gridDim.x) * TPB + threadIdx.x;
  const bool valid = i0 < n;
  const int64_t i = valid ? i0 : n - 1;
  const double* x = pts + 3 * i;
  const cpx<T> vi = vs[i * R + r];
  const double inv4pi = 1.0 / (4.0 * IFGF_PI);
  for (int d = dhi; d >= dlo; --d) {
    const ALevel<T>& lv = L.lv[d];
    const int A = lv.pbox[i];
    const int c0 = lv.cou_off[A], cnt = lv.cou_off[A + 1] - c0;
    int cmax = cnt;
    for (int off = 32; off > 0; off >>= 1) cmax = max(cmax, __shfl_xor(cmax, off, 64));
    for (int t = 0; t < cmax; ++t) {
      const bool has = valid && t < cnt;
      const int B = lv.cou[c0 + min(t, max(cnt - 1, 0))];
      T ts = 0, tt = 0, tp = 0, e_re = 0, e_im = 0;
      int sl = -1;
      if (cnt > 0) {
        double rr;
        int cid;
        if constexpr (Prec<T>::f32) {
          LocF loc = target_loc32(x, lv.centre + 3 * B, lv.g, &rr);
          cid = loc.cid;
          ts = loc.ts;
          tt = loc.tt;
          tp = loc.tp;
          float c, s;
          expi_reduced32(k * rr, &c, &s);
          float g = (float)inv4pi / (float)rr;
          e_re = g * c;
          e_im = g * s;
        } else {
          Loc loc = target_loc64(x, lv.centre + 3 * B, lv.g, &rr);
          cid = loc.cid;
          ts = loc.ts;
          tt = loc.tt;
          tp = loc.tp;
          double c, s;
          sincos(k * rr, &s, &c);
          double g = inv4pi / rr;
          e_re = g * c;
          e_im = g * s;
        }
        if (kind == IFGF_KERNEL_CONSTANT) {
          e_re = 1;
          e_im = 0;
        }
        sl = lv.slot[(int64_t)B * lv.g.ncone + cid];
        if (sl < 0 && has) atomicOr(err, 4);
      }
      if (!has) sl = -1;
      const cpx<T> wt = {e_re * vi.re - e_im * vi.im, e_re * vi.im + e_im * vi.re};
      anterp_uniform<T, PS, PA>(lv.G, sl, R, r, ts, tt, tp, wt, fbuf[threadIdx.x >> 6]);
    }
  }
}

// P_{d+1}^T: every node of every relevant cone of a level-d box P, holding
// the node-space adjoint Fhat, scatters ratio * Fhat * basis into the
// coefficient adjoint of the child cone that contains it, for each child.
template <typename T, int PS, int PA>
__global__ __launch_bounds__(TPB) void k_adj_prop(int nrel_up, const int* __restrict__ rel_box_up,
                                                  const int* __restrict__ rel_cone_up,
                                                  const int* __restrict__ child_lo_up, const int* __restrict__ coords,
                                                  const int* __restrict__ slot_c, const cpx<T>* __restrict__ Fhat_up,
                                                  cpx<T>* __restrict__ G_c, LevelGeom gp, LevelGeom gc, ChebTab ct,
                                                  double k, int kind, int R, int* __restrict__ err) {
  using S = AntShape<T, PS, PA>;
  constexpr int P = S::P;
  __shared__ T fbuf[TPB / 64][64 * S::NF];
  const int r = blockIdx.y;
  const int64_t t0 = (int64_t)xcd_block(blockIdx.x, gridDim.x) * TPB + threadIdx.x;
  const bool valid = t0 < (int64_t)nrel_up * P;
  const int64_t t = valid ? t0 : (int64_t)nrel_up * P - 1;
  const int sp = (int)(t / P), node = (int)(t % P);
  const int ai = node / (PA * PA), bi = (node / PA) % PA, ci = node % PA;
  const int Pb = rel_box_up[sp], pcid = rel_cone_up[sp];
  const cpx<T> fh = Fhat_up[((int64_t)sp * P + node) * R + r];
  T x[3], rp;
  if constexpr (Prec<T>::f32) node_rel32(pcid, ai, bi, ci, gp, ct, x, &rp);
  else node_rel64(pcid, ai, bi, ci, gp, ct, x, &rp);
  const int B0 = child_lo_up[Pb], nch = child_lo_up[Pb + 1] - B0;
  int cmax = nch;
  for (int off = 32; off > 0; off >>= 1) cmax = max(cmax, __shfl_xor(cmax, off, 64));
  for (int c = 0; c < cmax; ++c) {
    const bool has = valid && c < nch;
    const int B = B0 + min(c, nch - 1);
    const int oct = (coords[3 * B] & 1) | ((coords[3 * B + 1] & 1) << 1) | ((coords[3 * B + 2] & 1) << 2);
    typename PropGeomT<T>::P pr;
    if constexpr (Prec<T>::f32) pr = child_loc32(x, rp, oct, gc);
    else pr = child_loc64(x, rp, oct, gc);
    int sl = slot_c[(int64_t)B * gc.ncone + pr.loc.cid];
    if (sl < 0 && has) atomicOr(err, 2);
    if (!has) sl = -1;
    T rr = pr.rp_over_rc, c_, s_;
    if (kind == IFGF_KERNEL_CONSTANT) {
      c_ = 1;
      s_ = 0;
      rr = 1;
    } else {
      sincos_t<T>((T)k * pr.dr, &s_, &c_);
    }
    const T rre = rr * c_, rim = rr * s_;
    const cpx<T> wt = {rre * fh.re - rim * fh.im, rre * fh.im + rim * fh.re};
    anterp_uniform<T, PS, PA>(G_c, sl, R, r, pr.loc.ts, pr.loc.tt, pr.loc.tp, wt, fbuf[threadIdx.x >> 6]);
  }
}

// P_{d+1}^T as k_adj_prop, with fewer atomic additions: a wave takes NR
// rounds of 64 consecutive (parent cone, node) items (NR * 64 / P parent
// cones, mostly of one parent box) and, per child, collects the anterpolated
// contributions of all its rounds in a table of up to NT child slots held in
// registers (lane l holds coefficients l + 64 m of every entry).  Each entry
// is added to the child's coefficient adjoint once per wave and child
// instead of once per round; a full table is emptied early.
constexpr int kAdjRounds = 4;   // rounds of 64 items per wave in k_adj_prop_tab (8 measured no faster)

template <typename T, int PS, int PA>
__global__ __launch_bounds__(TPB) void k_adj_prop_tab(int nrel_up, const int* __restrict__ rel_box_up,
                                                      const int* __restrict__ rel_cone_up,
                                                      const int* __restrict__ child_lo_up,
                                                      const int* __restrict__ coords, const int* __restrict__ slot_c,
                                                      const cpx<T>* __restrict__ Fhat_up, cpx<T>* __restrict__ G_c,
                                                      LevelGeom gp, LevelGeom gc, ChebTab ct, double k, int kind, int R,
                                                      int* __restrict__ err) {
  using S = AntShape<T, PS, PA>;
  constexpr int P = S::P, NF = S::NF, NCP = S::NCP;
  constexpr int NR = kAdjRounds;
  constexpr int NT = Prec<T>::f32 ? 6 : 4;
  __shared__ T fbuf[TPB / 64][64 * NF];
  T* fb = fbuf[threadIdx.x >> 6];
  const int lane = threadIdx.x & 63, r = blockIdx.y;
  const int64_t nit = (int64_t)nrel_up * P;
  const int64_t wbase = ((int64_t)xcd_block(blockIdx.x, gridDim.x) * (TPB / 64) + (threadIdx.x >> 6)) * (64 * NR);
  if (wbase >= nit) return;   // wave-uniform; no block barrier below
  T xr[NR][3], rpr[NR];
  cpx<T> fhr[NR];
  int b0r[NR], nchr[NR];
  bool vr[NR];
  int cmax = 0;
#pragma unroll
  for (int q = 0; q < NR; ++q) {
    const int64_t t0 = wbase + 64 * q + lane;
    vr[q] = t0 < nit;
    const int64_t t = vr[q] ? t0 : nit - 1;
    const int sp = (int)(t / P), node = (int)(t % P);
    const int Pb = rel_box_up[sp], pcid = rel_cone_up[sp];
    fhr[q] = Fhat_up[((int64_t)sp * P + node) * R + r];
    if constexpr (Prec<T>::f32) node_rel32(pcid, node / (PA * PA), (node / PA) % PA, node % PA, gp, ct, xr[q], &rpr[q]);
    else node_rel64(pcid, node / (PA * PA), (node / PA) % PA, node % PA, gp, ct, xr[q], &rpr[q]);
    b0r[q] = child_lo_up[Pb];
    nchr[q] = child_lo_up[Pb + 1] - b0r[q];
    if (vr[q]) cmax = max(cmax, nchr[q]);
  }
  for (int off = 32; off > 0; off >>= 1) cmax = max(cmax, __shfl_xor(cmax, off, 64));
  int ia[NCP], ib[NCP], ic[NCP];   // this lane's coefficients in a basis row of fbuf
#pragma unroll
  for (int m = 0; m < NCP; ++m) {
    const int j = min(lane + 64 * m, P - 1);
    ia[m] = 2 + j / (PA * PA);
    ib[m] = 2 + PS + (j / PA) % PA;
    ic[m] = 2 + PS + PA + j % PA;
  }
  T* f = fb + lane * NF;
  for (int c = 0; c < cmax; ++c) {
    int tslot[NT];       // the table's child slots (wave-uniform)
    cpx<T> tacc[NT][NCP];
    int tn = 0;
    auto flush = [&]() {
#pragma unroll
      for (int x = 0; x < NT; ++x) {
        if (x < tn) {
          cpx<T>* dst = G_c + (int64_t)tslot[x] * P * R + r;
#pragma unroll
          for (int m = 0; m < NCP; ++m) {
            const int j = lane + 64 * m;
            if (j < P) {
              atomic_add_t<T>(&dst[(int64_t)j * R].re, tacc[x][m].re);
              atomic_add_t<T>(&dst[(int64_t)j * R].im, tacc[x][m].im);
            }
          }
        }
      }
      tn = 0;
    };
#pragma unroll
    for (int q = 0; q < NR; ++q) {
      const bool has = vr[q] && c < nchr[q];
      const int B = b0r[q] + min(c, nchr[q] - 1);
      const int oct = (coords[3 * B] & 1) | ((coords[3 * B + 1] & 1) << 1) | ((coords[3 * B + 2] & 1) << 2);
      typename PropGeomT<T>::P pr;
      if constexpr (Prec<T>::f32) pr = child_loc32(xr[q], rpr[q], oct, gc);
      else pr = child_loc64(xr[q], rpr[q], oct, gc);
      int sl = slot_c[(int64_t)B * gc.ncone + pr.loc.cid];
      if (sl < 0 && has) atomicOr(err, 2);
      if (!has) sl = -1;
      T rr = pr.rp_over_rc, c_, s_;
      if (kind == IFGF_KERNEL_CONSTANT) {
        c_ = 1;
        s_ = 0;
        rr = 1;
      } else {
        sincos_t<T>((T)k * pr.dr, &s_, &c_);
      }
      const T rre = rr * c_, rim = rr * s_;
      const cpx<T> fh = fhr[q];
      f[0] = rre * fh.re - rim * fh.im;
      f[1] = rre * fh.im + rim * fh.re;
      cheb_T<T, PS>(pr.loc.ts, f + 2);
      cheb_T<T, PA>(pr.loc.tt, f + 2 + PS);
      cheb_T<T, PA>(pr.loc.tp, f + 2 + PS + PA);
      __builtin_amdgcn_wave_barrier();
      uint64_t pending = __ballot(sl >= 0);
      while (pending) {
        const int lead = first_lane(pending);
        const int su = __builtin_amdgcn_readfirstlane(__shfl(sl, lead, 64));
        const uint64_t grp = __ballot(sl == su);
        pending &= ~grp;
        int e = -1;
#pragma unroll
        for (int x = 0; x < NT; ++x)
          if (x < tn && tslot[x] == su) e = x;
        if (e < 0) {   // a new entry (the table emptied first if full)
          if (tn == NT) flush();
          e = tn++;
#pragma unroll
          for (int x = 0; x < NT; ++x)
            if (x == e) {
              tslot[x] = su;
#pragma unroll
              for (int m = 0; m < NCP; ++m) tacc[x][m] = {0, 0};
            }
        }
#pragma unroll
        for (int x = 0; x < NT; ++x) {
          if (x != e) continue;
          uint64_t gg = grp;
          while (gg) {
            const int qq = first_lane(gg);
            gg &= gg - 1;
            const T* fq = fb + qq * NF;
            const T wre = fq[0], wim = fq[1];
#pragma unroll
            for (int m = 0; m < NCP; ++m) {
              const T b = fq[ia[m]] * fq[ib[m]] * fq[ic[m]];
              tacc[x][m].re += wre * b;
              tacc[x][m].im += wim * b;
            }
          }
        }
      }
      __builtin_amdgcn_wave_barrier();   // the round's rows are read before the next round writes them
    }
    flush();
  }
}

// ---------------------------------------------------------------------------
// P^T by gathering, on the levels with node records (the cone-major
// geometry, inverted).  All boxes of a level have one size, so parent node n
// of parent cone id q lands, seen from the child in octant o, in a child cone
// id, at local coordinates and with a ratio that depend on (q, o, n) only:
// the node records of (q, o), grouped by child cone id.  For a child box B
// (octant o) and its relevant cone c, the transposed pass is
//     G[B, c]_j = sum over the record groups (q, o, g) with child cone id c,
//                 over their nodes n, of ratio * Fhat[P(B), q]_n * T_j(coords),
// where Fhat[P(B), q] is zero unless q is relevant at the parent P(B).  A
// wave takes up to 64 child boxes of one (o, c) bucket, one box per lane:
// the group and node data are uniform across the wave, the parent values
// are gathered per lane.  Each G[B, c] has one writer (added onto the
// cousin-target part already there): no atomics, and the same sums in the
// same order on every run.
// ---------------------------------------------------------------------------
template <typename T, int PS, int PA> struct RecOf;
template <int PS, int PA> struct RecOf<float, PS, PA> { using type = TiGeo<PS, PA>; };
template <int PS, int PA> struct RecOf<double, PS, PA> { using type = TiGeo64<PS, PA>; };

template <int PS, int PA>
__device__ __forceinline__ void rec_entry(const TiGeo<PS, PA>& G, int e, float (&c)[3], float (&r)[2]) {
  const float4 l = G.loc[e];
  const float2 q = G.rat[e];
  c[0] = l.x;
  c[1] = l.y;
  c[2] = l.z;
  r[0] = q.x;
  r[1] = q.y;
}
template <int PS, int PA>
__device__ __forceinline__ void rec_entry(const TiGeo64<PS, PA>& G, int e, double (&c)[3], double (&r)[2]) {
  c[0] = G.crd[e][0];
  c[1] = G.crd[e][1];
  c[2] = G.crd[e][2];
  r[0] = G.rat[e][0];
  r[1] = G.rat[e][1];
}

// Coefficients C0 .. C0 + CN - 1 of the lane's child cone, summed over the bucket's groups.
template <typename T, int PS, int PA, int C0, int CN>
__device__ __forceinline__ void adj_gather_chunk(const typename RecOf<T, PS, PA>::type* __restrict__ recs,
                                                 const int2* __restrict__ gref, int g0, int g1,
                                                 const int* __restrict__ qlist, const int* __restrict__ slot_p,
                                                 int ncone_p, int pb, bool valid, const cpx<T>* __restrict__ Fhat_p,
                                                 cpx<T>* __restrict__ out) {
  constexpr int P = PS * PA * PA;
  cpx<T> acc[CN];
#pragma unroll
  for (int jj = 0; jj < CN; ++jj) acc[jj] = {0, 0};
  for (int gi = g0; gi < g1; ++gi) {   // wave-uniform
    const int2 ref = gref[gi];
    const auto& G = recs[ref.x];
    const int q = qlist[ref.x >> 3];
    const int psl = valid ? slot_p[(int64_t)pb * ncone_p + q] : -1;
    if (!__ballot(psl >= 0)) continue;   // no box of the tile has this parent cone
    const cpx<T>* F = Fhat_p + (int64_t)(psl >= 0 ? psl : 0) * P;
    const int e0 = G.gstart[ref.y], e1 = G.gstart[ref.y + 1];
    for (int e = e0; e < e1; ++e) {
      T c[3], r[2];
      rec_entry<PS, PA>(G, e, c, r);
      cpx<T> f = {0, 0};
      if (psl >= 0) f = F[G.node[e]];
      const T ar = r[0] * f.re - r[1] * f.im, ai = r[0] * f.im + r[1] * f.re;
      T Ts[PS], Tt[PA], Tp[PA];
      cheb_T<T, PS>(c[0], Ts);
      cheb_T<T, PA>(c[1], Tt);
      cheb_T<T, PA>(c[2], Tp);
#pragma unroll
      for (int jj = 0; jj < CN; ++jj) {
        const int j = C0 + jj;
        const T b = Ts[j / (PA * PA)] * Tt[(j / PA) % PA] * Tp[j % PA];
        acc[jj].re += ar * b;
        acc[jj].im += ai * b;
      }
    }
  }
  if (valid) {
#pragma unroll
    for (int jj = 0; jj < CN; ++jj) {
      cpx<T> v = out[C0 + jj];
      v.re += acc[jj].re;
      v.im += acc[jj].im;
      out[C0 + jj] = v;
    }
  }
}

template <typename T, int PS, int PA, int C0>
__device__ __forceinline__ void adj_gather_chunks(const typename RecOf<T, PS, PA>::type* __restrict__ recs,
                                                  const int2* __restrict__ gref, int g0, int g1,
                                                  const int* __restrict__ qlist, const int* __restrict__ slot_p,
                                                  int ncone_p, int pb, bool valid, const cpx<T>* __restrict__ Fhat_p,
                                                  cpx<T>* __restrict__ out) {
  constexpr int P = PS * PA * PA;
  constexpr int CH = Prec<T>::f32 ? 48 : 24;   // accumulators per lane per pass
  constexpr int CN = P - C0 < CH ? P - C0 : CH;
  adj_gather_chunk<T, PS, PA, C0, CN>(recs, gref, g0, g1, qlist, slot_p, ncone_p, pb, valid, Fhat_p, out);
  if constexpr (C0 + CN < P)
    adj_gather_chunks<T, PS, PA, C0 + CN>(recs, gref, g0, g1, qlist, slot_p, ncone_p, pb, valid, Fhat_p, out);
}

template <typename T, int PS, int PA>
__global__ __launch_bounds__(64) void k_adj_ti(const int4* __restrict__ tiles, const int* __restrict__ slots,
                                               const int2* __restrict__ gref, const int* __restrict__ gref_off,
                                               const typename RecOf<T, PS, PA>::type* __restrict__ recs,
                                               const int* __restrict__ qlist, const int* __restrict__ rel_box_c,
                                               const int* __restrict__ parent_c, const int* __restrict__ slot_p,
                                               int ncone_p, const cpx<T>* __restrict__ Fhat_p,
                                               cpx<T>* __restrict__ G_c) {
  constexpr int P = PS * PA * PA;
  const int4 tl = tiles[xcd_block(blockIdx.x, gridDim.x)];
  const int lane = threadIdx.x;
  const bool valid = lane < tl.z;
  const int cs = valid ? slots[tl.y + lane] : 0;
  const int pb = valid ? parent_c[rel_box_c[cs]] : 0;
  adj_gather_chunks<T, PS, PA, 0>(recs, gref, gref_off[tl.x], gref_off[tl.x + 1], qlist, slot_p, ncone_p, pb, valid,
                                  Fhat_p, G_c + (int64_t)cs * P);
}

// FP32 with P_s = 4: the same gather on MFMA (v_mfma_f32_16x16x4_f32).  A
// wave takes 8 child boxes of one bucket: rows = 8 boxes x (re, im), K = the
// bucket's nodes, 4 per step (a group's last step padded with zeros), columns
// = the P coefficients in (P_ang / 2)^2 tiles of 16: column 4a + 2 beta +
// gamma of tile t = tb (P_ang / 2) + tc is coefficient (a, b = 2 tb + beta,
// c = 2 tc + gamma).  A lane's (a, beta, gamma) is fixed, so it picks its
// Chebyshev values once per step and each tile's basis value is one product;
// its output addresses are a per-lane base plus a per-tile constant.
// Lane layouts as in the forward kernels: A[i][k] from lane 16k + i, B[k][j]
// from lane 16k + j, D[4q + v][j] in lane 16q + j, element v.
// Per-lane choice between two values (bit set in `mask`: b), as one
// v_cndmask: written out so that the compiler cannot turn a choice between
// neighbouring array elements into an indexed access of a private array.
__device__ __forceinline__ float lane_sel(uint64_t mask, float a, float b) {
  float r;
  asm("v_cndmask_b32_e64 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "s"(mask));
  return r;
}

template <int PA>
__global__ __launch_bounds__(64) void k_adj_ti_mfma(const int4* __restrict__ tiles, const int* __restrict__ slots,
                                                    const int2* __restrict__ gref, const int* __restrict__ gref_off,
                                                    const TiGeo<4, PA>* __restrict__ recs,
                                                    const int* __restrict__ qlist, const int* __restrict__ rel_box_c,
                                                    const int* __restrict__ parent_c, const int* __restrict__ slot_p,
                                                    int ncone_p, const cpx<float>* __restrict__ Fhat_p,
                                                    cpx<float>* __restrict__ G_c) {
  constexpr int PS = 4, NP = PA * PA, P = PS * NP, HM = PA / 2, NT = HM * HM;
  static_assert(PA % 2 == 0, "(b, c) in 2 x 2 blocks");
  const int4 tl = tiles[xcd_block(blockIdx.x, gridDim.x)];
  const int l = threadIdx.x;
  const int i = l & 15, k = l >> 4;
  const int bA = i >> 1, partA = i & 1;   // A row: box, re / im
  const bool validA = bA < tl.z;
  const int csA = validA ? slots[tl.y + bA] : 0;
  const int pbA = validA ? parent_c[rel_box_c[csA]] : 0;
  const int aB = i >> 2, bB = (i >> 1) & 1, cB = i & 1;   // B column: a, beta, gamma
  const uint64_t ma0 = __ballot(aB & 1), ma1 = __ballot(aB & 2), mb = __ballot(bB), mc = __ballot(cB);
  floatx4 acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = {0.0f, 0.0f, 0.0f, 0.0f};
  const int g0 = gref_off[tl.x], g1 = gref_off[tl.x + 1];
  for (int gi = g0; gi < g1; ++gi) {   // wave-uniform
    const int2 ref = gref[gi];
    const TiGeo<4, PA>& G = recs[ref.x];
    const int q = qlist[ref.x >> 3];
    const int psl = validA ? slot_p[(int64_t)pbA * ncone_p + q] : -1;
    if (!__ballot(psl >= 0)) continue;   // no box of the wave has this parent cone
    const cpx<float>* F = Fhat_p + (int64_t)(psl >= 0 ? psl : 0) * P;
    const int e0 = G.gstart[ref.y], e1 = G.gstart[ref.y + 1];
    // a step's records (coordinates, ratio, node) and parent node value; the
    // next step's node value and the records of the step after it are in
    // flight while a step runs
    auto rec_load = [&](int e, float4& lc, float2& rt, int& nd, bool& ok) {
      const int ek = e + k;
      ok = ek < e1;
      const int ee = ok ? ek : e0;
      lc = G.loc[ee];
      rt = G.rat[ee];
      nd = G.node[ee];
    };
    float4 lc0, lc1;
    float2 rt0, rt1;
    int nd0, nd1;
    bool ok0, ok1;
    rec_load(e0, lc0, rt0, nd0, ok0);
    cpx<float> f0 = {0.0f, 0.0f};
    if (ok0 && psl >= 0) f0 = F[nd0];
    rec_load(e0 + 4, lc1, rt1, nd1, ok1);
    for (int e = e0; e < e1; e += 4) {   // wave-uniform
      cpx<float> f1 = {0.0f, 0.0f};
      if (ok1 && psl >= 0) f1 = F[nd1];
      float4 lc2;
      float2 rt2;
      int nd2;
      bool ok2;
      rec_load(e + 8, lc2, rt2, nd2, ok2);
      const float4 loc = lc0;
      const float2 rt = rt0;
      const cpx<float> f = f0;
      lc0 = lc1;
      rt0 = rt1;
      f0 = f1;
      lc1 = lc2;
      rt1 = rt2;
      nd1 = nd2;
      ok1 = ok2;
      const float av = partA ? rt.x * f.im + rt.y * f.re : rt.x * f.re - rt.y * f.im;
      float Ts[PS], Tt[PA], Tp[PA];
      cheb_T<float, PS>(loc.x, Ts);
      cheb_T<float, PA>(loc.y, Tt);
      cheb_T<float, PA>(loc.z, Tp);
      const float ta = lane_sel(ma1, lane_sel(ma0, Ts[0], Ts[1]), lane_sel(ma0, Ts[2], Ts[3]));
      float tb[HM], tc[HM];
#pragma unroll
      for (int h = 0; h < HM; ++h) {
        tb[h] = ta * lane_sel(mb, Tt[2 * h], Tt[2 * h + 1]);
        tc[h] = lane_sel(mc, Tp[2 * h], Tp[2 * h + 1]);
      }
#pragma unroll
      for (int hb = 0; hb < HM; ++hb) {
#pragma unroll
        for (int hc = 0; hc < HM; ++hc) {
          const int t = hb * HM + hc;
          acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, tb[hb] * tc[hc], acc[t], 0, 0, 0);
        }
      }
    }
  }
  // lane 16 qd + jd holds rows 4 qd .. 4 qd + 3 = boxes 2 qd (re, im), 2 qd + 1 (re, im) of column jd
  const int qd = l >> 4, jd = l & 15;
  const int aD = jd >> 2, bD = (jd >> 1) & 1, cD = jd & 1;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int bx = 2 * qd + h;
    if (bx >= tl.z) continue;
    cpx<float>* out = G_c + (int64_t)slots[tl.y + bx] * P + aD * NP + bD * PA + cD;
#pragma unroll
    for (int hb = 0; hb < HM; ++hb) {
#pragma unroll
      for (int hc = 0; hc < HM; ++hc) {
        const int t = hb * HM + hc;
        cpx<float> v = out[2 * hb * PA + 2 * hc];
        v.re += acc[t][2 * h];
        v.im += acc[t][2 * h + 1];
        out[2 * hb * PA + 2 * hc] = v;
      }
    }
  }
}

// Groups per node record.
template <typename Rec>
__global__ __launch_bounds__(TPB) void k_rec_ngroup(const Rec* __restrict__ recs, int64_t nrec, int* __restrict__ out) {
  const int64_t r = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (r < nrec) out[r] = recs[r].ngroup;
}

// One key per (record r = 8 qi + o, group g): bucket (o, child cone id) high,
// (qi, g) low, so that a bucket's groups sort by parent cone, then group.
template <typename Rec>
__global__ __launch_bounds__(TPB) void k_rec_keys(const Rec* __restrict__ recs, int64_t nrec,
                                                  const int64_t* __restrict__ off, int ncone_c,
                                                  uint64_t* __restrict__ keys) {
  const int64_t r = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (r >= nrec) return;
  const int o = (int)(r & 7);
  const uint32_t qi = (uint32_t)(r >> 3);
  const int ng = recs[r].ngroup;
  for (int g = 0; g < ng; ++g) {
    const uint64_t bucket = (uint64_t)o * (uint64_t)ncone_c + (uint64_t)recs[r].gcid[g];
    keys[off[r] + g] = (bucket << 32) | (uint64_t)((qi << 8) | (uint32_t)g);
  }
}

// One key per relevant cone of the child level: bucket (octant of its box, cone id) high, slot low.
__global__ __launch_bounds__(TPB) void k_adj_child_keys(const int* __restrict__ rel_box, const int* __restrict__ rel_cone,
                                                        const int* __restrict__ coords, int64_t nrel, int ncone,
                                                        uint64_t* __restrict__ keys) {
  const int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (i >= nrel) return;
  const int b = rel_box[i];
  const int o = (coords[3 * b] & 1) | ((coords[3 * b + 1] & 1) << 1) | ((coords[3 * b + 2] & 1) << 2);
  const uint64_t bucket = (uint64_t)o * (uint64_t)ncone + (uint64_t)rel_cone[i];
  keys[i] = (bucket << 32) | (uint64_t)(uint32_t)i;
}

// L^T: each source y of a finest-level box gets sum over the box's relevant
// cones and their nodes of W_c(node, y) Fhat(node), added to acc.  The
// sources are taken SC at a time; each thread sums its share of the nodes in
// registers, then the block reduces per source.
constexpr int ADJ_LEAF_SC = 8;

template <typename T, int PS, int PA>
__global__ __launch_bounds__(TPB) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 4 : 1))) void k_adj_leaf(const double* __restrict__ pts, const double* __restrict__ nrm,
                                                  const int* __restrict__ start, const double* __restrict__ centre,
                                                  const int* __restrict__ slot_off, const int* __restrict__ rel_cone,
                                                  const cpx<T>* __restrict__ Fhat, LevelGeom g, ChebTab ct, double k,
                                                  double eta, int kind, int R, cpx<T>* __restrict__ acc_out) {
  constexpr int P = PS * PA * PA;
  constexpr int SC = ADJ_LEAF_SC;
  __shared__ T su[SC][3], sn[SC][3], suu[SC], sun[SC];
  __shared__ cpx<T> red[TPB / 64][SC];
  const int b = blockIdx.x, r = blockIdx.y;
  const int s0 = slot_off[b], ncn = slot_off[b + 1] - s0;
  const int p0 = start[b], np = start[b + 1] - p0;
  const double c0 = centre[3 * b], c1 = centre[3 * b + 1], c2 = centre[3 * b + 2];
  const double invh = 1.0 / g.h;
  const T kk = (T)k, ee = (T)eta, kh = (T)(k * g.h), ih = (T)invh;
  const int nitems = ncn * P;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int sb = 0; sb < np; sb += SC) {
    const int sc = min(SC, np - sb);
    __syncthreads();
    if (threadIdx.x < sc) {
      const int j = p0 + sb + threadIdx.x;
      T u0 = (T)((pts[3 * j] - c0) * invh), u1 = (T)((pts[3 * j + 1] - c1) * invh),
        u2 = (T)((pts[3 * j + 2] - c2) * invh);
      T n0 = (T)nrm[3 * j], n1 = (T)nrm[3 * j + 1], n2 = (T)nrm[3 * j + 2];
      su[threadIdx.x][0] = u0;
      su[threadIdx.x][1] = u1;
      su[threadIdx.x][2] = u2;
      sn[threadIdx.x][0] = n0;
      sn[threadIdx.x][1] = n1;
      sn[threadIdx.x][2] = n2;
      suu[threadIdx.x] = u0 * u0 + u1 * u1 + u2 * u2;
      sun[threadIdx.x] = u0 * n0 + u1 * n1 + u2 * n2;
    }
    __syncthreads();
    cpx<T> acc[SC];
#pragma unroll
    for (int q = 0; q < SC; ++q) acc[q] = {0, 0};
    for (int it = threadIdx.x; it < nitems; it += TPB) {
      const int cs = it / P, node = it % P;
      const int ai = node / (PA * PA), bi = (node / PA) % PA, ci = node % PA;
      const int cid = rel_cone[s0 + cs];
      T e[3], s;
      if constexpr (Prec<T>::f32) node_dir32(cid, ai, bi, ci, g, ct, e, &s);
      else node_dir64(cid, ai, bi, ci, g, ct, e, &s);
      const cpx<T> fh = Fhat[((int64_t)(s0 + cs) * P + node) * R + r];
#pragma unroll
      for (int q = 0; q < SC; ++q) {
        if (q >= sc) break;
        cpx<T> W;
        if (kind == IFGF_KERNEL_CONSTANT) {
          W = {1, 0};
        } else {
          T eu = e[0] * su[q][0] + e[1] * su[q][1] + e[2] * su[q][2];
          T en = e[0] * sn[q][0] + e[1] * sn[q][1] + e[2] * sn[q][2];
          T qq = s * suu[q] - (T)2 * eu;
          T nv, inv;
          sqrt_rsqrt<T>((T)1 + s * qq, &nv, &inv);
          T ph = kh * qq * rcp_t<T>(nv + (T)1);
          T sp, cp;
          // |ph| <= k h, as in the forward leaf factors
          if constexpr (Prec<T>::f32) sincos_hw(ph, &sp, &cp);
          else sincos_phase<T>(ph, &sp, &cp);
          T vn = en - s * sun[q];
          T A = vn * s * inv * inv * inv * ih;
          T Bv = kk * vn * inv * inv + ee * inv;
          W = {cp * A + sp * Bv, sp * A - cp * Bv};
        }
        acc[q].re += W.re * fh.re - W.im * fh.im;
        acc[q].im += W.re * fh.im + W.im * fh.re;
      }
    }
#pragma unroll
    for (int q = 0; q < SC; ++q) {
      T re = acc[q].re, im = acc[q].im;
      for (int off = 32; off > 0; off >>= 1) {
        re += __shfl_xor(re, off, 64);
        im += __shfl_xor(im, off, 64);
      }
      if (lane == 0) red[wid][q] = {re, im};
    }
    __syncthreads();
    if (threadIdx.x < sc) {
      cpx<T> t = {0, 0};
      for (int w = 0; w < TPB / 64; ++w) {
        t.re += red[w][threadIdx.x].re;
        t.im += red[w][threadIdx.x].im;
      }
      const int64_t o = (int64_t)(p0 + sb + threadIdx.x) * R + r;
      acc_out[o].re += t.re;
      acc_out[o].im += t.im;
    }
  }
}

// out[perm_j] = conj?(w_j g_j) in the caller's dtype.
template <typename T>
__global__ __launch_bounds__(TPB) void k_adj_out(const cpx<T>* __restrict__ g, const int* __restrict__ perm,
                                                 const double* __restrict__ w, int64_t n, int R, int dtype, int conj_out,
                                                 void* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (i >= n) return;
  const double wi = w[i];
  for (int r = 0; r < R; ++r) {
    const cpx<T> v = g[i * R + r];
    double re = wi * (double)v.re, im = wi * (double)v.im;
    if (conj_out) im = -im;
    const int64_t o = (int64_t)perm[i] * R + r;
    if (dtype == IFGF_C128) {
      ((double*)out)[2 * o] = re;
      ((double*)out)[2 * o + 1] = im;
    } else {
      ((float*)out)[2 * o] = (float)re;
      ((float*)out)[2 * o + 1] = (float)im;
    }
  }
}

// ---------------------------------------------------------------------------
// Far-field pattern (Sec. 5, eq. FarField).  For x = R xh with R -> inf,
// |x - y_B| = R - xh.y_B + O(1/R) and s = h / |x - y_B| -> 0: the field of
// level-3 box B tends to exp(ikR)/(4 pi R) exp(-ik xh.y_B) F_B(0, xh), so
//     u_inf(xh) = 1/(4 pi) sum_B exp(-ik xh.y_B) F_B(0, theta(xh), phi(xh)),
// F_B's interpolant taken at the left end (t_s = -1) of the first radial
// interval of the cone holding xh's angles.  One wave per direction, one
// lane per level-3 box (at most 4^3 = 64); the phase and the sum over boxes
// in FP64.
// ---------------------------------------------------------------------------
template <typename T, int PS, int PA>
__global__ __launch_bounds__(TPB) void k_far_field(const double* __restrict__ dirs, int64_t ndir, int nb,
                                                   const double* __restrict__ centre, const int* __restrict__ slot,
                                                   const cpx<T>* __restrict__ Fc, LevelGeom g, double k, int dtype,
                                                   void* __restrict__ out, int* __restrict__ err) {
  constexpr int P = PS * PA * PA;
  const int64_t dr = ((int64_t)blockIdx.x * TPB + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (dr >= ndir) return;   // wave-uniform
  const double xh0 = dirs[3 * dr], xh1 = dirs[3 * dr + 1], xh2 = dirs[3 * dr + 2];
  const Loc loc = locate64(xh0, xh1, xh2, 0.0, g);
  double re = 0.0, im = 0.0;
  if (lane < nb) {
    const int sl = slot[(int64_t)lane * g.ncone + loc.cid];
    if (sl < 0) {
      atomicOr(err, 8);
    } else {
      T Ts[PS], Tt[PA], Tp[PA];
      cheb_T<T, PS>((T)loc.ts, Ts);
      cheb_T<T, PA>((T)loc.tt, Tt);
      cheb_T<T, PA>((T)loc.tp, Tp);
      const cpx<T>* C = Fc + (int64_t)sl * P;
      double vr = 0.0, vi = 0.0;
      for (int a = 0; a < PS; ++a) {
        T hr = 0, hi = 0;
        for (int b = 0; b < PA; ++b) {
          T gr = 0, gi = 0;
          for (int c = 0; c < PA; ++c) {
            const cpx<T> x = C[(a * PA + b) * PA + c];
            gr += x.re * Tp[c];
            gi += x.im * Tp[c];
          }
          hr += gr * Tt[b];
          hi += gi * Tt[b];
        }
        vr += (double)(hr * Ts[a]);
        vi += (double)(hi * Ts[a]);
      }
      const double* y = centre + 3 * lane;
      double sp, cp;
      sincos(-k * (xh0 * y[0] + xh1 * y[1] + xh2 * y[2]), &sp, &cp);
      re = cp * vr - sp * vi;
      im = cp * vi + sp * vr;
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    re += __shfl_xor(re, off, 64);
    im += __shfl_xor(im, off, 64);
  }
  if (lane == 0) {
    const double q = 1.0 / (4.0 * IFGF_PI);
    if (dtype == IFGF_C128) {
      ((double*)out)[2 * dr] = q * re;
      ((double*)out)[2 * dr + 1] = q * im;
    } else {
      ((float*)out)[2 * dr] = (float)(q * re);
      ((float*)out)[2 * dr + 1] = (float)(q * im);
    }
  }
}

// The far-field sum of eq. FarField taken directly over the (sorted) points,
// for trees without interpolation levels (D <= 2): one wave per direction.
template <typename T>
__global__ __launch_bounds__(TPB) void k_far_direct(const double* __restrict__ dirs, int64_t ndir,
                                                    const double* __restrict__ pts, const double* __restrict__ nrm,
                                                    const cpx<T>* __restrict__ a, int64_t n, double k, double eta,
                                                    int dtype, void* __restrict__ out) {
  const int64_t dr = ((int64_t)blockIdx.x * TPB + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (dr >= ndir) return;   // wave-uniform
  const double xh0 = dirs[3 * dr], xh1 = dirs[3 * dr + 1], xh2 = dirs[3 * dr + 2];
  double re = 0.0, im = 0.0;
  for (int64_t j = lane; j < n; j += 64) {
    double sp, cp;
    sincos(-k * (xh0 * pts[3 * j] + xh1 * pts[3 * j + 1] + xh2 * pts[3 * j + 2]), &sp, &cp);
    const double xn = xh0 * nrm[3 * j] + xh1 * nrm[3 * j + 1] + xh2 * nrm[3 * j + 2];
    // e^{-ik xh.y} (-i k xh.n - i eta) a_j
    const double fr = cp, fi = sp, g = -(k * xn + eta);   // factor = (fr + i fi) * (i g)
    const double tr = -fi * g, ti = fr * g;
    const double ar = (double)a[j].re, ai = (double)a[j].im;
    re += tr * ar - ti * ai;
    im += tr * ai + ti * ar;
  }
  for (int off = 32; off > 0; off >>= 1) {
    re += __shfl_xor(re, off, 64);
    im += __shfl_xor(im, off, 64);
  }
  if (lane == 0) {
    const double q = 1.0 / (4.0 * IFGF_PI);
    if (dtype == IFGF_C128) {
      ((double*)out)[2 * dr] = q * re;
      ((double*)out)[2 * dr + 1] = q * im;
    } else {
      ((float*)out)[2 * dr] = (float)(q * re);
      ((float*)out)[2 * dr + 1] = (float)(q * im);
    }
  }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
// Orders with cone-major upward-pass tiles (P <= 144: the tile keeps a
// child's P_ang^2 coefficients per radial index in registers).
constexpr bool cone_major_order(int ps, int pa) { return ps <= 4 && ps * pa * pa <= 144; }

// The upward pass from child level d into level d - 1 (Algorithm 1, parent
// interpolation nodes), with the formulation the plan holds for that level:
// MFMA over RHS groups (FP32, nrhs a multiple of 16), cone-major tiles (one
// RHS, levels with tiles) or the node formulation.
template <typename T, int PS, int PA>
void prop_level(ifgf_plan_s* p, int d, int R, hipStream_t s) {
  constexpr int P = PS * PA * PA;
  const int kind = p->opt.kernel;
  const T* Ms = (const T*)(Prec<T>::f32 ? p->Msf.p : p->Ms.p);
  const T* Ma = (const T*)(Prec<T>::f32 ? p->Maf.p : p->Ma.p);
  const bool mfma = Prec<T>::f32 && R % MF_RG == 0 && PS <= 4;

  LevelPlan& lc = p->lev[d];
  LevelPlan& lp = p->lev[d - 1];
  if (lp.nrel == 0 || lp.nwork == 0) return;
  if constexpr (Prec<T>::f32 && PS <= 4) {
    if (mfma) {
      const int64_t items = (int64_t)lp.nrel * P;
      {
        StageTimer tm(p, s, IFGF_STAGE_PROP);
        (void)items;
        k_prop_mfma_cone<PS, PA><<<dim3((unsigned)lp.nrel, R / MF_RG), TPB, 0, s>>>(
            lp.rel_box.as<int>(), lp.rel_cone.as<int>(), lp.child_lo.as<int>(), lc.coords.as<int>(),
            lc.slot.as<int>(), lc.Fc.as<cpx<T>>(), lp.geom, lc.geom, p->cheb, (const float*)Ms,
            (const float*)Ma, p->k, kind, R,
            lp.ti_geo_built && lp.ti_rec.p ? lp.ti_geo.as<TiGeo<PS, PA>>() : nullptr,
            lp.ti_geo_built && lp.ti_rec.p ? lp.ti_rec.as<int>() : nullptr, lp.Fc.as<cpx<T>>(), p->err.as<int>());
      }
      HIPCHK(hipGetLastError());
      return;
    }
  }
  if constexpr (rows_ok<T, PS, PA>()) {
    if (R == 1 && lp.up_use && lp.nup > 0) {   // from the level's pair list
      StageTimer tm(p, s, IFGF_STAGE_PROP);
      const PLevel<T> ul{lp.nup, lp.up_slot.as<int>(), lp.up_loc.as<typename Vec4<T>::type>(), lp.up_fim.as<T>(),
                         lp.up_val.as<cpx<T>>(), nullptr, lp.up_pos.as<int>(), lc.Fc.as<cpx<T>>()};
      k_upairs<T, PS, PA><<<(unsigned)((lp.nup + TPB - 1) / TPB), TPB, 0, s>>>(ul);
      HIPCHK(hipGetLastError());
      k_upsum_coeffs<T, PS, PA><<<(unsigned)((lp.nrel + coeff_cones(P) - 1) / coeff_cones(P)), TPB, 0, s>>>(
          lp.up_base.as<int>(), lp.up_pos.as<int>(), lp.up_val.as<cpx<T>>(), lp.nrel, Ms, Ma, lp.Fc.as<cpx<T>>());
      HIPCHK(hipGetLastError());
      return;
    }
  }
  if constexpr (Prec<T>::f32 && cone_major_order(PS, PA)) {
    if (R == 1 && lp.ntile > 0) {
      StageTimer tm(p, s, IFGF_STAGE_PROP_CONE);
      auto launch = [&](auto kern, int nw) {
        kern<<<(unsigned)lp.ntile, 64 * nw, 0, s>>>(
            lp.ti_tile.as<int4>(), lp.ti_slot.as<int>(), lp.ti_child.as<int>(), lp.ti_geo.as<TiGeo<PS, PA>>(),
            lc.slot.as<int>(), lc.Fc.as<cpx<float>>(), lp.geom, lc.geom, p->cheb, (const float*)Ms,
            (const float*)Ma, p->k, kind, lp.Fc.as<cpx<float>>(), p->err.as<int>());
      };
      if (lp.ti_nw == 4) launch(k_prop_ti<PS, PA, 4>, 4);
      else if (lp.ti_nw == 2) launch(k_prop_ti<PS, PA, 2>, 2);
      else launch(k_prop_ti<PS, PA, 1>, 1);
      HIPCHK(hipGetLastError());
      return;
    }
  }
  if constexpr (!Prec<T>::f32 && cone_major_order(PS, PA)) {
    if (R == 1 && lp.ntile > 0) {
      StageTimer tm(p, s, IFGF_STAGE_PROP_CONE);
      auto launch = [&](auto kern, int nw) {
        kern<<<(unsigned)lp.ntile, 64 * nw, 0, s>>>(
            lp.ti_tile.as<int4>(), lp.ti_slot.as<int>(), lp.ti_child.as<int>(), lp.ti_geo.as<TiGeo64<PS, PA>>(),
            lc.slot.as<int>(), lc.Fc.as<cpx<double>>(), lp.geom, lc.geom, p->cheb, (const double*)Ms,
            (const double*)Ma, p->k, kind, lp.Fc.as<cpx<double>>(), p->err.as<int>());
      };
      if (lp.ti_nw == 2) launch(k_prop_ti64<PS, PA, 2>, 2);
      else launch(k_prop_ti64<PS, PA, 1>, 1);
      HIPCHK(hipGetLastError());
      return;
    }
  }
  StageTimer tm(p, s, IFGF_STAGE_PROP);
  auto kp = R == 1 ? k_prop<T, PS, PA, true> : k_prop<T, PS, PA, false>;
  kp<<<dim3((unsigned)lp.nwork, R), PropShape<P>::BS, 0, s>>>(
      lp.work.as<int4>(), lp.rel_cone.as<int>(), lp.child_lo.as<int>(), lc.coords.as<int>(), lc.slot.as<int>(),
      lc.Fc.as<cpx<T>>(), lp.geom, lc.geom, p->cheb, Ms, Ma, p->k, kind, R, lp.Fc.as<cpx<T>>(), p->err.as<int>());
  HIPCHK(hipGetLastError());
}

template <typename T, int PS, int PA>
void apply_impl(ifgf_plan_s* p, const void* sigma, void* u, int R, int dtype, int stage_mask, int level_lo,
                int level_hi, hipStream_t s) {
  constexpr int P = PS * PA * PA;
  const int64_t n = p->n;
  const int D = p->D;
  cpx<T>* a = p->a.as<cpx<T>>();
  cpx<T>* uacc = p->uacc.as<cpx<T>>();
  dim3 gpts(nblocks(n), R);
  {
    StageTimer tm(p, s, IFGF_STAGE_GATHER);
    k_gather<T><<<nblocks(n * R), TPB, 0, s>>>(sigma, dtype, 0, p->perm.as<int>(), p->w.as<double>(), n, R, a,
                                               p->n_src);
  }
  HIPCHK(hipGetLastError());
  const int kind = p->opt.kernel;
  LevelPlan& lD = p->lev[D];
  const bool near = stage_mask & 1;
  // right-hand sides in groups of 16 per launch column (the group kernels hold
  // P x 16 values per block in LDS: orders up to P = 144)
  constexpr bool kGroups = P <= 144;
  const bool grouped = kGroups && R % MF_RG == 0;
  if (near) {
    StageTimer tm(p, s, IFGF_STAGE_NEAR);
    if (grouped)
      k_near<T, false, MF_RG><<<dim3(lD.n_near, R / MF_RG), TPB, 0, s>>>(
          lD.near_work.as<int4>(), p->pts.as<double>(), p->nrm.as<double>(), a, R, lD.start.as<int>(),
          lD.nbr_off.as<int>(), lD.nbr.as<int>(), lD.centre.as<double>(), p->k, p->eta, kind, uacc);
    else
      k_near<T, false, 1><<<dim3(lD.n_near, R), TPB, 0, s>>>(lD.near_work.as<int4>(), p->pts.as<double>(),
                                                             p->nrm.as<double>(), a, R, lD.start.as<int>(),
                                                             lD.nbr_off.as<int>(), lD.nbr.as<int>(),
                                                             lD.centre.as<double>(), p->k, p->eta, kind, uacc);
    HIPCHK(hipGetLastError());
  }
  if (D >= 3) {
    const T* Ms = (const T*)(Prec<T>::f32 ? p->Msf.p : p->Ms.p);
    const T* Ma = (const T*)(Prec<T>::f32 ? p->Maf.p : p->Ma.p);
    if (lD.n_leaf > 0) {
      StageTimer tm(p, s, IFGF_STAGE_LEAF);
      if (grouped) {
        if constexpr (kGroups)
          k_leaf<T, PS, PA, MF_RG, false><<<dim3(lD.n_leaf, R / MF_RG), TPB, 0, s>>>(
              lD.leaf_work.as<int4>(), p->pts.as<double>(), p->nrm.as<double>(), a, R, lD.start.as<int>(),
              lD.centre.as<double>(), lD.slot_off.as<int>(), lD.rel_cone.as<int>(), lD.geom, p->cheb, p->k, p->eta,
              kind, lD.Fn.as<cpx<T>>(), Ms, Ma, lD.Fc.as<cpx<T>>());
      } else if (R == 1)
        k_leaf<T, PS, PA, 1, true><<<dim3(lD.n_leaf, 1), TPB, 0, s>>>(
            lD.leaf_work.as<int4>(), p->pts.as<double>(), p->nrm.as<double>(), a, R, lD.start.as<int>(),
            lD.centre.as<double>(), lD.slot_off.as<int>(), lD.rel_cone.as<int>(), lD.geom, p->cheb, p->k, p->eta,
            kind, lD.Fn.as<cpx<T>>(), Ms, Ma, lD.Fc.as<cpx<T>>());
      else
        k_leaf<T, PS, PA, 1, false><<<dim3(lD.n_leaf, R), TPB, 0, s>>>(
            lD.leaf_work.as<int4>(), p->pts.as<double>(), p->nrm.as<double>(), a, R, lD.start.as<int>(),
            lD.centre.as<double>(), lD.slot_off.as<int>(), lD.rel_cone.as<int>(), lD.geom, p->cheb, p->k, p->eta,
            kind, lD.Fn.as<cpx<T>>(), Ms, Ma, lD.Fc.as<cpx<T>>());
    }
    HIPCHK(hipGetLastError());
    if (lD.nrel > 0 && (grouped || R > 1)) {   // one RHS: done inside k_leaf
      StageTimer tm(p, s, IFGF_STAGE_COEFFS);
      if (grouped) {
        if constexpr (kGroups)
          k_coeffs_rg<T, PS, PA, MF_RG><<<dim3(lD.nrel, R / MF_RG), TPB, 0, s>>>(lD.Fn.as<cpx<T>>(), R, Ms, Ma,
                                                                                lD.Fc.as<cpx<T>>());
      } else
        k_coeffs<T, PS, PA, false><<<dim3((lD.nrel + coeff_cones(P) - 1) / coeff_cones(P), R), TPB, 0, s>>>(lD.Fn.as<cpx<T>>(), lD.nrel, R, Ms, Ma,
                                                                   lD.Fc.as<cpx<T>>());
      HIPCHK(hipGetLastError());
    }
    for (int d = D; d >= 4; --d) prop_level<T, PS, PA>(p, d, R, s);
  }
  TLevels<T> L{};
  for (int d = 3; d <= D; ++d) {
    LevelPlan& lv = p->lev[d];
    L.lv[d] = {gas(lv.pbox.as<const int>()), gas(lv.cou_off.as<const int>()), gas(lv.cou.as<const int>()),
               gas(lv.centre.as<const double>()), gas(lv.slot.as<const int>()), gas(lv.Fc.as<const cpx<T>>()),
               lv.geom};
  }
  int dlo = 3, dhi = D;
  if (!(stage_mask & 2)) {
    dlo = 1;
    dhi = 0;
  } else {
    dlo = std::max(dlo, level_lo);
    dhi = std::min(dhi, level_hi);
  }
  if constexpr (Prec<T>::f32 && PS <= 4) {
    if (R % MF_RG == 0 && p->pairs && p->pairs_rg &&
        (p->opt.target_kernel == IFGF_TARGET_AUTO || p->opt.target_kernel == IFGF_TARGET_PAIRS)) {
      StageTimer tm(p, s, IFGF_STAGE_TARGETS);
      PLevels<float> PL{};
      int64_t maxp = 0;
      for (int d = 3; d <= D; ++d) {
        LevelPlan& lv = p->lev[d];
        PL.lv[d] = {lv.npair, lv.pr_slot.as<int>(), lv.pr_loc.as<float4>(), lv.pr_fim.as<float>(),
                    lv.pr_val.as<cpx<float>>(), lv.pr_off.as<int>(), lv.pr_pos.as<int>(), lv.Fc.as<cpx<float>>()};
        if (d >= dlo && d <= dhi) maxp = std::max(maxp, lv.npair);
      }
      const int nlev = dlo <= dhi ? dhi - dlo + 1 : 0;
      for (int g = 0; g < R / MF_RG; ++g) {   // the value buffer holds one group at a time
        if (nlev > 0 && maxp > 0) {
          k_targets_pairs_rg<PS, PA><<<dim3(nblocks(maxp), nlev), TPB, 0, s>>>(PL, dlo, R, g);
          HIPCHK(hipGetLastError());
        }
        k_targets_pairsum_rg<<<nblocks(n * MF_RG), TPB, 0, s>>>(n, p->perm.as<int>(), (const cpx<float>*)uacc, near ? 1 : 0,
                                                       PL, dlo, dhi, R, g, dtype, u);
        HIPCHK(hipGetLastError());
      }
      return;
    }
    if (R % MF_RG == 0) {
      StageTimer tm(p, s, IFGF_STAGE_TARGETS);
      k_targets_mfma<PS, PA><<<dim3(nblocks(n), R / MF_RG), TPB, 0, s>>>(p->pts.as<double>(), n, p->perm.as<int>(),
                                                                        uacc, near ? 1 : 0, L, dlo, dhi, p->k, kind, R,
                                                                        dtype, u, p->err.as<int>());
      HIPCHK(hipGetLastError());
      return;
    }
  }
  if constexpr (rows_ok<T, PS, PA>()) {   // orders with a generated row stage
    if (R == 1 && p->pairs && (p->opt.target_kernel == IFGF_TARGET_AUTO || p->opt.target_kernel == IFGF_TARGET_PAIRS)) {
      StageTimer tm(p, s, IFGF_STAGE_TARGETS);
      PLevels<T> PL{};
      int64_t maxp = 0;
      for (int d = 3; d <= D; ++d) {
        LevelPlan& lv = p->lev[d];
        PL.lv[d] = {lv.npair, lv.pr_slot.as<int>(), lv.pr_loc.as<typename Vec4<T>::type>(), lv.pr_fim.as<T>(),
                    lv.pr_val.as<cpx<T>>(), lv.pr_off.as<int>(), lv.pr_pos.as<int>(), lv.Fc.as<cpx<T>>()};
        if (d >= dlo && d <= dhi) maxp = std::max(maxp, lv.npair);
      }
      const int nlev = dlo <= dhi ? dhi - dlo + 1 : 0;
      if (nlev > 0 && maxp > 0) {
        k_targets_pairs<T, PS, PA><<<dim3(nblocks(maxp), nlev), TPB, 0, s>>>(PL, dlo);
        HIPCHK(hipGetLastError());
      }
      k_targets_pairsum<T><<<nblocks(16 * n), TPB, 0, s>>>(n, p->perm.as<int>(), uacc, near ? 1 : 0, PL, dlo, dhi, dtype,
                                                     u);
      HIPCHK(hipGetLastError());
      return;
    }
    if (R == 1 && p->opt.target_kernel != IFGF_TARGET_WAVE) {
      StageTimer tm(p, s, IFGF_STAGE_TARGETS);
      const int nlev = dlo <= dhi ? dhi - dlo + 1 : 0;
      if ((size_t)nlev * n * sizeof(cpx<T>) > p->tpart.bytes) throw Error{IFGF_EINTERNAL, "target level buffer"};
      cpx<T>* part = p->tpart.as<cpx<T>>();
      if (nlev > 0) {
        k_targets_rows<T, PS, PA><<<dim3(nblocks(n), nlev), TPB, 0, s>>>(p->pts.as<double>(), n, L, dlo, p->k,
                                                                         kind, part, p->err.as<int>());
        HIPCHK(hipGetLastError());
      }
      k_targets_sum<T><<<nblocks(n), TPB, 0, s>>>(n, p->perm.as<int>(), uacc, near ? 1 : 0, part, nlev, dtype, u);
      HIPCHK(hipGetLastError());
      return;
    }
  }
  {
    StageTimer tm(p, s, IFGF_STAGE_TARGETS);
    k_targets<T, PS, PA><<<gpts, TPB, 0, s>>>(p->pts.as<double>(), n, p->perm.as<int>(), uacc, near ? 1 : 0, L, dlo,
                                              dhi, p->k, kind, R, dtype, 0, nullptr, u, p->err.as<int>());
  }
  HIPCHK(hipGetLastError());
}

// The gather index of the transposed upward pass from level d (node records)
// into level d + 1: built once, at the first transposed apply.
// The MFMA form of the gather: FP32 with P_s = 4 (8 boxes per wave).
template <typename T, int PS, int PA>
constexpr bool adj_mfma() { return Prec<T>::f32 && PS == 4 && (PA * PA) % 4 == 0; }

template <typename T, int PS, int PA>
void build_adj_gather(ifgf_plan_s* p, int d, hipStream_t s) {
  using Rec = typename RecOf<T, PS, PA>::type;
  LevelPlan& lv = p->lev[d];
  LevelPlan& lc = p->lev[d + 1];
  const int nc = lc.geom.ncone;
  const int64_t nrec = 8 * lv.ti_nq;
  const Rec* recs = lv.ti_geo.as<Rec>();
  // (record, group) pairs by (octant, child cone id), then parent cone, then group
  DevBuf ngd;
  ngd.alloc(sizeof(int) * nrec);
  k_rec_ngroup<Rec><<<nblocks(nrec), TPB, 0, s>>>(recs, nrec, ngd.as<int>());
  HIPCHK(hipGetLastError());
  std::vector<int> ng(nrec);
  HIPCHK(hipMemcpyAsync(ng.data(), ngd.p, sizeof(int) * nrec, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  std::vector<int64_t> off(nrec + 1, 0);
  for (int64_t r = 0; r < nrec; ++r) off[r + 1] = off[r] + ng[r];
  const int64_t total = off[nrec];
  DevBuf offd, keys;
  offd.alloc(sizeof(int64_t) * (nrec + 1));
  keys.alloc(sizeof(uint64_t) * sort_padded_length(std::max<int64_t>(1, total)));
  HIPCHK(hipMemcpyAsync(offd.p, off.data(), sizeof(int64_t) * (nrec + 1), hipMemcpyHostToDevice, s));
  k_rec_keys<Rec><<<nblocks(nrec), TPB, 0, s>>>(recs, nrec, offd.as<int64_t>(), nc, keys.as<uint64_t>());
  HIPCHK(hipGetLastError());
  sort_u64(keys.as<uint64_t>(), total, s);
  std::vector<uint64_t> hk(total);
  HIPCHK(hipMemcpyAsync(hk.data(), keys.p, sizeof(uint64_t) * total, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  const int64_t nbucket = 8 * (int64_t)nc;
  std::vector<int> goff(nbucket + 1, 0);
  std::vector<int2> gref(std::max<int64_t>(1, total));
  for (int64_t i = 0; i < total; ++i) {
    const int64_t bucket = (int64_t)(hk[i] >> 32);
    const uint32_t lo = (uint32_t)hk[i];
    const int o = (int)(bucket / nc);
    gref[i] = make_int2((int)((lo >> 8) * 8 + o), (int)(lo & 255));
    ++goff[bucket + 1];
  }
  for (int64_t b = 0; b < nbucket; ++b) goff[b + 1] += goff[b];
  // the child level's relevant cones by (octant, cone id, slot), in tiles of <= 64
  DevBuf ck;
  ck.alloc(sizeof(uint64_t) * sort_padded_length(std::max<int64_t>(1, lc.nrel)));
  k_adj_child_keys<<<nblocks(lc.nrel), TPB, 0, s>>>(lc.rel_box.as<int>(), lc.rel_cone.as<int>(), lc.coords.as<int>(),
                                                   lc.nrel, nc, ck.as<uint64_t>());
  HIPCHK(hipGetLastError());
  sort_u64(ck.as<uint64_t>(), lc.nrel, s);
  std::vector<uint64_t> hc(lc.nrel);
  HIPCHK(hipMemcpyAsync(hc.data(), ck.p, sizeof(uint64_t) * lc.nrel, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  std::vector<int> slots(std::max<int64_t>(1, lc.nrel));
  std::vector<int4> tiles;
  for (int64_t i = 0; i < lc.nrel;) {
    const uint64_t bucket = hc[i] >> 32;
    int64_t j = i;
    while (j < lc.nrel && (hc[j] >> 32) == bucket) ++j;
    const int cap = adj_mfma<T, PS, PA>() ? 8 : 64;   // boxes per wave
    for (int64_t t = i; t < j; t += cap)
      tiles.push_back(make_int4((int)bucket, (int)t, (int)std::min<int64_t>(cap, j - t), 0));
    i = j;
  }
  for (int64_t i = 0; i < lc.nrel; ++i) slots[i] = (int)(uint32_t)hc[i];
  lv.adj_gref.alloc(sizeof(int2) * gref.size());
  lv.adj_gref_off.alloc(sizeof(int) * goff.size());
  lv.adj_slots.alloc(sizeof(int) * slots.size());
  lv.adj_tiles.alloc(sizeof(int4) * std::max<size_t>(1, tiles.size()));
  HIPCHK(hipMemcpy(lv.adj_gref.p, gref.data(), sizeof(int2) * gref.size(), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(lv.adj_gref_off.p, goff.data(), sizeof(int) * goff.size(), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(lv.adj_slots.p, slots.data(), sizeof(int) * slots.size(), hipMemcpyHostToDevice));
  if (!tiles.empty())
    HIPCHK(hipMemcpy(lv.adj_tiles.p, tiles.data(), sizeof(int4) * tiles.size(), hipMemcpyHostToDevice));
  lv.adj_ntile = (int64_t)tiles.size();
  lv.adj_built = true;
}

// ---------------------------------------------------------------------------
// Transposed cousin targets from the pair lists (gather form).  The pairs of
// a level are sorted by cone slot, so the pairs of one slot form a run; one
// wave takes a run and sums, in the run's order, every pair's target value
// times its centred factor times the basis at its local coordinates into
// the slot's P coefficient adjoints: one writer per coefficient, the same
// sums on every call.  Lane (b, c) (lanes < p_ang^2) holds the coefficients
// (a, b, c) for every a; the run is read in chunks of 64 pairs whose
// Chebyshev vectors and weights each lane first puts in LDS.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(TPB) void k_run_flag(const int* __restrict__ slot, int64_t np, int* __restrict__ flag) {
  const int64_t q = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (q < np) flag[q] = (q == 0 || slot[q] != slot[q - 1]) ? 1 : 0;
}

__global__ __launch_bounds__(TPB) void k_run_place(const int* __restrict__ flag, const int* __restrict__ idx,
                                                   int64_t np, int* __restrict__ run) {
  const int64_t q = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (q < np && flag[q]) run[idx[q]] = (int)q;
  if (q == 0) run[idx[np]] = (int)np;
}

// target of every sorted pair: pairs off[i] .. off[i+1]-1 of target i sit at pos[]
__global__ __launch_bounds__(TPB) void k_pair_tgt(int64_t n, const int* __restrict__ off, const int* __restrict__ pos,
                                                  int* __restrict__ tgt) {
  const int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (i >= n) return;
  for (int t = off[i]; t < off[i + 1]; ++t) tgt[pos[t]] = (int)i;
}

template <typename T, int PS, int PA, bool ACC>
__global__ __launch_bounds__(TPB) void k_adj_pairs(const int* __restrict__ run, int64_t nrun,
                                                   const typename Vec4<T>::type* __restrict__ loc,
                                                   const T* __restrict__ fim, const int* __restrict__ tgt,
                                                   const int* __restrict__ slot, const cpx<T>* __restrict__ vs, int R,
                                                   cpx<T>* __restrict__ G) {
  constexpr int P = PS * PA * PA;
  constexpr int NBC = PA * PA;
  static_assert(NBC <= 64, "one lane per (b, c)");
  constexpr int NF = PS + 2 * PA + 2;   // Ts, Tt, Tp, weight (re, im)
  __shared__ T buf[TPB / 64][64][NF + 1];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63, r = blockIdx.y;
  const int64_t ri = (int64_t)blockIdx.x * (TPB / 64) + wv;
  if (ri >= nrun) return;   // wave-uniform; the kernel has no block barrier
  const int q0 = run[ri], q1 = run[ri + 1];
  const int su = slot[q0];
  const int bl = lane / PA, cl = lane % PA;
  cpx<T> acc[PS];
#pragma unroll
  for (int a = 0; a < PS; ++a) acc[a] = {0, 0};
  T* f = buf[wv][lane];
  for (int qb = q0; qb < q1; qb += 64) {
    const int q = qb + lane;
    if (q < q1) {
      const typename Vec4<T>::type lc = loc[q];
      const T fi = fim[q];
      const cpx<T> v = vs[(int64_t)tgt[q] * R + r];
      cheb_T<T, PS>(lc.x, f);
      cheb_T<T, PA>(lc.y, f + PS);
      cheb_T<T, PA>(lc.z, f + PS + PA);
      f[NF - 2] = lc.w * v.re - fi * v.im;
      f[NF - 1] = lc.w * v.im + fi * v.re;
    }
    __builtin_amdgcn_wave_barrier();
    const int cnt = min(64, q1 - qb);
    if (lane < NBC) {
      for (int k = 0; k < cnt; ++k) {
        const T* fk = buf[wv][k];
        const T tbc = fk[PS + bl] * fk[PS + PA + cl];
        const T wre = fk[NF - 2], wim = fk[NF - 1];
#pragma unroll
        for (int a = 0; a < PS; ++a) {
          const T fa = fk[a] * tbc;
          acc[a].re += fa * wre;
          acc[a].im += fa * wim;
        }
      }
    }
    __builtin_amdgcn_wave_barrier();   // the chunk is read before the next one is written
  }
  if (lane < NBC) {
#pragma unroll
    for (int a = 0; a < PS; ++a) {
      cpx<T>& g = G[((int64_t)su * P + a * NBC + lane) * R + r];
      if constexpr (ACC) g = {g.re + acc[a].re, g.im + acc[a].im};
      else g = acc[a];
    }
  }
}

// Runs of equal slots of a sorted list of np pairs: run[] gets the starts,
// then np; returns the number of runs.
int64_t build_slot_runs(const int* slot, int64_t np, DevBuf& run, hipStream_t s) {
  DevBuf flag, idx;
  flag.alloc(sizeof(int) * (np + 1));
  idx.alloc(sizeof(int) * (np + 1));
  k_run_flag<<<nblocks(np), TPB, 0, s>>>(slot, np, flag.as<int>());
  HIPCHK(hipGetLastError());
  scan_exclusive_i32(flag.as<int>(), idx.as<int>(), np, s);
  int nr32 = 0;
  HIPCHK(hipMemcpyAsync(&nr32, idx.as<int>() + np, sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  run.alloc(sizeof(int) * ((int64_t)nr32 + 1));
  k_run_place<<<nblocks(np), TPB, 0, s>>>(flag.as<int>(), idx.as<int>(), np, run.as<int>());
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s));   // the temporaries are freed on return
  return nr32;
}

// The transposed-pass index of level d's upward pair list (on the first
// transposed apply): the parent node of every sorted pair, the slot runs.
void build_up_adj(ifgf_plan_s* p, int d, hipStream_t s) {
  LevelPlan& lv = p->lev[d];
  const int P = p->P;
  lv.up_node.alloc(sizeof(int) * lv.nup);
  const int64_t nn = (int64_t)lv.nrel * P;
  k_upair_node<<<nblocks(nn), TPB, 0, s>>>(lv.nrel, P, lv.up_base.as<int>(), lv.up_pos.as<int>(),
                                           lv.up_node.as<int>());
  HIPCHK(hipGetLastError());
  lv.up_nrun = build_slot_runs(lv.up_slot.as<int>(), lv.nup, lv.up_run, s);
}

// k_adj_pairs on MFMA (FP32, P_s P_ang <= 32, 2 P_ang <= 16).  For one slot
// run the coefficient adjoints are a matrix product over the run's pairs p:
// G[(a, b), (c, re/im)] = sum_p Ts_a(p) Tt_b(p) * Tp_c(p) w_(re/im)(p), with
// w the pair's factor times its target value.  A wave takes a run, stages 64
// pairs at a time in LDS (lane = pair: its Chebyshev values and w, as
// k_adj_pairs, so that as many waves stay resident) and accumulates 4 pairs
// per v_mfma_f32_16x16x4_f32 into MT row tiles, each lane forming its A
// entry Ts_a Tt_b and B entry Tp_c w from the staged values; one writer per
// coefficient and a fixed order, as k_adj_pairs.
template <int PS, int PA> constexpr bool adj_pairs_mfma_ok() { return PS * PA <= 32 && 2 * PA <= 16; }

template <int PS, int PA, bool ACC>
__global__ __launch_bounds__(TPB) void k_adj_pairs_mfma(const int* __restrict__ run, int64_t nrun,
                                                        const float4* __restrict__ loc, const float* __restrict__ fim,
                                                        const int* __restrict__ tgt, const int* __restrict__ slot,
                                                        const cpx<float>* __restrict__ vs, int R,
                                                        cpx<float>* __restrict__ G) {
  static_assert(adj_pairs_mfma_ok<PS, PA>(), "rows (a, b) in two tiles, columns (c, re/im) in one");
  constexpr int P = PS * PA * PA;
  constexpr int MR = PS * PA;               // A rows used
  constexpr int MT = (MR + 15) / 16;        // row tiles
  constexpr int NC = 2 * PA;                // B columns used
  constexpr int NW = TPB / 64;
  constexpr int NF = PS + 2 * PA + 2;       // Ts, Tt, Tp, w (re, im)
  __shared__ float buf[NW][64][NF + 1];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63, r = blockIdx.y;
  const int64_t ri = (int64_t)blockIdx.x * NW + wv;
  if (ri >= nrun) return;   // wave-uniform; the kernel has no block barrier
  const int q0 = run[ri], q1 = run[ri + 1];
  const int su = slot[q0];
  const int li = lane & 15, lk = lane >> 4;
  // this lane's A entries (row 16 m + li: Ts_a Tt_b) and B entry (column li: Tp_c w_re/im)
  int fa[MT], fb[MT];
  bool va[MT];
#pragma unroll
  for (int m = 0; m < MT; ++m) {
    const int i = 16 * m + li;
    va[m] = i < MR;
    fa[m] = va[m] ? i / PA : 0;
    fb[m] = va[m] ? PS + i % PA : 0;
  }
  const bool vb = li < NC;
  const int fc = vb ? PS + PA + (li >> 1) : 0, fw = vb ? PS + 2 * PA + (li & 1) : 0;
  floatx4 d[MT];
#pragma unroll
  for (int m = 0; m < MT; ++m) d[m] = {0.f, 0.f, 0.f, 0.f};
  for (int qb = q0; qb < q1; qb += 64) {
    {   // stage pair qb + lane; past the run's end: zero weight
      const int q = qb + lane;
      float* f = buf[wv][lane];
      float4 lc = make_float4(0.f, 0.f, 0.f, 0.f);
      float wre = 0.f, wim = 0.f;
      if (q < q1) {
        lc = loc[q];
        const float fi = fim[q];
        const cpx<float> v = vs[(int64_t)tgt[q] * R + r];
        wre = lc.w * v.re - fi * v.im;
        wim = lc.w * v.im + fi * v.re;
      }
      cheb_T<float, PS>(lc.x, f);
      cheb_T<float, PA>(lc.y, f + PS);
      cheb_T<float, PA>(lc.z, f + PS + PA);
      f[NF - 2] = wre;
      f[NF - 1] = wim;
    }
    __builtin_amdgcn_wave_barrier();
    const int cnt = min(64, q1 - qb);
    for (int k = 0; k < cnt; k += 4) {   // pairs past the run's end carry zero weight
      const float* fk = buf[wv][k + lk];
      const float bv = vb ? fk[fc] * fk[fw] : 0.f;
#pragma unroll
      for (int m = 0; m < MT; ++m)
        d[m] = __builtin_amdgcn_mfma_f32_16x16x4f32(va[m] ? fk[fa[m]] * fk[fb[m]] : 0.f, bv, d[m], 0, 0, 0);
    }
    __builtin_amdgcn_wave_barrier();   // the chunk is read before the next one is written
  }
  // lane 16 lk + j holds rows 4 lk .. 4 lk + 3 of column j of every row tile
  if (vb) {
    const int c = li >> 1, ri2 = li & 1;
    float* Gf = reinterpret_cast<float*>(G);
#pragma unroll
    for (int m = 0; m < MT; ++m) {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int i = 16 * m + 4 * lk + e;
        if (i >= MR) continue;
        const int a = i / PA, b = i % PA;
        float& g = Gf[2 * (((int64_t)su * P + (a * PA + b) * PA + c) * R + r) + ri2];
        g = ACC ? g + d[m][e] : d[m][e];
      }
    }
  }
}

// The transposed-apply index of the pair lists: per sorted pair its target,
// per level the runs of equal slots.
void build_adj_pairs(ifgf_plan_s* p, hipStream_t s) {
  const int64_t n = p->n;
  for (int d = 3; d <= p->D; ++d) {
    LevelPlan& lv = p->lev[d];
    const int64_t np = lv.npair;
    lv.nrun = 0;
    if (np == 0) continue;
    lv.pr_tgt.alloc(sizeof(int) * np);
    k_pair_tgt<<<nblocks(n), TPB, 0, s>>>(n, lv.pr_off.as<int>(), lv.pr_pos.as<int>(), lv.pr_tgt.as<int>());
    HIPCHK(hipGetLastError());
    lv.nrun = build_slot_runs(lv.pr_slot.as<int>(), np, lv.pr_run, s);
  }
  p->adj_pairs = true;
}

template <typename T, int PS, int PA>
void adjoint_impl(ifgf_plan_s* p, const void* v, void* out, int R, int dtype, int conj, hipStream_t s) {
  constexpr int P = PS * PA * PA;
  const int64_t n = p->n;
  const int D = p->D;
  const int kind = p->opt.kernel;
  cpx<T>* vs = p->a.as<cpx<T>>();
  cpx<T>* g = p->uacc.as<cpx<T>>();
  dim3 gpts(nblocks(n), R);
  {
    StageTimer tm(p, s, IFGF_STAGE_GATHER);
    k_gather<T><<<nblocks(n * R), TPB, 0, s>>>(v, dtype, conj, p->perm.as<int>(), nullptr, n, R, vs, n);
  }
  HIPCHK(hipGetLastError());
  LevelPlan& lD = p->lev[D];
  {
    StageTimer tm(p, s, IFGF_STAGE_ADJ_NEAR);
    k_near<T, true, 1><<<dim3(lD.n_near, R), TPB, 0, s>>>(lD.near_work.as<int4>(), p->pts.as<double>(),
                                                        p->nrm.as<double>(), vs, R, lD.start.as<int>(),
                                                        lD.nbr_off.as<int>(), lD.nbr.as<int>(),
                                                        lD.centre.as<double>(), p->k, p->eta, kind, g);
  }
  HIPCHK(hipGetLastError());
  if (D >= 3) {
    const size_t csz = sizeof(cpx<T>);
    ALevels<T> L{};
    for (int d = 3; d <= D; ++d) {
      LevelPlan& lv = p->lev[d];
      size_t need = csz * (size_t)std::max(1, lv.nrel) * P * p->opt.max_rhs;
      if (p->adj_g[d].bytes < need) p->adj_g[d].alloc(need);
      const int64_t cnt = (int64_t)lv.nrel * R * P;
      if (cnt > 0) {
        k_fill_zero<T><<<nblocks(cnt), TPB, 0, s>>>(p->adj_g[d].as<cpx<T>>(), cnt);
        HIPCHK(hipGetLastError());
      }
      L.lv[d] = {lv.pbox.as<int>(), lv.cou_off.as<int>(), lv.cou.as<int>(), lv.centre.as<double>(),
                 lv.slot.as<int>(), p->adj_g[d].as<cpx<T>>(), lv.geom};
    }
    bool gathered = false;
    if constexpr (rows_ok<T, PS, PA>()) {
      if (p->pairs && !p->adj_pairs) build_adj_pairs(p, s);
      if (p->pairs && p->adj_pairs) {   // gather form from the pair lists
        StageTimer tm(p, s, IFGF_STAGE_ADJ_TARGETS);
        for (int d = 3; d <= D; ++d) {
          LevelPlan& lv = p->lev[d];
          if (lv.nrun == 0) continue;
          const dim3 grid((unsigned)((lv.nrun + TPB / 64 - 1) / (TPB / 64)), R);
          if constexpr (Prec<T>::f32 && adj_pairs_mfma_ok<PS, PA>())
            k_adj_pairs_mfma<PS, PA, false><<<grid, TPB, 0, s>>>(
                lv.pr_run.as<int>(), lv.nrun, lv.pr_loc.as<float4>(), lv.pr_fim.as<float>(), lv.pr_tgt.as<int>(),
                lv.pr_slot.as<int>(), (const cpx<float>*)vs, R, p->adj_g[d].as<cpx<float>>());
          else
            k_adj_pairs<T, PS, PA, false><<<grid, TPB, 0, s>>>(
                lv.pr_run.as<int>(), lv.nrun, lv.pr_loc.as<typename Vec4<T>::type>(), lv.pr_fim.as<T>(),
                lv.pr_tgt.as<int>(), lv.pr_slot.as<int>(), vs, R, p->adj_g[d].as<cpx<T>>());
          HIPCHK(hipGetLastError());
        }
        gathered = true;
      }
    }
    if (!gathered) {
      StageTimer tm(p, s, IFGF_STAGE_ADJ_TARGETS);
      k_adj_targets<T, PS, PA><<<gpts, TPB, 0, s>>>(p->pts.as<double>(), n, vs, L, 3, D, p->k, kind, R,
                                                    p->err.as<int>());
    }
    HIPCHK(hipGetLastError());
    const T* Ms = (const T*)(Prec<T>::f32 ? p->Msf.p : p->Ms.p);
    const T* Ma = (const T*)(Prec<T>::f32 ? p->Maf.p : p->Ma.p);
    for (int d = 3; d <= D; ++d) {
      LevelPlan& lv = p->lev[d];
      if (lv.nrel > 0) {
        StageTimer tm(p, s, IFGF_STAGE_ADJ_COEFFS);
        k_coeffs<T, PS, PA, true><<<dim3((lv.nrel + coeff_cones(P) - 1) / coeff_cones(P), R), TPB, 0, s>>>(p->adj_g[d].as<cpx<T>>(), lv.nrel, R, Ms, Ma,
                                                                  p->adj_g[d].as<cpx<T>>());
      }
      HIPCHK(hipGetLastError());
      if (d == D || lv.nrel == 0) continue;
      LevelPlan& lc = p->lev[d + 1];
      int64_t items = (int64_t)lv.nrel * P;
      if constexpr (rows_ok<T, PS, PA>()) {
        if (lv.nup > 0) {   // gather form from the upward pair list: one writer per child coefficient
          if (lv.up_nrun == 0) build_up_adj(p, d, s);
          StageTimer tm(p, s, IFGF_STAGE_ADJ_PROP);
          const dim3 grid((unsigned)((lv.up_nrun + TPB / 64 - 1) / (TPB / 64)), R);
          if constexpr (Prec<T>::f32 && adj_pairs_mfma_ok<PS, PA>())
            k_adj_pairs_mfma<PS, PA, true><<<grid, TPB, 0, s>>>(
                lv.up_run.as<int>(), lv.up_nrun, lv.up_loc.as<float4>(), lv.up_fim.as<float>(), lv.up_node.as<int>(),
                lv.up_slot.as<int>(), p->adj_g[d].as<cpx<float>>(), R, p->adj_g[d + 1].as<cpx<float>>());
          else
            k_adj_pairs<T, PS, PA, true><<<grid, TPB, 0, s>>>(
                lv.up_run.as<int>(), lv.up_nrun, lv.up_loc.as<typename Vec4<T>::type>(), lv.up_fim.as<T>(),
                lv.up_node.as<int>(), lv.up_slot.as<int>(), p->adj_g[d].as<cpx<T>>(), R,
                p->adj_g[d + 1].as<cpx<T>>());
          HIPCHK(hipGetLastError());
          continue;
        }
      }
      if constexpr (cone_major_order(PS, PA)) {
        if (R == 1 && lv.ti_geo_built) {   // gather form: one writer per child coefficient
          if (!lv.adj_built) build_adj_gather<T, PS, PA>(p, d, s);
          StageTimer tm(p, s, IFGF_STAGE_ADJ_PROP);
          if constexpr (adj_mfma<T, PS, PA>()) {
            if (lv.adj_ntile > 0)
              k_adj_ti_mfma<PA><<<(unsigned)lv.adj_ntile, 64, 0, s>>>(
                  lv.adj_tiles.as<int4>(), lv.adj_slots.as<int>(), lv.adj_gref.as<int2>(),
                  lv.adj_gref_off.as<int>(), lv.ti_geo.as<TiGeo<4, PA>>(), lv.ti_qlist.as<int>(),
                  lc.rel_box.as<int>(), lc.parent.as<int>(), lv.slot.as<int>(), lv.geom.ncone,
                  (const cpx<float>*)p->adj_g[d].p, (cpx<float>*)p->adj_g[d + 1].p);
          } else if (lv.adj_ntile > 0)
            k_adj_ti<T, PS, PA><<<(unsigned)lv.adj_ntile, 64, 0, s>>>(
                lv.adj_tiles.as<int4>(), lv.adj_slots.as<int>(), lv.adj_gref.as<int2>(), lv.adj_gref_off.as<int>(),
                lv.ti_geo.as<typename RecOf<T, PS, PA>::type>(), lv.ti_qlist.as<int>(), lc.rel_box.as<int>(),
                lc.parent.as<int>(), lv.slot.as<int>(), lv.geom.ncone, p->adj_g[d].as<cpx<T>>(),
                p->adj_g[d + 1].as<cpx<T>>());
          HIPCHK(hipGetLastError());
          continue;
        }
      }
      {
        StageTimer tm(p, s, IFGF_STAGE_ADJ_PROP);
        if constexpr (Prec<T>::f32) {   // the register table (FP64 would need twice the registers)
          const int64_t nwave = (items + 64 * kAdjRounds - 1) / (64 * kAdjRounds);
          k_adj_prop_tab<T, PS, PA><<<dim3((unsigned)((nwave + TPB / 64 - 1) / (TPB / 64)), R), TPB, 0, s>>>(
              lv.nrel, lv.rel_box.as<int>(), lv.rel_cone.as<int>(), lv.child_lo.as<int>(), lc.coords.as<int>(),
              lc.slot.as<int>(), p->adj_g[d].as<cpx<T>>(), p->adj_g[d + 1].as<cpx<T>>(), lv.geom, lc.geom, p->cheb,
              p->k, kind, R, p->err.as<int>());
        } else {
          k_adj_prop<T, PS, PA><<<dim3(nblocks(items), R), TPB, 0, s>>>(
              lv.nrel, lv.rel_box.as<int>(), lv.rel_cone.as<int>(), lv.child_lo.as<int>(), lc.coords.as<int>(),
              lc.slot.as<int>(), p->adj_g[d].as<cpx<T>>(), p->adj_g[d + 1].as<cpx<T>>(), lv.geom, lc.geom, p->cheb,
              p->k, kind, R, p->err.as<int>());
        }
      }
      HIPCHK(hipGetLastError());
    }
    {
      StageTimer tm(p, s, IFGF_STAGE_ADJ_LEAF);
      k_adj_leaf<T, PS, PA><<<dim3(lD.nb, R), TPB, 0, s>>>(p->pts.as<double>(), p->nrm.as<double>(),
                                                           lD.start.as<int>(), lD.centre.as<double>(),
                                                           lD.slot_off.as<int>(), lD.rel_cone.as<int>(),
                                                           p->adj_g[D].as<cpx<T>>(), lD.geom, p->cheb, p->k, p->eta,
                                                           kind, R, g);
    }
    HIPCHK(hipGetLastError());
  }
  {
    StageTimer tm(p, s, IFGF_STAGE_ADJ_OUT);
    k_adj_out<T><<<nblocks(n), TPB, 0, s>>>(g, p->perm.as<int>(), p->w.as<double>(), n, R, dtype, conj, out);
  }
  HIPCHK(hipGetLastError());
}

// ---------------------------------------------------------------------------
// Ragged batch: several plans (geometries) in one launch (one work-group per queue item).
//
// The whole apply of every geometry is cut into work items - gather chunks,
// near-field boxes, leaf boxes, coefficient chunks of the finest level,
// upward-pass items per level, target chunks - and laid out in one queue in
// an order that respects the data flow (gather < leaf, near < coefficients <
// upward pass d = D..4 < targets, per geometry; geometries interleaved within
// each phase).  A queue segment is a run of items of one kind, geometry and
// level; it names up to two (counter, count) pairs it needs and the counter
// its items increment.  Work-groups take items in queue order from one
// atomic head and wait, before an item, until its counters reach their
// counts.  Every counter an item waits on is incremented only by items of
// earlier segments, which running work-groups already hold, so the lowest
// unfinished item can always proceed: no cycle is possible, whatever the
// number of resident work-groups.  The wait is bounded (spin_limit polls);
// past the bound the item proceeds and the batch error flag is raised.
//
// Memory ordering across work-groups (and XCDs, whose L2 caches are not
// coherent with one another): after its item every wave issues an
// agent-scope release fence (its stores written back) before the block's
// counter increment; after a wait every wave issues an agent-scope acquire
// fence (stale cache lines dropped) before it reads.
// ---------------------------------------------------------------------------
enum { BT_GATHER = 0, BT_LEAF = 1, BT_NEAR = 2, BT_PROP = 4, BT_TARGET = 5, BT_PROPTI = 6, BT_PAIRS = 7, BT_PAIRSUM = 8,
       BT_UPAIRS = 9, BT_UPSUM = 10 };
// Threads per work-group of the batch launch: every stage body runs at this
// size (the cone-major tiles need 4 waves of 8 boxes).
constexpr int BBS = 256;
// Work units per queue item (fewer items, fewer counter updates and fences):
// gather chunks of BS points, upward-pass work items, the plan's balanced
// near-field and leaf work items (the leaf items also turn their whole
// cones' node values into coefficients); target items hold BBS points; a
// cone-major item is one tile.
constexpr int BG_GATHER = 4, BG_PROP = 8, BG_NEAR = 16, BG_LEAF = 8;
// pair items: BG_PAIRS chunks of BS sorted pairs; pair-sum items: BG_PAIRSUM x BS / 16 targets;
// upward pair items: BG_UPAIRS chunks of BS pairs; upward sum items: BG_UPSUM chunks of coeff_cones(P) cones
constexpr int BG_PAIRS = 32, BG_PAIRSUM = 8, BG_UPAIRS = 64, BG_UPSUM = 16;

template <typename T> struct BLevel {
  int nb, nrel, nwork, n_near, n_leaf;
  const int IFGF_GAS* start;
  const int IFGF_GAS* nbr_off;
  const int IFGF_GAS* nbr;
  const int IFGF_GAS* slot_off;
  const int IFGF_GAS* rel_cone;
  const int IFGF_GAS* rel_box;
  const int IFGF_GAS* child_lo;
  const int IFGF_GAS* coords;
  const int IFGF_GAS* slot;
  const double IFGF_GAS* centre;
  const int4 IFGF_GAS* work;
  const int4 IFGF_GAS* near_work;   // finest level: near-field work items
  const int4 IFGF_GAS* leaf_work;   // finest level: leaf work items (whole cones)
  const int4 IFGF_GAS* ti_tile;   // cone-major tiles of the pass into this level (FP32)
  const int IFGF_GAS* ti_slot;
  const int IFGF_GAS* ti_child;
  const uint4 IFGF_GAS* ti_geo;   // node records per (cone id, octant) of the tiles (FP32)
  cpx<T> IFGF_GAS* Fn;
  cpx<T> IFGF_GAS* Fc;
  LevelGeom g;
};

template <typename T> struct BGeom {
  int64_t n;
  int D, kind;
  int trows;   // cousin targets in the row-broadcast formulation
  int pairs;   // cousin targets from the plan's pair lists (two item kinds)
  int64_t pchunk[IFGF_MAX_LEVELS + 1];   // pair items: level d's first item (d = 3 .. D), then the total
  double k, eta;
  const double IFGF_GAS* pts;
  const double IFGF_GAS* nrm;
  const double IFGF_GAS* w;
  const int IFGF_GAS* perm;
  const T IFGF_GAS* Ms;
  const T IFGF_GAS* Ma;
  cpx<T> IFGF_GAS* a;
  cpx<T> IFGF_GAS* uacc;
  int IFGF_GAS* err;
  ChebTab ct;
  TLevels<T> tl;
  PLevels<T> pl;
  PLevels<T> up;                                  // upward pair lists of the passes into level l (index l)
  const int IFGF_GAS* up_base[IFGF_MAX_LEVELS];
  BLevel<T> lv[IFGF_MAX_LEVELS];
};

// Per-apply input and output pointers, one pair per geometry.
struct BIo {
  const void* sigma[IFGF_BATCH_MAX];
  void* u[IFGF_BATCH_MAX];
};

__device__ __forceinline__ void batch_wait(int* ctr, int dep, int need, int spin_limit, int* berr) {
  if (dep < 0) return;
  int polls = 0;
  while (__hip_atomic_load(&ctr[dep], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
    if (polls++ >= spin_limit) {
      atomicOr(berr, 1);
      return;
    }
    __builtin_amdgcn_s_sleep(4);
  }
}

// A leaf item with its cones' coefficient transform (one RHS).
template <typename T, int PS, int PA> struct BLeafSmem {
  static constexpr int P = PS * PA * PA;
  static constexpr int NCF = kLeafChunk / P > 0 ? kLeafChunk / P : 1;
  LeafSmem<T, 1> leaf;
  cpx<T> fv[NCF * P], ft[NCF * P];
  T ms[PS * PS], ma[PA * PA];
};

template <typename T, int PS, int PA> struct BatchSmem {
  static constexpr size_t a = sizeof(PropSmem<T, PS, PA, BBS>), b = sizeof(NearSmem<T, 1, BBS>),
                          c = sizeof(BLeafSmem<T, PS, PA>), t = Prec<T>::f32 ? sizeof(TiSmem<PS, PA, 4>) : 0;
  static constexpr size_t u = sizeof(UpsumSmem<T, PS, PA>);
  static constexpr size_t ab = a > b ? a : b, ct = c > t ? c : t, abu = ab > u ? ab : u;
  static constexpr size_t bytes = abu > ct ? abu : ct;
};

// One launch of `total` work-groups; each takes the next ticket of the queue
// when it starts and processes that item.  A work-group holds its ticket only
// while it runs, so every lower ticket belongs to a running or finished
// work-group.  (A loop over several items per work-group would let the
// compiler hoist every body's per-thread invariants out of the loop and keep
// them all live at once, which costs far more registers than any one body.)
// FP32: 3 waves per SIMD, as the standalone upward pass; FP64: 1 (its bodies need
// more than the 256 registers a wave can address, the rest goes to AGPRs).
template <typename T, int PS, int PA>
__global__ __launch_bounds__(BBS)
__attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 3 : 1))) void k_batch(const BSeg* __restrict__ segs,
                                                                          const int* __restrict__ seg_of, int total,
                                                                          const BGeom<T>* __restrict__ geoms, BIo io,
                                                                          int dtype, int* ctr, int spin_limit,
                                                                          int* berr) {
  constexpr int P = PS * PA * PA;
  constexpr int BS = BBS;
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int s_item, s_seg;
  if (threadIdx.x == 0) {
    const int it = atomicAdd(&ctr[0], 1);
    int sg = -1;
    if (it < total) {
      sg = seg_of[it];
      batch_wait(ctr, segs[sg].dep0, segs[sg].need0, spin_limit, berr);
      batch_wait(ctr, segs[sg].dep1, segs[sg].need1, spin_limit, berr);
    }
    // one agent-scope acquire per item that consumes other work-groups'
    // results: the L1/L2 lines it drops are dropped for every wave of the
    // work-group
    if (sg >= 0 && (segs[sg].dep0 >= 0 || segs[sg].dep1 >= 0)) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    s_item = it;
    s_seg = sg;
  }
  __syncthreads();
  // block-uniform; readfirstlane lets the compiler branch on them as such
  const int it = __builtin_amdgcn_readfirstlane(s_item), sg = __builtin_amdgcn_readfirstlane(s_seg);
  if (it >= total) return;
  const BSeg S = segs[sg];
  const BGeom<T>& G = geoms[S.geom];
  const int local = it - S.first;
  const int D = G.D;
  switch (S.type) {
    case BT_GATHER:
      for (int u = 0; u < BG_GATHER; ++u)
        gather_one<T>(((int64_t)local * BG_GATHER + u) * BS + threadIdx.x, io.sigma[S.geom], dtype, 0, gen(G.perm),
                      gen(G.w), G.n, 1, gen(G.a), G.n);
      break;
    case BT_NEAR: {   // near-field work items (box, first target, targets)
      const BLevel<T>& L = G.lv[D];
      const int w1 = min((local + 1) * BG_NEAR, L.n_near);
      for (int w = local * BG_NEAR; w < w1; ++w) {
        if (w > local * BG_NEAR) __syncthreads();   // LDS reuse
        const int4 wk = gen(L.near_work)[w];
        near_box<T, false, 1, BS>(*reinterpret_cast<NearSmem<T, 1, BS>*>(smem), wk.x, wk.y, wk.z, 0, gen(G.pts),
                                  gen(G.nrm), gen(G.a), 1, gen(L.start), gen(L.nbr_off), gen(L.nbr), gen(L.centre),
                                  G.k, G.eta, G.kind, gen(G.uacc));
      }
      break;
    }
    case BT_LEAF: {   // leaf work items (box, first item, items; whole cones), then their coefficients
      auto& sm = *reinterpret_cast<BLeafSmem<T, PS, PA>*>(smem);
      const BLevel<T>& L = G.lv[D];
      if (threadIdx.x < PS * PS) sm.ms[threadIdx.x] = G.Ms[threadIdx.x];
      if (threadIdx.x < PA * PA) sm.ma[threadIdx.x] = G.Ma[threadIdx.x];
      const int w1 = min((local + 1) * BG_LEAF, L.n_leaf);
      for (int w = local * BG_LEAF; w < w1; ++w) {
        if (w > local * BG_LEAF) __syncthreads();   // LDS reuse
        const int4 wk = gen(L.leaf_work)[w];
        leaf_box<T, PS, PA, 1, BS>(sm.leaf, wk.x, wk.y, wk.z, 0, gen(G.pts), gen(G.nrm), gen(G.a), 1, gen(L.start),
                                   gen(L.centre), gen(L.slot_off), gen(L.rel_cone), L.g, G.ct, G.k, G.eta, G.kind,
                                   gen(L.Fn), sm.fv);
        __syncthreads();
        const int* so = gen(L.slot_off);
        const int ncn = so[wk.x + 1] - so[wk.x];
        const int c0 = wk.y / P, nc = min(ncn * P, wk.y + wk.z) / P - c0;
        lds_coeffs_store<T, PS, PA, BS>(sm.fv, sm.ft, nc, sm.ms, sm.ma, gen(L.Fc) + ((int64_t)so[wk.x] + c0) * P,
                                        1, 0);
      }
      break;
    }
    case BT_PROP: {
      const int d = S.level;   // child level
      const BLevel<T>& lc = G.lv[d];
      const BLevel<T>& lp = G.lv[d - 1];
      const int w1 = min((local + 1) * BG_PROP, lp.nwork);
      for (int w = local * BG_PROP; w < w1; ++w) {
        if (w > local * BG_PROP) __syncthreads();   // LDS reuse
        prop_item<T, PS, PA, true, BBS>(*reinterpret_cast<PropSmem<T, PS, PA, BBS>*>(smem), gen(lp.work)[w], 0,
                                   gen(lp.rel_cone), gen(lp.child_lo), gen(lc.coords), gen(lc.slot), gen(lc.Fc), lp.g,
                                   lc.g, G.ct, gen(G.Ms), gen(G.Ma), G.k, G.kind, 1, gen(lp.Fc), gen(G.err));
      }
      break;
    }
    case BT_PROPTI: {
      if constexpr (Prec<T>::f32) {
        const int d = S.level;   // child level
        const BLevel<T>& lc = G.lv[d];
        const BLevel<T>& lp = G.lv[d - 1];
        prop_ti_tile<PS, PA, 4>(*reinterpret_cast<TiSmem<PS, PA, 4>*>(smem), gen(lp.ti_tile)[local],
                                gen(lp.ti_slot), gen(lp.ti_child),
                                reinterpret_cast<const TiGeo<PS, PA>*>(gen(lp.ti_geo)), gen(lc.slot), gen(lc.Fc),
                                lp.g, lc.g, G.ct, gen(G.Ms), gen(G.Ma), G.k, G.kind, gen(lp.Fc), gen(G.err));
      }
      break;
    }
    case BT_UPAIRS: {   // BG_UPAIRS chunks of BS sorted upward pairs of the pass S.level -> S.level - 1
      const PLevel<T>& ul = G.up.lv[S.level - 1];
      const int64_t n = (ul.np + BS - 1) / BS;
      const int64_t c0 = (int64_t)local * BG_UPAIRS, c1 = min(c0 + BG_UPAIRS, n);
      for (int64_t c = c0; c < c1; ++c) pairs_block<T, PS, PA>(ul, c * BS);
      break;
    }
    case BT_UPSUM: {   // BG_UPSUM chunks of coeff_cones(P) cones of level S.level - 1: node sums, coefficients
      constexpr int NC = coeff_cones(PS * PA * PA);
      const int l = S.level - 1;
      const BLevel<T>& lp = G.lv[l];
      for (int u = 0; u < BG_UPSUM; ++u) {
        const int c0 = (local * BG_UPSUM + u) * NC;
        if (c0 >= lp.nrel) break;   // block-uniform
        if (u > 0) __syncthreads();   // LDS reuse
        upsum_chunk<T, PS, PA>(*reinterpret_cast<UpsumSmem<T, PS, PA>*>(smem), c0, gen(G.up_base[l]),
                               G.up.lv[l].pos, G.up.lv[l].val, lp.nrel, gen(G.Ms), gen(G.Ma), gen(lp.Fc));
      }
      break;
    }
    case BT_PAIRS: {   // BG_PAIRS chunks of BS sorted pairs of level S.level: their values
      const int d = S.level;
      const int64_t n = G.pchunk[d + 1] - G.pchunk[d];
      const int64_t c0 = (int64_t)local * BG_PAIRS, c1 = min(c0 + BG_PAIRS, n);
      for (int64_t c = c0; c < c1; ++c) pairs_block<T, PS, PA>(G.pl.lv[d], c * BS);
      break;
    }
    case BT_PAIRSUM:   // BG_PAIRSUM x BS / 16 targets: near field + their pair values, to the caller's order
      for (int u = 0; u < BG_PAIRSUM; ++u)
        pairsum16<T>(((int64_t)local * BG_PAIRSUM + u) * BS + threadIdx.x, G.n, gen(G.perm), gen(G.uacc), 1, G.pl,
                     3, D, dtype, io.u[S.geom]);
      break;
    case BT_TARGET: {
      const int dlo = D >= 3 ? 3 : 1, dhi = D >= 3 ? D : 0;
      if (G.trows) {
        // the row-broadcast formulation, all levels in turn (as the separate
        // apply adds them: near field, then the levels from the finest down)
        const int64_t i0 = (int64_t)local * BS + threadIdx.x;
        const bool valid = i0 < G.n;
        const int64_t i = valid ? i0 : G.n - 1;
        const double* P3 = gen(G.pts) + 3 * i;
        const double x[3] = {P3[0], P3[1], P3[2]};
        const cpx<T> un = gen(G.uacc)[i];
        double re = un.re, im = un.im;
        for (int d = dhi; d >= dlo; --d) {
          T lr = 0, li = 0;
          rows_level<T, PS, PA>(G.tl.lv[d], x, valid, i, G.k, G.kind, gen(G.err), lr, li);
          re += lr;
          im += li;
        }
        if (valid) {
          const int64_t o = gen(G.perm)[i];
          if (dtype == IFGF_C128) {
            ((double*)io.u[S.geom])[2 * o] = re;
            ((double*)io.u[S.geom])[2 * o + 1] = im;
          } else {
            ((float*)io.u[S.geom])[2 * o] = (float)re;
            ((float*)io.u[S.geom])[2 * o + 1] = (float)im;
          }
        }
      } else {
        auto& sm = *reinterpret_cast<PropSmem<T, PS, PA, BBS>*>(smem);
        target_point<T, PS, PA>(sm.cbuf[threadIdx.x >> 6], (int64_t)local * BS + threadIdx.x, 0, gen(G.pts), G.n,
                                gen(G.perm), gen(G.uacc), 1, G.tl, dlo, dhi, G.k, G.kind, 1, dtype, 0, nullptr,
                                io.u[S.geom], gen(G.err));
      }
      break;
    }
    default:
      break;
  }
  // every wave waits until its stores have reached L2; then one agent-scope
  // release (L2 write-back) covers the stores of the whole work-group
  if (S.type == BT_TARGET || S.type == BT_PAIRSUM) return;   // nothing in the launch consumes the targets' output
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    atomicAdd(&ctr[S.done], 1);
  }
}

__global__ __launch_bounds__(TPB) void k_zero_i32(int* __restrict__ x, int n) {
  const int i = blockIdx.x * TPB + threadIdx.x;
  if (i < n) x[i] = 0;
}

template <typename T, int PS, int PA>
void batch_prepare_impl(ifgf_batch_s* b) {
  constexpr int P = PS * PA * PA;
  constexpr int BS = BBS;
  const int ng = (int)b->plans.size();
  std::vector<BGeom<T>> geo(ng);
  for (int g = 0; g < ng; ++g) {
    ifgf_plan_s* p = b->plans[g];
    BGeom<T>& G = geo[g];
    G = BGeom<T>{};
    G.n = p->n;
    G.D = p->D;
    G.kind = p->opt.kernel;
    G.trows = p->opt.target_kernel != IFGF_TARGET_WAVE;
    G.k = p->k;
    G.eta = p->eta;
    G.pts = gas(p->pts.as<const double>());
    G.nrm = gas(p->nrm.as<const double>());
    G.w = gas(p->w.as<const double>());
    G.perm = gas(p->perm.as<const int>());
    G.Ms = gas((const T*)(Prec<T>::f32 ? p->Msf.p : p->Ms.p));
    G.Ma = gas((const T*)(Prec<T>::f32 ? p->Maf.p : p->Ma.p));
    G.a = gas(p->a.as<cpx<T>>());
    G.uacc = gas(p->uacc.as<cpx<T>>());
    G.err = gas(p->err.as<int>());
    G.ct = p->cheb;
    G.pairs = p->pairs && rows_ok<T, PS, PA>() ? 1 : 0;
    int64_t pc = 0;
    for (int d = 0; d <= IFGF_MAX_LEVELS; ++d) G.pchunk[d] = 0;
    for (int d = 3; d <= p->D && G.pairs; ++d) {
      const LevelPlan& l = p->lev[d];
      G.pl.lv[d] = {l.npair, l.pr_slot.as<int>(), l.pr_loc.as<typename Vec4<T>::type>(), l.pr_fim.as<T>(),
                    l.pr_val.as<cpx<T>>(), l.pr_off.as<int>(), l.pr_pos.as<int>(), l.Fc.as<cpx<T>>()};
      G.pchunk[d] = pc;
      pc += (l.npair + BBS - 1) / BBS;
    }
    if (G.pairs) G.pchunk[p->D + 1] = pc;
    if constexpr (rows_ok<T, PS, PA>()) {
      for (int l = 3; l < p->D; ++l) {   // upward pair lists the plan's applies use
        const LevelPlan& lp = p->lev[l];
        if (!lp.up_use || lp.nup == 0) continue;
        G.up.lv[l] = {lp.nup, lp.up_slot.as<int>(), lp.up_loc.as<typename Vec4<T>::type>(), lp.up_fim.as<T>(),
                      lp.up_val.as<cpx<T>>(), nullptr, lp.up_pos.as<int>(), p->lev[l + 1].Fc.as<cpx<T>>()};
        G.up_base[l] = gas(lp.up_base.as<const int>());
      }
    }
    for (int d = 1; d <= p->D; ++d) {
      const LevelPlan& l = p->lev[d];
      BLevel<T>& L = G.lv[d];
      L.nb = l.nb;
      L.nrel = l.nrel;
      L.nwork = (int)l.nwork;
      L.n_near = l.n_near;
      L.n_leaf = l.n_leaf;
      L.start = gas(l.start.as<const int>());
      L.nbr_off = gas(l.nbr_off.as<const int>());
      L.nbr = gas(l.nbr.as<const int>());
      L.slot_off = gas(l.slot_off.as<const int>());
      L.rel_cone = gas(l.rel_cone.as<const int>());
      L.rel_box = gas(l.rel_box.as<const int>());
      L.child_lo = gas(l.child_lo.as<const int>());
      L.coords = gas(l.coords.as<const int>());
      L.slot = gas(l.slot.as<const int>());
      L.centre = gas(l.centre.as<const double>());
      L.work = gas(l.work.as<const int4>());
      L.near_work = gas(l.near_work.as<const int4>());
      L.leaf_work = gas(l.leaf_work.as<const int4>());
      L.ti_tile = gas(l.ti_tile.as<const int4>());
      L.ti_slot = gas(l.ti_slot.as<const int>());
      L.ti_child = gas(l.ti_child.as<const int>());
      L.ti_geo = gas(l.ti_geo.as<const uint4>());
      L.Fn = gas(l.Fn.as<cpx<T>>());
      L.Fc = gas(l.Fc.as<cpx<T>>());
      L.g = l.geom;
      if (d >= 3)
        G.tl.lv[d] = {gas(l.pbox.as<const int>()), gas(l.cou_off.as<const int>()), gas(l.cou.as<const int>()),
                      gas(l.centre.as<const double>()), gas(l.slot.as<const int>()), gas(l.Fc.as<const cpx<T>>()),
                      l.geom};
    }
  }

  // ---- the queue ----------------------------------------------------------------
  auto C = [](int g, int k) { return 1 + kBatchCtrPerGeom * g + k; };   // counters: 0 = queue head, then per geometry
  // K_PROP0 + l: the coefficients of level l; K_UPV0 + l: the upward pair values of the pass into level l
  enum { K_GATHER = 0, K_LEAF = 1, K_NEAR = 2, K_PAIRS = 3, K_PROP0 = 4, K_UPV0 = 16, K_TARGET = 31 };
  static_assert(K_PROP0 + IFGF_MAX_LEVELS - 1 < K_UPV0 && K_UPV0 + IFGF_MAX_LEVELS - 1 < K_TARGET &&
                    K_TARGET < kBatchCtrPerGeom, "batch counter layout");
  std::vector<BSeg> segs;
  int64_t first = 0;
  auto emit = [&](int type, int g, int level, int64_t count, int dep0, int need0, int dep1, int need1, int done) {
    if (count <= 0) return;
    BSeg q{};
    q.type = type;
    q.geom = g;
    q.level = level;
    q.count = (int)count;
    q.first = (int)first;
    q.dep0 = need0 > 0 ? dep0 : -1;
    q.need0 = need0;
    q.dep1 = need1 > 0 ? dep1 : -1;
    q.need1 = need1;
    q.done = done;
    segs.push_back(q);
    first += count;
    if (first > (int64_t)0x7fffffff) throw Error{IFGF_EUNSUPPORTED, "batch queue too long"};
  };
  std::vector<int64_t> ngat(ng), nnear(ng), nleaf(ng);
  std::vector<std::pair<int, int>> last(ng, {-1, 0});   // producer of the newest coefficient level
  for (int g = 0; g < ng; ++g) {
    ngat[g] = (b->plans[g]->n + (int64_t)BS * BG_GATHER - 1) / ((int64_t)BS * BG_GATHER);
    emit(BT_GATHER, g, 0, ngat[g], -1, 0, -1, 0, C(g, K_GATHER));
  }
  for (int g = 0; g < ng; ++g) {   // leaf factors with the finest level's coefficients
    ifgf_plan_s* p = b->plans[g];
    nleaf[g] = p->D >= 3 ? (p->lev[p->D].n_leaf + BG_LEAF - 1) / BG_LEAF : 0;
    emit(BT_LEAF, g, p->D, nleaf[g], C(g, K_GATHER), (int)ngat[g], -1, 0, C(g, K_LEAF));
    if (nleaf[g] > 0) last[g] = {C(g, K_LEAF), (int)nleaf[g]};
  }
  for (int g = 0; g < ng; ++g) {
    ifgf_plan_s* p = b->plans[g];
    nnear[g] = (p->lev[p->D].n_near + BG_NEAR - 1) / BG_NEAR;
    emit(BT_NEAR, g, p->D, nnear[g], C(g, K_GATHER), (int)ngat[g], -1, 0, C(g, K_NEAR));
  }
  // Upward pass in steps j = 0, 1, ...: step j takes level D_g - j -> D_g - j - 1
  // of every geometry g.  A geometry's targets follow its last step, so the
  // targets of shallow trees overlap the upward pass of deeper ones.
  int maxD = 0;
  for (auto* p : b->plans) maxD = std::max(maxD, p->D);
  // Pair values of level d need only level d's coefficients: they are queued
  // right behind the next upward step, whose waits they fill.
  std::vector<std::vector<std::pair<int, int>>> made(ng);   // made[g][d]: producer of level d's coefficients
  std::vector<int> pend(ng);                                // next level whose pairs are not queued
  std::vector<int64_t> npair(ng, 0);
  for (int g = 0; g < ng; ++g) {
    made[g].assign(IFGF_MAX_LEVELS + 1, {-1, 0});
    made[g][b->plans[g]->D] = last[g];
    pend[g] = b->plans[g]->D;
  }
  auto emit_pairs = [&](int g, int dmin) {   // the pair items of levels pend[g] down to dmin
    const BGeom<T>& G = geo[g];
    for (; G.pairs && pend[g] >= std::max(3, dmin); --pend[g]) {
      const int d = pend[g];
      const int64_t np = (G.pchunk[d + 1] - G.pchunk[d] + BG_PAIRS - 1) / BG_PAIRS;
      emit(BT_PAIRS, g, d, np, made[g][d].first, made[g][d].second, -1, 0, C(g, K_PAIRS));
      npair[g] += std::max<int64_t>(0, np);
    }
  };
  auto emit_targets = [&](int g) {
    const BGeom<T>& G = geo[g];
    if (G.pairs) {   // the remaining pair values, then the per-target sums
      emit_pairs(g, 3);
      emit(BT_PAIRSUM, g, 0, (16 * b->plans[g]->n + (int64_t)BS * BG_PAIRSUM - 1) / ((int64_t)BS * BG_PAIRSUM),
           C(g, K_PAIRS), (int)npair[g], C(g, K_NEAR), (int)nnear[g], C(g, K_TARGET));
    } else {
      emit(BT_TARGET, g, 0, (b->plans[g]->n + BS - 1) / BS, C(g, K_NEAR), (int)nnear[g], last[g].first,
           last[g].second, C(g, K_TARGET));
    }
  };
  for (int g = 0; g < ng; ++g)
    if (b->plans[g]->D < 4) emit_targets(g);
  for (int j = 0; j + 4 <= maxD; ++j) {
    for (int g = 0; g < ng; ++g) {
      ifgf_plan_s* p = b->plans[g];
      const int d = p->D - j;   // child level
      if (d < 4) continue;
      const LevelPlan& lp = p->lev[d - 1];
      if (lp.nrel == 0 || lp.nwork == 0) continue;
      if (geo[g].up.lv[d - 1].np > 0) {   // the plan's upward pair list: pair values, then node sums
        const int64_t nv = ((geo[g].up.lv[d - 1].np + BS - 1) / BS + BG_UPAIRS - 1) / BG_UPAIRS;
        const int NC = coeff_cones(P);
        const int64_t ns = ((lp.nrel + NC - 1) / NC + BG_UPSUM - 1) / BG_UPSUM;
        emit(BT_UPAIRS, g, d, nv, last[g].first, last[g].second, -1, 0, C(g, K_UPV0 + d - 1));
        emit(BT_UPSUM, g, d, ns, C(g, K_UPV0 + d - 1), (int)nv, -1, 0, C(g, K_PROP0 + d - 1));
        last[g] = {C(g, K_PROP0 + d - 1), (int)ns};
        continue;
      }
      // the cone-major tiles where the plan has them (FP32), else node work items
      const bool ti = Prec<T>::f32 && lp.ntile > 0;
      const int64_t cnt = ti ? lp.ntile : (lp.nwork + BG_PROP - 1) / BG_PROP;
      emit(ti ? BT_PROPTI : BT_PROP, g, d, cnt, last[g].first, last[g].second, -1, 0, C(g, K_PROP0 + d - 1));
      last[g] = {C(g, K_PROP0 + d - 1), (int)cnt};
    }
    for (int g = 0; g < ng; ++g) {
      const int d = b->plans[g]->D - j;
      if (d < 4) continue;
      made[g][d - 1] = last[g];
      emit_pairs(g, d);   // level d's pairs behind the step out of it
    }
    for (int g = 0; g < ng; ++g)
      if (b->plans[g]->D - j == 4) emit_targets(g);   // its last step was this one
  }

  // Every counter a segment waits on must be complete-able by earlier segments
  // alone, with exactly the awaited number of items.
  for (size_t i = 0; i < segs.size(); ++i) {
    for (int w = 0; w < 2; ++w) {
      const int dep = w ? segs[i].dep1 : segs[i].dep0, need = w ? segs[i].need1 : segs[i].need0;
      if (dep < 0) continue;
      int64_t before = 0, after = 0;
      for (size_t j = 0; j < segs.size(); ++j)
        if (segs[j].done == dep) (j < i ? before : after) += segs[j].count;
      if (before != need || after != 0) throw Error{IFGF_EUNSUPPORTED, "internal error: batch queue order"};
    }
  }

  b->nseg = (int)segs.size();
  b->total = (int)first;
  std::vector<int> seg_of((size_t)std::max<int64_t>(1, first));
  for (size_t i = 0; i < segs.size(); ++i)
    for (int q = 0; q < segs[i].count; ++q) seg_of[(size_t)segs[i].first + q] = (int)i;
  b->seg_of.alloc(sizeof(int) * seg_of.size());
  HIPCHK(hipMemcpy(b->seg_of.p, seg_of.data(), sizeof(int) * seg_of.size(), hipMemcpyHostToDevice));
  b->nctr = 1 + kBatchCtrPerGeom * ng;
  b->segs.alloc(sizeof(BSeg) * std::max<size_t>(1, segs.size()));
  if (!segs.empty()) HIPCHK(hipMemcpy(b->segs.p, segs.data(), sizeof(BSeg) * segs.size(), hipMemcpyHostToDevice));
  b->geoms.alloc(sizeof(BGeom<T>) * ng);
  HIPCHK(hipMemcpy(b->geoms.p, geo.data(), sizeof(BGeom<T>) * ng, hipMemcpyHostToDevice));
  b->ctr.alloc(sizeof(int) * b->nctr);
  b->err.alloc(sizeof(int) * 4);
  HIPCHK(hipMemset(b->err.p, 0, sizeof(int) * 4));
  b->smem = BatchSmem<T, PS, PA>::bytes;
  int per_cu = 0;
  HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch<T, PS, PA>, BS, b->smem));
  if (per_cu < 1) throw Error{IFGF_EUNSUPPORTED, "batch kernel does not fit on a compute unit"};
  b->grid = b->total;
  b->block = BS;
}

template <typename T, int PS, int PA>
void batch_apply_impl(ifgf_batch_s* b, const void* const* sigma, void* const* u, int dtype, int* ctr,
                      hipStream_t s) {
  BIo io{};
  const int ng = (int)b->plans.size();
  for (int g = 0; g < ng; ++g) {
    io.sigma[g] = sigma[g];
    io.u[g] = u[g];
  }
  // the counters start at zero; a fill kernel rather than a memset, so that a
  // captured graph replays it as an ordinary kernel node
  k_zero_i32<<<nblocks(b->nctr), TPB, 0, s>>>(ctr, b->nctr);
  HIPCHK(hipGetLastError());
  if (b->total == 0) return;
  k_batch<T, PS, PA><<<b->grid, b->block, b->smem, s>>>(b->segs.as<BSeg>(), b->seg_of.as<int>(), b->total,
                                                        b->geoms.as<BGeom<T>>(), io, dtype, ctr, b->spin_limit,
                                                        b->err.as<int>());
  HIPCHK(hipGetLastError());
}

// Interpolation orders (P_s, P_ang) compiled in: the ORDERS_ALL list in both
// precisions (every formulation: node and cone-major upward pass, row and
// wave targets, batched right-hand sides, ragged batch); the ORDERS_FP64 list
// in FP64 only, for accuracy beyond FP32's reach (node upward pass, wave
// targets, transposed apply; no ragged batch).
#define IFGF_ORDERS_ALL(X) X(3, 5) X(4, 6)
#define IFGF_ORDERS_FP64(X) X(8, 8)

template <typename T>
void dispatch_adjoint(ifgf_plan_s* p, const void* v, void* out, int R, int dtype, int conj, hipStream_t s) {
  const int ps = p->opt.p_s, pa = p->opt.p_ang;
#define X(a, b) \
  if (ps == a && pa == b) return adjoint_impl<T, a, b>(p, v, out, R, dtype, conj, s);
  IFGF_ORDERS_ALL(X)
  if constexpr (!Prec<T>::f32) {
    IFGF_ORDERS_FP64(X)
  }
#undef X
  throw Error{IFGF_EUNSUPPORTED, "interpolation order not compiled"};
}

template <typename T>
void dispatch_apply(ifgf_plan_s* p, const void* sigma, void* u, int R, int dtype, int stage_mask, int lo, int hi,
                    hipStream_t s) {
  const int ps = p->opt.p_s, pa = p->opt.p_ang;
#define X(a, b) \
  if (ps == a && pa == b) return apply_impl<T, a, b>(p, sigma, u, R, dtype, stage_mask, lo, hi, s);
  IFGF_ORDERS_ALL(X)
  if constexpr (!Prec<T>::f32) {
    IFGF_ORDERS_FP64(X)
  }
#undef X
  throw Error{IFGF_EUNSUPPORTED, "interpolation order not compiled"};
}

// The finest level's node values of the last apply, from its coefficients:
// v_abc = sum_ijl T_i(x_a) T_j(x_b) T_l(x_c) c_ijl (the inverse of the
// coefficient transform, the same three separable passes with the matrices
// of Chebyshev values at the nodes).  The single-RHS apply keeps the node
// values in LDS only, so they are recovered here when asked for.
template <typename T, int PS, int PA>
void export_nodes_impl(ifgf_plan_s* p, void* dst, hipStream_t s) {
  constexpr int P = PS * PA * PA;
  LevelPlan& l = p->lev[p->D];
  const int R = std::max(1, p->last_rhs);
  if (l.nrel == 0) return;
  std::vector<T> mi(PS * PS), ai(PA * PA);
  for (int a = 0; a < PS; ++a)
    for (int i = 0; i < PS; ++i) mi[a * PS + i] = (T)std::cos(i * (2.0 * a + 1.0) * IFGF_PI / (2.0 * PS));
  for (int b = 0; b < PA; ++b)
    for (int j = 0; j < PA; ++j) ai[b * PA + j] = (T)std::cos(j * (2.0 * b + 1.0) * IFGF_PI / (2.0 * PA));
  DevBuf md, ad;
  md.alloc(sizeof(T) * mi.size());
  ad.alloc(sizeof(T) * ai.size());
  HIPCHK(hipMemcpyAsync(md.p, mi.data(), sizeof(T) * mi.size(), hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(ad.p, ai.data(), sizeof(T) * ai.size(), hipMemcpyHostToDevice, s));
  k_coeffs<T, PS, PA, false><<<dim3((l.nrel + coeff_cones(P) - 1) / coeff_cones(P), R), TPB, 0, s>>>(
      l.Fc.as<cpx<T>>(), l.nrel, R, md.as<T>(), ad.as<T>(), (cpx<T>*)dst);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s));   // the matrices are freed on return
}

template <typename T, int PS, int PA>
void far_field_impl(ifgf_plan_s* p, const void* sigma, int64_t ndir, const double* dirs, void* uinf, int dtype,
                    hipStream_t s) {
  // the leaf factors and the upward pass to level 3, as in the apply
  // (stage mask 0: no near field, no cousin targets; u, of sigma's dtype,
  // is discarded)
  DevBuf tmp;
  tmp.alloc(sizeof(cpx<double>) * (size_t)p->n);
  apply_impl<T, PS, PA>(p, sigma, tmp.p, 1, dtype, 0, 0, 0, s);
  const unsigned grid = (unsigned)((ndir * 64 + TPB - 1) / TPB);
  if (p->D >= 3) {
    const LevelPlan& l3 = p->lev[3];
    k_far_field<T, PS, PA><<<grid, TPB, 0, s>>>(dirs, ndir, l3.nb, l3.centre.as<double>(), l3.slot.as<int>(),
                                                l3.Fc.as<cpx<T>>(), l3.geom, p->k, dtype, uinf, p->err.as<int>());
  } else {
    k_far_direct<T><<<grid, TPB, 0, s>>>(dirs, ndir, p->pts.as<double>(), p->nrm.as<double>(), p->a.as<cpx<T>>(),
                                         p->n, p->k, p->eta, dtype, uinf);
  }
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s));   // tmp is freed on return
}

template <typename T>
void dispatch_far_field(ifgf_plan_s* p, const void* sigma, int64_t ndir, const double* dirs, void* uinf, int dtype,
                        hipStream_t s) {
  const int ps = p->opt.p_s, pa = p->opt.p_ang;
#define X(a, b) \
  if (ps == a && pa == b) return far_field_impl<T, a, b>(p, sigma, ndir, dirs, uinf, dtype, s);
  IFGF_ORDERS_ALL(X)
  if constexpr (!Prec<T>::f32) {
    IFGF_ORDERS_FP64(X)
  }
#undef X
  throw Error{IFGF_EUNSUPPORTED, "interpolation order not compiled"};
}

__global__ __launch_bounds__(TPB) void k_fill_one(double* __restrict__ x, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (i < n) {
    x[2 * i] = 1.0;
    x[2 * i + 1] = 0.0;
  }
}

// Measured choice of the one-RHS formulations of a plan: for every level of
// the upward pass, the node formulation against cone-major tiles of 8, 16 and
// 32 boxes (those the level and precision allow), each timed with events over
// `reps` passes on the plan's own data; then row-broadcast against per-wave
// cousin targets, over `reps` whole applies.  The fastest is kept in the plan.
template <typename T, int PS, int PA>
void autotune_impl(ifgf_plan_s* p, int reps, ifgf_tune_report* rep, hipStream_t s) {
  const int D = p->D;
  *rep = ifgf_tune_report{};
  DevBuf sig, out;
  sig.alloc(sizeof(double) * 2 * (size_t)p->n);
  out.alloc(sizeof(double) * 2 * (size_t)p->n);
  k_fill_one<<<nblocks(p->n), TPB, 0, s>>>(sig.as<double>(), p->n);
  HIPCHK(hipGetLastError());
  auto full_apply = [&]() { apply_impl<T, PS, PA>(p, sig.p, out.p, 1, IFGF_C128, 3, 0, 1 << 20, s); };
  full_apply();   // every level's coefficients in place for the per-level timings
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  auto timed = [&](auto&& fn) -> double {
    fn();
    HIPCHK(hipEventRecord(e0, s));
    for (int r = 0; r < reps; ++r) fn();
    HIPCHK(hipEventRecord(e1, s));
    HIPCHK(hipEventSynchronize(e1));
    float ms = 0.0f;
    HIPCHK(hipEventElapsedTime(&ms, e0, e1));
    return (double)ms / reps;
  };
  const bool f32 = Prec<T>::f32;
  if (p->opt.prop_kernel == IFGF_PROP_AUTO) {
    int nl = 0;
    for (int d = D; d >= 4; --d) {   // child level d into parent level d - 1
      LevelPlan& lp = p->lev[d - 1];
      if (lp.nrel == 0 || lp.nwork == 0) continue;
      const bool cone = cone_major_order(PS, PA) && cone_prop_supported(p) && lp.ti_allowed;
      const bool pairs = up_pairs_possible(p, d - 1);
      static const int kNw[4] = {0, 1, 2, 4};
      int best = -1;
      lp.up_use = false;
      for (int c = 0; c < 4; ++c) {
        rep->ms[nl][c] = -1.0;
        if (c > 0 && (!cone || (!f32 && kNw[c] > 2))) continue;
        build_cone_tiles(p, d - 1, kNw[c], s);
        rep->ms[nl][c] = timed([&]() { prop_level<T, PS, PA>(p, d, 1, s); });
        if (best < 0 || rep->ms[nl][c] < rep->ms[nl][best]) best = c;
      }
      rep->ms[nl][4] = -1.0;
      if (pairs) {   // the pair list (built here if the plan has none)
        build_cone_tiles(p, d - 1, 0, s);
        if (lp.nup == 0) build_up_pairs(p, d - 1, s);
        lp.up_use = lp.nup > 0;
        if (lp.up_use) {
          rep->ms[nl][4] = timed([&]() { prop_level<T, PS, PA>(p, d, 1, s); });
          if (rep->ms[nl][4] < rep->ms[nl][best]) best = 4;
        }
      }
      lp.up_use = best == 4;
      // tiles won: their gathered transposed pass serves the adjoint too; the
      // node formulation won: the list stays for the adjoint's gather
      if (best >= 1 && best <= 3 && lp.nup > 0) release_up_pairs(lp);
      build_cone_tiles(p, d - 1, best == 4 ? 0 : kNw[best], s);
      rep->parent_level[nl] = d - 1;
      rep->choice[nl] = best == 4 ? 1 : 8 * kNw[best];
      ++nl;
    }
    rep->nlevels = nl;
  }
  rep->target_ms[0] = rep->target_ms[1] = rep->target_ms[2] = -1.0;
  if constexpr (rows_ok<T, PS, PA>()) {
    if (p->opt.target_kernel == IFGF_TARGET_AUTO && p->tpart.bytes > 0) {
      static const int kT[3] = {IFGF_TARGET_ROWS, IFGF_TARGET_WAVE, IFGF_TARGET_PAIRS};
      int best = -1;
      for (int c = 0; c < 3; ++c) {
        if (kT[c] == IFGF_TARGET_PAIRS && !p->pairs) continue;
        p->opt.target_kernel = kT[c];
        rep->target_ms[c] = timed(full_apply);
        if (best < 0 || rep->target_ms[c] < rep->target_ms[best]) best = c;
      }
      p->opt.target_kernel = kT[best];
      rep->target_choice = kT[best];
      if (kT[best] != IFGF_TARGET_PAIRS && p->pairs) release_target_pairs(p);
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  HIPCHK(hipStreamSynchronize(s));   // sig and out are freed on return
}

template <typename T>
void dispatch_autotune(ifgf_plan_s* p, int reps, ifgf_tune_report* rep, hipStream_t s) {
  const int ps = p->opt.p_s, pa = p->opt.p_ang;
#define X(a, b) \
  if (ps == a && pa == b) return autotune_impl<T, a, b>(p, reps, rep, s);
  IFGF_ORDERS_ALL(X)
  if constexpr (!Prec<T>::f32) {
    IFGF_ORDERS_FP64(X)
  }
#undef X
  throw Error{IFGF_EUNSUPPORTED, "interpolation order not compiled"};
}

template <int PS, int PA>
void ti_geo_impl(ifgf_plan_s* p, int d, const std::vector<int>& qlist, hipStream_t s) {
  LevelPlan& lp = p->lev[d];
  const LevelPlan& lc = p->lev[d + 1];
  DevBuf qd;
  qd.alloc(sizeof(int) * qlist.size());
  HIPCHK(hipMemcpyAsync(qd.p, qlist.data(), sizeof(int) * qlist.size(), hipMemcpyHostToDevice, s));
  const unsigned grid = (unsigned)(8 * qlist.size());
  if (p->opt.precision == IFGF_PREC_FP32_INTERP) {
    lp.ti_geo.alloc(sizeof(TiGeo<PS, PA>) * 8 * qlist.size());
    k_ti_geo<PS, PA><<<grid, 256, 0, s>>>(qd.as<int>(), lp.geom, lc.geom, p->cheb, p->k, p->opt.kernel,
                                          lp.ti_geo.as<TiGeo<PS, PA>>());
  } else {
    lp.ti_geo.alloc(sizeof(TiGeo64<PS, PA>) * 8 * qlist.size());
    k_ti_geo64<PS, PA><<<grid, 256, 0, s>>>(qd.as<int>(), lp.geom, lc.geom, p->cheb, p->k, p->opt.kernel,
                                            lp.ti_geo.as<TiGeo64<PS, PA>>());
  }
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s));   // qd is freed on return
}

}  // namespace

size_t ti_geo_bytes(int ps, int pa, bool f32) {
  if (ps == 3 && pa == 5) return f32 ? sizeof(TiGeo<3, 5>) : sizeof(TiGeo64<3, 5>);
  if (ps == 4 && pa == 6) return f32 ? sizeof(TiGeo<4, 6>) : sizeof(TiGeo64<4, 6>);
  return 0;
}

void build_ti_geo(ifgf_plan_s* p, int d, const std::vector<int>& qlist, hipStream_t s) {
  if (qlist.empty()) return;
  const int ps = p->opt.p_s, pa = p->opt.p_ang;
  if (ps == 3 && pa == 5) return ti_geo_impl<3, 5>(p, d, qlist, s);
  if (ps == 4 && pa == 6) return ti_geo_impl<4, 6>(p, d, qlist, s);
  throw Error{IFGF_EUNSUPPORTED, "interpolation order not compiled"};
}

int prop_chunk(int P) {
  if (P == 75) return PropShape<75>::CH;
  if (P == 144) return PropShape<144>::CH;
  if (P == 512) return PropShape<512>::CH;
  return 1;
}

static bool order_in_all(int ps, int pa) {
#define X(a, b) \
  if (ps == a && pa == b) return true;
  IFGF_ORDERS_ALL(X)
#undef X
  return false;
}

bool supported_order(int ps, int pa, int precision) {
  if (order_in_all(ps, pa)) return true;
  if (precision != IFGF_PREC_FP64) return false;
#define X(a, b) \
  if (ps == a && pa == b) return true;
  IFGF_ORDERS_FP64(X)
#undef X
  return false;
}

bool cone_prop_supported(const ifgf_plan_s* p) {
  return p->opt.p_s <= 4 && p->opt.prop_kernel != IFGF_PROP_NODE && order_in_all(p->opt.p_s, p->opt.p_ang);
}

template <typename T>
void build_target_pairs_impl(ifgf_plan_s* p, hipStream_t s) {
  using V4 = typename Vec4<T>::type;
  const int64_t n = p->n;
  // RHS groups of 16 (FP32, P_s <= 4): the value list holds 16 values per pair
  p->pairs_rg = Prec<T>::f32 && p->opt.max_rhs >= MF_RG && p->opt.p_s <= 4;
  DevBuf cnt;
  cnt.alloc(sizeof(int) * (n + 1));
  for (int d = 3; d <= p->D; ++d) {
    LevelPlan& lv = p->lev[d];
    lv.pr_off.alloc(sizeof(int) * (n + 1));
    k_pair_count<<<nblocks(n), TPB, 0, s>>>(lv.pbox.as<int>(), lv.cou_off.as<int>(), n, cnt.as<int>());
    HIPCHK(hipGetLastError());
    scan_exclusive_i32(cnt.as<int>(), lv.pr_off.as<int>(), n, s);
    int np32 = 0;   // the list's length: the scan's total
    HIPCHK(hipMemcpyAsync(&np32, lv.pr_off.as<int>() + n, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    const int64_t np = np32;
    lv.npair = np;
    const size_t npa = (size_t)std::max<int64_t>(1, np);
    lv.pr_slot.alloc(sizeof(int) * npa);
    lv.pr_loc.alloc(sizeof(V4) * npa);
    lv.pr_fim.alloc(sizeof(T) * npa);
    lv.pr_val.alloc(sizeof(cpx<T>) * npa * (p->pairs_rg ? MF_RG : 1));
    lv.pr_pos.alloc(sizeof(int) * npa);
    if (np == 0) continue;
    DevBuf keys, tloc, tfim;
    keys.alloc(sizeof(uint64_t) * sort_padded_length(np));
    tloc.alloc(sizeof(V4) * npa);
    tfim.alloc(sizeof(T) * npa);
    TLevel<T> tl{gas(lv.pbox.as<const int>()), gas(lv.cou_off.as<const int>()), gas(lv.cou.as<const int>()),
                 gas(lv.centre.as<const double>()), gas(lv.slot.as<const int>()), gas(lv.Fc.as<const cpx<T>>()),
                 lv.geom};
    k_pair_gen<T><<<nblocks(n), TPB, 0, s>>>(p->pts.as<double>(), n, tl, lv.pr_off.as<int>(), p->k, p->opt.kernel,
                                            keys.as<uint64_t>(), tloc.as<V4>(), tfim.as<T>(), p->err.as<int>());
    HIPCHK(hipGetLastError());
    sort_u64(keys.as<uint64_t>(), np, s);
    k_pair_place<T><<<nblocks(np), TPB, 0, s>>>(keys.as<uint64_t>(), np, tloc.as<V4>(), tfim.as<T>(),
                                               lv.pr_slot.as<int>(), lv.pr_loc.as<V4>(), lv.pr_fim.as<T>(),
                                               lv.pr_pos.as<int>());
    HIPCHK(hipGetLastError());
    {   // row-stage passes, for the statistics
      DevBuf acc;
      acc.alloc(sizeof(unsigned long long));
      HIPCHK(hipMemsetAsync(acc.p, 0, sizeof(unsigned long long), s));   // plan time
      const int64_t nrow = (np + 15) / 16;
      k_pair_rows<<<nblocks(nrow), TPB, 0, s>>>(lv.pr_slot.as<int>(), np, acc.as<unsigned long long>());
      HIPCHK(hipGetLastError());
      unsigned long long h = 0;
      HIPCHK(hipMemcpyAsync(&h, acc.p, sizeof(h), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      lv.pair_rows = nrow;
      lv.pair_row_cones = (int64_t)h;
    }
    HIPCHK(hipStreamSynchronize(s));   // the temporaries are freed on return
  }
  p->pairs = true;
}

template <typename T>
bool pairs_compiled(int ps, int pa) {
#define X(a, b) \
  if (ps == a && pa == b) return rows_ok<T, a, b>();
  IFGF_ORDERS_ALL(X)
  if constexpr (!Prec<T>::f32) {
    IFGF_ORDERS_FP64(X)
  }
#undef X
  return false;
}

void release_target_pairs(ifgf_plan_s* p) {
  for (int d = 0; d < IFGF_MAX_LEVELS; ++d) {
    LevelPlan& lv = p->lev[d];
    lv.npair = 0;
    lv.pr_slot.release();
    lv.pr_loc.release();
    lv.pr_fim.release();
    lv.pr_val.release();
    lv.pr_off.release();
    lv.pr_pos.release();
    lv.pr_tgt.release();
    lv.pr_run.release();
    lv.nrun = 0;
    lv.pair_rows = lv.pair_row_cones = 0;
  }
  p->pairs = false;
  p->adj_pairs = false;
  p->pairs_rg = false;
}

// Pair lists are built where the order has a row stage, one RHS is possible
// and the lists stay within 2^28 pairs (about 10 GB in FP32).
void build_target_pairs(ifgf_plan_s* p, hipStream_t s) {
  const bool f32 = p->opt.precision == IFGF_PREC_FP32_INTERP;
  if (p->D < 3) return;
  if (p->opt.target_kernel != IFGF_TARGET_AUTO && p->opt.target_kernel != IFGF_TARGET_PAIRS) return;
  if (!(f32 ? pairs_compiled<float>(p->opt.p_s, p->opt.p_ang) : pairs_compiled<double>(p->opt.p_s, p->opt.p_ang)))
    return;
  int64_t tot = 0;
  for (int d = 3; d <= p->D; ++d) tot += p->lev[d].cousin_pairs;
  if (tot > ((int64_t)1 << 28)) return;
  try {   // where the device memory runs out the plan keeps the row targets
    if (f32)
      build_target_pairs_impl<float>(p, s);
    else
      build_target_pairs_impl<double>(p, s);
  } catch (const Error& e) {
    if (e.st != IFGF_ENOMEM) throw;
    HIPCHK(hipStreamSynchronize(s));   // the lists' generators are done before they are freed
    release_target_pairs(p);
  }
}

void release_up_pairs(LevelPlan& lv) {
  lv.nup = 0;
  lv.up_use = false;
  lv.up_nrun = 0;
  lv.up_slot.release();
  lv.up_loc.release();
  lv.up_fim.release();
  lv.up_val.release();
  lv.up_base.release();
  lv.up_pos.release();
  lv.up_node.release();
  lv.up_run.release();
}

// Upward pairs of the pass d+1 -> d: located, keyed by child slot, sorted.
template <typename T, int PS, int PA>
void build_up_pairs_impl(ifgf_plan_s* p, int d, hipStream_t s) {
  using V4 = typename Vec4<T>::type;
  constexpr int P = PS * PA * PA;
  LevelPlan& lp = p->lev[d];
  const LevelPlan& lc = p->lev[d + 1];
  release_up_pairs(lp);
  const int64_t np = lc.prop_evals;   // sum over the relevant cones of P x children
  if (lp.nrel == 0 || np == 0) return;
  lp.up_base.alloc(sizeof(int) * ((int64_t)lp.nrel + 1));
  {
    DevBuf cnt;
    cnt.alloc(sizeof(int) * ((int64_t)lp.nrel + 1));
    k_upair_count<<<nblocks(lp.nrel), TPB, 0, s>>>(lp.nrel, lp.rel_box.as<int>(), lp.child_lo.as<int>(), P,
                                                   cnt.as<int>());
    HIPCHK(hipGetLastError());
    scan_exclusive_i32(cnt.as<int>(), lp.up_base.as<int>(), lp.nrel, s);
    int tot = 0;
    HIPCHK(hipMemcpyAsync(&tot, lp.up_base.as<int>() + lp.nrel, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (tot != np) throw Error{IFGF_EUNSUPPORTED, "internal error: upward pair count"};
  }
  lp.up_slot.alloc(sizeof(int) * np);
  lp.up_loc.alloc(sizeof(V4) * np);
  lp.up_fim.alloc(sizeof(T) * np);
  lp.up_val.alloc(sizeof(cpx<T>) * np);
  lp.up_pos.alloc(sizeof(int) * np);
  DevBuf keys, tloc, tfim;
  keys.alloc(sizeof(uint64_t) * sort_padded_length(np));
  tloc.alloc(sizeof(V4) * np);
  tfim.alloc(sizeof(T) * np);
  const int64_t nn = (int64_t)lp.nrel * P;
  k_upair_gen<T, PS, PA><<<nblocks(nn), TPB, 0, s>>>(
      lp.nrel, lp.rel_box.as<int>(), lp.rel_cone.as<int>(), lp.child_lo.as<int>(), lc.coords.as<int>(),
      lc.slot.as<int>(), lp.up_base.as<int>(), lp.geom, lc.geom, p->cheb, p->k, p->opt.kernel, keys.as<uint64_t>(),
      tloc.as<V4>(), tfim.as<T>(), p->err.as<int>());
  HIPCHK(hipGetLastError());
  sort_u64(keys.as<uint64_t>(), np, s);
  k_pair_place<T><<<nblocks(np), TPB, 0, s>>>(keys.as<uint64_t>(), np, tloc.as<V4>(), tfim.as<T>(),
                                             lp.up_slot.as<int>(), lp.up_loc.as<V4>(), lp.up_fim.as<T>(),
                                             lp.up_pos.as<int>());
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s));   // the temporaries are freed on return
  lp.nup = np;
}

template <typename T>
void dispatch_up_pairs(ifgf_plan_s* p, int d, hipStream_t s) {
  const int ps = p->opt.p_s, pa = p->opt.p_ang;
#define X(a, b) \
  if (ps == a && pa == b) { if constexpr (rows_ok<T, a, b>()) build_up_pairs_impl<T, a, b>(p, d, s); return; }
  IFGF_ORDERS_ALL(X)
  if constexpr (!Prec<T>::f32) {
    IFGF_ORDERS_FP64(X)
  }
#undef X
}

// Whether level d's pass d+1 -> d can run from a pair list: an order with a
// row stage and at most 2^28 pairs (about 9 GB in FP32).
bool up_pairs_possible(const ifgf_plan_s* p, int d) {
  if (d < 3 || d >= p->D || p->lev[d].nrel == 0) return false;
  const bool f32 = p->opt.precision == IFGF_PREC_FP32_INTERP;
  if (!(f32 ? pairs_compiled<float>(p->opt.p_s, p->opt.p_ang) : pairs_compiled<double>(p->opt.p_s, p->opt.p_ang)))
    return false;
  const int64_t np = p->lev[d + 1].prop_evals;
  return np > 0 && np <= ((int64_t)1 << 28);
}

// Where the device memory runs out the level keeps the node formulation.
void build_up_pairs(ifgf_plan_s* p, int d, hipStream_t s) {
  try {
    if (p->opt.precision == IFGF_PREC_FP32_INTERP)
      dispatch_up_pairs<float>(p, d, s);
    else
      dispatch_up_pairs<double>(p, d, s);
  } catch (const Error& e) {
    if (e.st != IFGF_ENOMEM) throw;
    HIPCHK(hipStreamSynchronize(s));   // nothing in flight reads the list before it is freed
    release_up_pairs(p->lev[d]);
  }
}

// At plan creation: PAIRS takes the lists wherever possible; AUTO where the
// level has no cone-major tiles (the sparse levels); NODE and CONE never.
void build_plan_up_pairs(ifgf_plan_s* p, hipStream_t s) {
  const int pk = p->opt.prop_kernel;
  if (pk != IFGF_PROP_AUTO && pk != IFGF_PROP_PAIRS) return;
  for (int d = 3; d < p->D; ++d) {
    LevelPlan& lv = p->lev[d];
    if (!up_pairs_possible(p, d)) continue;
    if (pk == IFGF_PROP_AUTO && lv.ntile > 0) continue;
    build_up_pairs(p, d, s);
    lv.up_use = lv.nup > 0;
  }
}

template <typename T>
void dispatch_export_nodes(ifgf_plan_s* p, void* dst, hipStream_t s) {
  const int ps = p->opt.p_s, pa = p->opt.p_ang;
#define X(a, b) \
  if (ps == a && pa == b) return export_nodes_impl<T, a, b>(p, dst, s);
  IFGF_ORDERS_ALL(X)
  if constexpr (!Prec<T>::f32) {
    IFGF_ORDERS_FP64(X)
  }
#undef X
  throw Error{IFGF_EUNSUPPORTED, "interpolation order not compiled"};
}

void run_export_nodes(ifgf_plan_s* p, void* dst, hipStream_t s) {
  if (p->opt.precision == IFGF_PREC_FP32_INTERP)
    dispatch_export_nodes<float>(p, dst, s);
  else
    dispatch_export_nodes<double>(p, dst, s);
}

void run_apply(ifgf_plan_s* p, const void* sigma, void* u, int nrhs, int dtype, int stage_mask, int level_lo,
               int level_hi, hipStream_t s) {
  // with separate targets the apply runs over sources and targets together
  // (targets carrying zero density) and the targets' values are copied out
  void* dst = p->n_src < p->n ? p->uext.p : u;
  if (p->opt.precision == IFGF_PREC_FP32_INTERP)
    dispatch_apply<float>(p, sigma, dst, nrhs, dtype, stage_mask, level_lo, level_hi, s);
  else
    dispatch_apply<double>(p, sigma, dst, nrhs, dtype, stage_mask, level_lo, level_hi, s);
  if (p->n_src < p->n) {
    const int64_t nt = p->n - p->n_src;
    k_copy_targets<<<nblocks(nt * nrhs), TPB, 0, s>>>(dst, p->n_src, nt, nrhs, dtype, u);
    HIPCHK(hipGetLastError());
  }
  p->last_rhs = nrhs;
}

void run_far_field(ifgf_plan_s* p, const void* sigma, int64_t ndir, const double* dirs, void* uinf, int dtype,
                   hipStream_t s) {
  if (p->opt.precision == IFGF_PREC_FP32_INTERP)
    dispatch_far_field<float>(p, sigma, ndir, dirs, uinf, dtype, s);
  else
    dispatch_far_field<double>(p, sigma, ndir, dirs, uinf, dtype, s);
  p->last_rhs = 1;
}

void run_autotune(ifgf_plan_s* p, int reps, ifgf_tune_report* rep, hipStream_t s) {
  if (p->opt.precision == IFGF_PREC_FP32_INTERP)
    dispatch_autotune<float>(p, reps, rep, s);
  else
    dispatch_autotune<double>(p, reps, rep, s);
  p->last_rhs = 1;
}

void run_adjoint(ifgf_plan_s* p, const void* v, void* out, int nrhs, int dtype, int conj, hipStream_t s) {
  if (p->opt.precision == IFGF_PREC_FP32_INTERP)
    dispatch_adjoint<float>(p, v, out, nrhs, dtype, conj, s);
  else
    dispatch_adjoint<double>(p, v, out, nrhs, dtype, conj, s);
}

void run_batch_prepare(ifgf_batch_s* b) {
  ifgf_plan_s* p = b->plans[0];
  const bool f32 = p->opt.precision == IFGF_PREC_FP32_INTERP;
  const int ps = p->opt.p_s, pa = p->opt.p_ang;
  if (!order_in_all(ps, pa)) throw Error{IFGF_EUNSUPPORTED, "the ragged batch is not compiled for this order"};
  if (ps == 3 && pa == 5) return f32 ? batch_prepare_impl<float, 3, 5>(b) : batch_prepare_impl<double, 3, 5>(b);
  if (ps == 4 && pa == 6) return f32 ? batch_prepare_impl<float, 4, 6>(b) : batch_prepare_impl<double, 4, 6>(b);
  throw Error{IFGF_EUNSUPPORTED, "interpolation order not compiled"};
}

void run_batch_apply(ifgf_batch_s* b, const void* const* sigma, void* const* u, int dtype, int* ctr, hipStream_t s) {
  ifgf_plan_s* p = b->plans[0];
  const bool f32 = p->opt.precision == IFGF_PREC_FP32_INTERP;
  const int ps = p->opt.p_s, pa = p->opt.p_ang;
  if (!ctr) ctr = b->ctr.as<int>();
  if (ps == 3 && pa == 5)
    return f32 ? batch_apply_impl<float, 3, 5>(b, sigma, u, dtype, ctr, s)
               : batch_apply_impl<double, 3, 5>(b, sigma, u, dtype, ctr, s);
  if (ps == 4 && pa == 6)
    return f32 ? batch_apply_impl<float, 4, 6>(b, sigma, u, dtype, ctr, s)
               : batch_apply_impl<double, 4, 6>(b, sigma, u, dtype, ctr, s);
  throw Error{IFGF_EUNSUPPORTED, "interpolation order not compiled"};
}

// ---------------------------------------------------------------------------
// Completion counters of the allocation-free batch apply.  The launch's queue
// head and its 16 counters per geometry live in this fixed device array (one
// copy per GPU, held until the process ends) instead of the batch's own
// buffer.  Host code never names the array in a launch or a copy: its device
// address is looked up once per device, with that device current, and that
// address is what the kernels receive.
// ---------------------------------------------------------------------------
static __device__ __align__(256) int scratch[BATCH_STATIC_COUNTERS];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
int* g_scratch_addr[kMaxDevices] = {};
}  // namespace

int* batch_static_counters(int device) {
  if (device < 0 || device >= kMaxDevices) throw Error{IFGF_EINVAL, "device ordinal out of range"};
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_addr[device]) {
    int cur = -1;
    HIPCHK(hipGetDevice(&cur));
    if (cur != device) throw Error{IFGF_EINVAL, "the counters' device is not the current device"};
    void* ptr = nullptr;
    HIPCHK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) throw Error{IFGF_EHIP, "no device address for the static counters"};
    g_scratch_addr[device] = (int*)ptr;
  }
  return g_scratch_addr[device];
}

}  // namespace ifgf
