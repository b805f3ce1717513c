// Internal device/host helpers of the IFGF library (gfx950).
//
// Geometry conventions (paper Section 3):
//   * box B(y0, H) is half-open (eq. box); h = sqrt(3) H / 2 and s = h / r
//     with r = |x - y0| (eq. def_eps); every interpolation point has
//     s <= sqrt(3)/3 (eq. s_rest);
//   * x(s, theta, phi; y0) = y0 + (h/s)(sin th cos ph, sin th sin ph, cos th)
//     (eqs. defparametrizationins, defparametrizationr);
//   * cone segment gamma = (i_s, i_th, i_ph) of a box with n_s x n_C x 2n_C
//     segments, ds = sqrt(3)/3 / n_s, dth = dph = pi / n_C (eqs. deltas,
//     ConeIntervals); its id is (i_s * n_C + i_th) * 2 n_C + i_ph, i.e. the
//     radial index is the slowest and the azimuthal the fastest;
//   * indices are floor(value / interval) clamped to the last interval, so
//     the closed upper ends s = sqrt(3)/3, theta = pi, phi -> 2 pi belong to
//     the last segment;
//   * interpolation nodes are tensor products of first-kind Chebyshev points
//     cos((2k+1) pi / (2n)) mapped affinely to each interval (eq.
//     ChebyNodes); local coordinates t in [-1, 1].
//
// The same locate function is used when relevant cones are marked at plan
// time and when they are looked up at apply time, with floating-point
// contraction disabled inside it, so both compute bit-identical cone ids.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define IFGF_MAXP 16        // max points per interpolation axis
#define IFGF_PI 3.14159265358979323846
#define IFGF_TWO_PI 6.28318530717958647692

template <typename T> struct cpx { T re, im; };

template <typename T> __host__ __device__ __forceinline__ cpx<T> cmul(cpx<T> a, cpx<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}

// Per-level cone-segment geometry, passed to kernels by value.
struct LevelGeom {
  double H;          // box side
  double h;          // sqrt(3)/2 * H
  float hf;          // h in FP32
  int ns, nc;        // n_s, n_C
  int ncone;         // n_s * n_C * 2 n_C
  double ds, da;     // sqrt(3)/3 / n_s, pi / n_C
  double inv_ds, inv_da;
  float dsf, daf, inv_dsf, inv_daf;
};

// Chebyshev node offsets u_k = (1 + x_k) / 2 in [0, 1] per axis, and the
// node-value -> coefficient matrices (row i: (2 - delta_i0)/n T_i(x_k)).
struct ChebTab {
  int ps, pa;
  double us[IFGF_MAXP], ua[IFGF_MAXP];
  float usf[IFGF_MAXP], uaf[IFGF_MAXP];
};

struct Loc {
  int cid;
  double ts, tt, tp;   // local coordinates in [-1, 1]
};
struct LocF {
  int cid;
  float ts, tt, tp;
};

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// ---------------------------------------------------------------------------
// Cone location, FP64: relative vector d = x - y0 and s = h / |d|.
// ---------------------------------------------------------------------------
__device__ __forceinline__ Loc locate64(double dx, double dy, double dz, double s, const LevelGeom& g) {
#pragma clang fp contract(off)
  Loc L;
  double rho = sqrt(dx * dx + dy * dy);
  double th = atan2(rho, dz);
  double ph = atan2(dy, dx);
  if (ph < 0.0) ph += IFGF_TWO_PI;
  double us = s / g.ds, ut = th / g.da, up = ph / g.da;   // correctly rounded quotients
  int is = clampi((int)floor(us), 0, g.ns - 1);
  int it = clampi((int)floor(ut), 0, g.nc - 1);
  int ip = clampi((int)floor(up), 0, 2 * g.nc - 1);
  L.cid = (is * g.nc + it) * (2 * g.nc) + ip;
  L.ts = 2.0 * (us - is) - 1.0;
  L.tt = 2.0 * (ut - it) - 1.0;
  L.tp = 2.0 * (up - ip) - 1.0;
  return L;
}

// FP32 helpers of the FP32-interpolation mode: hardware reciprocal and
// square root (about 1 ulp) and a polynomial atan2.  The atan kernel is an
// odd polynomial fitted by least squares on |t| <= tan(pi/8) (max error
// 4.4e-8 rad); larger ratios are folded with atan(t) = pi/4 + atan((t-1)/(t+1))
// and the octant symmetries.  Used identically at plan and apply time.
__device__ __forceinline__ float rcp_f(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float sqrt_f(float x) { return __builtin_amdgcn_sqrtf(x); }

__device__ __forceinline__ float atan2_f(float y, float x) {
#pragma clang fp contract(off)
  const float ax = fabsf(x), ay = fabsf(y);
  const float mx = fmaxf(ax, ay), mn = fminf(ax, ay);
  if (mx == 0.0f) return 0.0f;
  const float t = mn * rcp_f(mx);
  const bool big = t > 0.41421356f;
  const float u = big ? (t - 1.0f) * rcp_f(t + 1.0f) : t;
  const float u2 = u * u;
  float q = fmaf(u2, 0.0772617757f, -0.1375157684f);
  q = fmaf(u2, q, 0.1996154934f);
  q = fmaf(u2, q, -0.3333218396f);
  q = fmaf(u2, q, 0.9999998808f);
  float r = u * q;
  if (big) r += 0.785398163f;
  if (ay > ax) r = 1.570796327f - r;
  if (x < 0.0f) r = 3.141592654f - r;
  return y < 0.0f ? -r : r;
}

// sin and cos in FP32 from the hardware sine and cosine, whose argument is
// in revolutions.  The rounding of x / (2 pi) in FP32 dominates: the
// absolute error measured on gfx950 is about 1.5e-7 + 8.7e-8 |x| (3.9e-7 for
// |x| <= 4, 1.4e-6 for |x| <= 16).  For phases of a few radians only.
__device__ __forceinline__ void sincos_hw(float x, float* sn, float* cs) {
  const float rv = x * 0.159154943f;
  *sn = __builtin_amdgcn_sinf(rv);
  *cs = __builtin_amdgcn_cosf(rv);
}

// sin and cos in FP64 for |x| <= 2^20: quadrant q = rint(2x/pi), remainder
// r = x - q pi/2 by a two-term Cody-Waite reduction with FMAs (pi/2 = HI +
// LO, HI the double nearest pi/2), then the Taylor series of sin and cos on
// |r| <= pi/4 through r^15 and r^16 (truncation below 5e-17), and the
// quadrant's signs and swap.  Within about 2 ulp of sin and cos; larger |x|
// go to the library sincos.
__device__ __forceinline__ void sincos_cw64(double x, double* sn, double* cs) {
  if (!(fabs(x) <= 1048576.0)) {
    sincos(x, sn, cs);
    return;
  }
  constexpr double PIO2_HI = 1.5707963267948966;       // nearest double to pi/2
  constexpr double PIO2_LO = 6.123233995736766e-17;    // pi/2 - PIO2_HI
  constexpr double TWO_OVER_PI = 0.6366197723675814;
  const double q = rint(x * TWO_OVER_PI);
  double r = fma(-q, PIO2_HI, x);
  r = fma(-q, PIO2_LO, r);
  const double r2 = r * r;
  // 1/n! for the Taylor terms
  constexpr double F2 = 1.0 / 2, F3 = F2 / 3, F4 = F3 / 4, F5 = F4 / 5, F6 = F5 / 6, F7 = F6 / 7, F8 = F7 / 8,
                   F9 = F8 / 9, F10 = F9 / 10, F11 = F10 / 11, F12 = F11 / 12, F13 = F12 / 13, F14 = F13 / 14,
                   F15 = F14 / 15, F16 = F15 / 16;
  double ps = fma(r2, -F15, F13);
  ps = fma(r2, ps, -F11);
  ps = fma(r2, ps, F9);
  ps = fma(r2, ps, -F7);
  ps = fma(r2, ps, F5);
  ps = fma(r2, ps, -F3);
  const double s_r = fma(r * r2, ps, r);
  double pc = fma(r2, F16, -F14);
  pc = fma(r2, pc, F12);
  pc = fma(r2, pc, -F10);
  pc = fma(r2, pc, F8);
  pc = fma(r2, pc, -F6);
  pc = fma(r2, pc, F4);
  const double c_r = fma(r2 * r2, pc, fma(r2, -F2, 1.0));
  const int n = (int)q & 3;
  const double a = (n & 1) ? c_r : s_r, b = (n & 1) ? s_r : c_r;
  *sn = (n & 2) ? -a : a;
  *cs = ((n + 1) & 2) ? -b : b;
}

// FP64 1/sqrt(x) and sqrt(x) for positive normal x: the hardware estimate
// refined by two Newton-Raphson steps y <- y + y (1 - x y^2) / 2, then
// sqrt(x) = x y corrected once by its residual x - (x y)^2.
__device__ __forceinline__ void sqrt_rsqrt_nr64(double x, double* sq, double* rs) {
  double y = __builtin_amdgcn_rsq(x);
  double e = fma(-(x * y), y, 1.0);
  y = fma(0.5 * y, e, y);
  e = fma(-(x * y), y, 1.0);
  y = fma(0.5 * y, e, y);
  double s = x * y;
  s = fma(0.5 * y, fma(-s, s, x), s);
  *rs = y;
  *sq = s;
}

// FP64 1/x for normal x: the hardware estimate refined by two Newton-Raphson
// steps y <- y + y (1 - x y).
__device__ __forceinline__ double rcp_nr64(double x) {
  double y = __builtin_amdgcn_rcp(x);
  y = fma(y, fma(-x, y, 1.0), y);
  y = fma(y, fma(-x, y, 1.0), y);
  return y;
}

// sin and cos in FP32: quadrant k = rint(2x/pi), remainder x - k pi/2 by a
// three-term Cody-Waite reduction with FMAs (pi/2 split into FP32 parts),
// then polynomials on |r| <= pi/4 whose coefficients are a least-squares fit
// (max error 6e-8 for sin, 8e-8 for cos).  Meant for |x| up to ~1e5.
__device__ __forceinline__ void sincos_f(float x, float* sn, float* cs) {
#pragma clang fp contract(off)
  const float kq = rintf(x * 0.636619772f);
  float r = fmaf(-kq, 1.57079637f, x);
  r = fmaf(-kq, -4.37113883e-08f, r);
  r = fmaf(-kq, -1.77635684e-15f, r);
  const float r2 = r * r;
  float ps = fmaf(r2, -0.000194934968f, 0.00833195820f);
  ps = fmaf(r2, ps, -0.166666508f);
  const float sr = fmaf(r * r2, ps, r);
  float pc = fmaf(r2, 2.43892027e-05f, -0.00138867483f);
  pc = fmaf(r2, pc, 0.0416666232f);
  pc = fmaf(r2, pc, -0.5f);
  const float cr = fmaf(r2, pc, 1.0f);
  const int q = ((int)kq) & 3;
  const float s0 = (q & 1) ? cr : sr;
  const float c0 = (q & 1) ? sr : cr;
  *sn = (q & 2) ? -s0 : s0;
  *cs = ((q + 1) & 2) ? -c0 : c0;
}

// Cone location, FP32 (used by the FP32-interpolation precision mode).
__device__ __forceinline__ LocF locate32(float dx, float dy, float dz, float s, const LevelGeom& g) {
#pragma clang fp contract(off)
  LocF L;
  float rho = sqrt_f(dx * dx + dy * dy);
  float th = atan2_f(rho, dz);
  float ph = atan2_f(dy, dx);
  if (ph < 0.0f) ph += (float)IFGF_TWO_PI;
  float us = s * g.inv_dsf, ut = th * g.inv_daf, up = ph * g.inv_daf;
  int is = clampi((int)floorf(us), 0, g.ns - 1);
  int it = clampi((int)floorf(ut), 0, g.nc - 1);
  int ip = clampi((int)floorf(up), 0, 2 * g.nc - 1);
  L.cid = (is * g.nc + it) * (2 * g.nc) + ip;
  L.ts = 2.0f * (us - (float)is) - 1.0f;
  L.tt = 2.0f * (ut - (float)it) - 1.0f;
  L.tp = 2.0f * (up - (float)ip) - 1.0f;
  return L;
}

// ---------------------------------------------------------------------------
// A surface point x about a box centre c (cousin-target interpolation and
// the marking of cousin points).  Returns the location and r = |x - c| in
// FP64.
// ---------------------------------------------------------------------------
__device__ __forceinline__ Loc target_loc64(const double* x, const double* c, const LevelGeom& g, double* r_out) {
#pragma clang fp contract(off)
  double dx = x[0] - c[0], dy = x[1] - c[1], dz = x[2] - c[2];
  double r = sqrt(dx * dx + dy * dy + dz * dz);
  *r_out = r;
  return locate64(dx, dy, dz, g.h / r, g);
}

__device__ __forceinline__ LocF target_loc32(const double* x, const double* c, const LevelGeom& g, double* r_out) {
#pragma clang fp contract(off)
  double dx = x[0] - c[0], dy = x[1] - c[1], dz = x[2] - c[2];
  double r = sqrt(dx * dx + dy * dy + dz * dz);
  *r_out = r;
  float rf = (float)r;
  return locate32((float)dx, (float)dy, (float)dz, g.hf * rcp_f(rf), g);
}

// ---------------------------------------------------------------------------
// Interpolation node of a cone: position relative to the box centre.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void cone_split(int cid, int nc, int* is, int* it, int* ip) {
  int nph = 2 * nc;
  *ip = cid % nph;
  int rest = cid / nph;
  *it = rest % nc;
  *is = rest / nc;
}

// node (a, b, c) of cone cid: unit direction e, s and r = h / s
__device__ __forceinline__ void node_dir64(int cid, int a, int b, int c, const LevelGeom& g, const ChebTab& ct,
                                           double* e, double* s_out) {
#pragma clang fp contract(off)
  int is, it, ip;
  cone_split(cid, g.nc, &is, &it, &ip);
  double s = ((double)is + ct.us[a]) * g.ds;
  double th = ((double)it + ct.ua[b]) * g.da;
  double ph = ((double)ip + ct.ua[c]) * g.da;
  double st, ctt, sp, cp;
  sincos(th, &st, &ctt);
  sincos(ph, &sp, &cp);
  e[0] = st * cp;
  e[1] = st * sp;
  e[2] = ctt;
  *s_out = s;
}

__device__ __forceinline__ void node_dir32(int cid, int a, int b, int c, const LevelGeom& g, const ChebTab& ct,
                                           float* e, float* s_out) {
#pragma clang fp contract(off)
  int is, it, ip;
  cone_split(cid, g.nc, &is, &it, &ip);
  float s = ((float)is + ct.usf[a]) * g.dsf;
  float th = ((float)it + ct.uaf[b]) * g.daf;
  float ph = ((float)ip + ct.uaf[c]) * g.daf;
  float st, ctt, sp, cp;
  sincos_f(th, &st, &ctt);
  sincos_f(ph, &sp, &cp);
  e[0] = st * cp;
  e[1] = st * sp;
  e[2] = ctt;
  *s_out = s;
}

// ---------------------------------------------------------------------------
// A parent-cone node about one of its parent's children (upward pass and
// the marking of parent nodes).  The child centre is the parent centre
// plus delta = (+-H_c/2, +-H_c/2, +-H_c/2) by octant bits (x: bit 0,
// y: bit 1, z: bit 2; bit set = upper half).  Returns the child-cone
// location, and the ratio of centred factors
//   K(x, y_child) / K(x, y_parent) = (r_p / r_c) exp(i k (r_c - r_p)),
// with r_c - r_p = (|delta|^2 - 2 <x - y_p, delta>) / (r_c + r_p), a form
// free of cancellation (Algorithm 1, the parent-node update).
// ---------------------------------------------------------------------------
struct PropF {
  LocF loc;
  float rp_over_rc;
  float dr;            // r_c - r_p
};
struct Prop64 {
  Loc loc;
  double rp_over_rc;
  double dr;
};

// Position of node (a, b, c) of parent cone pcid relative to the parent
// centre, and its distance r_p = h_p / s.
__device__ __forceinline__ void node_rel64(int pcid, int a, int b, int c, const LevelGeom& gp, const ChebTab& ct,
                                           double* x, double* rp) {
#pragma clang fp contract(off)
  double e[3], s;
  node_dir64(pcid, a, b, c, gp, ct, e, &s);
  double r = gp.h / s;
  x[0] = r * e[0];
  x[1] = r * e[1];
  x[2] = r * e[2];
  *rp = r;
}

__device__ __forceinline__ void node_rel32(int pcid, int a, int b, int c, const LevelGeom& gp, const ChebTab& ct,
                                           float* x, float* rp) {
#pragma clang fp contract(off)
  float e[3], s;
  node_dir32(pcid, a, b, c, gp, ct, e, &s);
  float r = gp.hf * rcp_f(s);
  x[0] = r * e[0];
  x[1] = r * e[1];
  x[2] = r * e[2];
  *rp = r;
}

// The node x (relative to the parent centre, |x| = rp) about the child of
// octant `oct`.
__device__ __forceinline__ Prop64 child_loc64(const double* x, double rp, int oct, const LevelGeom& gc) {
#pragma clang fp contract(off)
  double hd = 0.5 * gc.H;
  double dl[3] = {(oct & 1) ? hd : -hd, (oct & 2) ? hd : -hd, (oct & 4) ? hd : -hd};
  double x0 = x[0] - dl[0], x1 = x[1] - dl[1], x2 = x[2] - dl[2];
  double rc = sqrt(x0 * x0 + x1 * x1 + x2 * x2);
  Prop64 P;
  P.loc = locate64(x0, x1, x2, gc.h / rc, gc);
  double dd = dl[0] * dl[0] + dl[1] * dl[1] + dl[2] * dl[2];
  double xd = x[0] * dl[0] + x[1] * dl[1] + x[2] * dl[2];
  P.dr = (dd - 2.0 * xd) / (rc + rp);
  P.rp_over_rc = rp / rc;
  return P;
}

__device__ __forceinline__ PropF child_loc32(const float* x, float rp, int oct, const LevelGeom& gc) {
#pragma clang fp contract(off)
  float hd = (float)(0.5 * gc.H);
  float dl[3] = {(oct & 1) ? hd : -hd, (oct & 2) ? hd : -hd, (oct & 4) ? hd : -hd};
  float x0 = x[0] - dl[0], x1 = x[1] - dl[1], x2 = x[2] - dl[2];
  float rc = sqrt_f(x0 * x0 + x1 * x1 + x2 * x2);
  float irc = rcp_f(rc);
  PropF P;
  P.loc = locate32(x0, x1, x2, gc.hf * irc, gc);
  float dd = dl[0] * dl[0] + dl[1] * dl[1] + dl[2] * dl[2];
  float xd = x[0] * dl[0] + x[1] * dl[1] + x[2] * dl[2];
  P.dr = (dd - 2.0f * xd) * rcp_f(rc + rp);
  P.rp_over_rc = rp * irc;
  return P;
}

// ---------------------------------------------------------------------------
// Chebyshev polynomials T_0..T_{n-1} at t by the three-term recurrence.
// ---------------------------------------------------------------------------
template <typename T, int N>
__device__ __forceinline__ void cheb_T(T t, T* out) {
  out[0] = (T)1;
  if (N > 1) out[1] = t;
#pragma unroll
  for (int i = 2; i < N; ++i) out[i] = (T)2 * t * out[i - 1] - out[i - 2];
}

// exp(i phase) for a possibly large FP64 phase: Cody-Waite reduction modulo
// 2 pi in FP64 with a two-term constant, then FP32 sin/cos of the remainder.
__device__ __forceinline__ void expi_reduced32(double phase, float* c, float* s) {
  const double inv2pi = 0.15915494309189533577;
  const double p_hi = 6.283185307179586232;        // nearest double to 2 pi
  const double p_lo = 2.4492935982947064e-16;      // 2 pi - p_hi
  double nq = rint(phase * inv2pi);
  double red = fma(-nq, p_hi, phase);
  red = fma(-nq, p_lo, red);
  sincos_f((float)red, s, c);
}

// ---------------------------------------------------------------------------
// Morton keys: bit b of ix -> 3b, iy -> 3b + 1, iz -> 3b + 2.
// ---------------------------------------------------------------------------
__host__ __device__ __forceinline__ uint32_t spread3(uint32_t v) {
  v &= 0x3ffu;
  v = (v | (v << 16)) & 0x030000FFu;
  v = (v | (v << 8)) & 0x0300F00Fu;
  v = (v | (v << 4)) & 0x030C30C3u;
  v = (v | (v << 2)) & 0x09249249u;
  return v;
}
__host__ __device__ __forceinline__ uint32_t compact3(uint32_t v) {
  v &= 0x09249249u;
  v = (v | (v >> 2)) & 0x030C30C3u;
  v = (v | (v >> 4)) & 0x0300F00Fu;
  v = (v | (v >> 8)) & 0x030000FFu;
  v = (v | (v >> 16)) & 0x000003FFu;
  return v;
}
__host__ __device__ __forceinline__ uint32_t morton_encode(uint32_t x, uint32_t y, uint32_t z) {
  return spread3(x) | (spread3(y) << 1) | (spread3(z) << 2);
}
__host__ __device__ __forceinline__ void morton_decode(uint32_t key, int* x, int* y, int* z) {
  *x = (int)compact3(key);
  *y = (int)compact3(key >> 1);
  *z = (int)compact3(key >> 2);
}

// Pointers to global memory held in device-side structs.  A pointer loaded
// from memory is otherwise of unknown address space, and its accesses become
// flat instructions (64-bit VGPR addresses, waits shared with LDS); typed
// global pointers keep global instructions with scalar bases.
#define IFGF_GAS __attribute__((address_space(1)))
template <typename T> __host__ __device__ inline T IFGF_GAS* gas(T* p) { return (T IFGF_GAS*)p; }
template <typename T> __device__ __forceinline__ T* gen(T IFGF_GAS* p) { return (T*)p; }

// Wave-level helpers (wave64).
__device__ __forceinline__ int first_lane(uint64_t mask) { return __ffsll((unsigned long long)mask) - 1; }

// Workgroups of a launch are dealt to the 8 XCDs round-robin (block b to XCD
// b mod 8), and each XCD has its own L2.  xcd_block(b, G) maps the block index
// to a work index so that the blocks of one XCD take one contiguous range of
// the G work items: neighbouring items (the same parent box, nearby targets in
// Morton order) then share that XCD's L2.  A bijection of [0, G).
__device__ __forceinline__ int xcd_block(int b, int G) {
  constexpr int NX = 8;
  const int x = b % NX, l = b / NX, q = G / NX, r = G % NX;
  return x < r ? x * (q + 1) + l : r * (q + 1) + (x - r) * q + l;
}
