// GMRES solution of the combined-field integral equation (Sec. 2.2, eq.
// CombLayIE; Sec. 5 solves it with complex GMRES):
//
//     (alpha I + A) sigma = f,   alpha = 1/2 for eq. CombLayIE, f = -u^i,
//
// with A the IFGF-accelerated discrete combined-field operator of the plan.
// Restarted GMRES(m) with classical Gram-Schmidt applied twice; the Krylov
// vectors, the inner products, norms and updates are complex FP64 whatever
// the plan's interpolation precision.  Inner products are reduced in a fixed
// order (per-block partial sums, then one block per product), so a solve is
// deterministic.  The small Hessenberg least-squares problem (Givens
// rotations, back substitution) runs on the host.
#include <cmath>
#include <complex>
#include <vector>

#include "internal.h"

namespace ifgf {
namespace {

constexpr int GTPB = 256;
constexpr int GBLK = 512;   // blocks of the partial-sum pass (fixed: deterministic order)

struct z2 {
  double re, im;
};

__device__ __forceinline__ void block_reduce2(double& re, double& im, double* sre, double* sim) {
  for (int off = 32; off > 0; off >>= 1) {
    re += __shfl_xor(re, off, 64);
    im += __shfl_xor(im, off, 64);
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) {
    sre[w] = re;
    sim[w] = im;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0, b = 0;
    for (int i = 0; i < GTPB / 64; ++i) {
      a += sre[i];
      b += sim[i];
    }
    re = a;
    im = b;
  }
  __syncthreads();
}

// part[b * nv + i] = sum over this block's share of t of conj(V_i[t]) w[t],
// i < nv (V row-major: vector i at V + i * ld).
__global__ __launch_bounds__(GTPB) void k_mdot_part(const z2* __restrict__ V, int64_t ld, int nv,
                                                    const z2* __restrict__ w, int64_t n, z2* __restrict__ part) {
  __shared__ double sre[GTPB / 64], sim[GTPB / 64];
  for (int i = 0; i < nv; ++i) {
    const z2* v = V + (int64_t)i * ld;
    double re = 0, im = 0;
    for (int64_t t = (int64_t)blockIdx.x * GTPB + threadIdx.x; t < n; t += (int64_t)gridDim.x * GTPB) {
      const z2 a = v[t], b = w[t];
      re += a.re * b.re + a.im * b.im;
      im += a.re * b.im - a.im * b.re;
    }
    block_reduce2(re, im, sre, sim);
    if (threadIdx.x == 0) part[(int64_t)blockIdx.x * nv + i] = {re, im};
  }
}

// out[i] = sum over the blocks b (ascending) of part[b * nv + i].
__global__ __launch_bounds__(GTPB) void k_mdot_final(const z2* __restrict__ part, int nb, int nv,
                                                     z2* __restrict__ out) {
  __shared__ double sre[GTPB / 64], sim[GTPB / 64];
  const int i = blockIdx.x;
  double re = 0, im = 0;
  for (int b = threadIdx.x; b < nb; b += GTPB) {
    re += part[(int64_t)b * nv + i].re;
    im += part[(int64_t)b * nv + i].im;
  }
  block_reduce2(re, im, sre, sim);
  if (threadIdx.x == 0) out[i] = {re, im};
}

// w -= sum_i V_i h_i   (nv vectors)
__global__ __launch_bounds__(GTPB) void k_gs_sub(const z2* __restrict__ V, int64_t ld, int nv,
                                                 const z2* __restrict__ h, z2* __restrict__ w, int64_t n) {
  const int64_t t = (int64_t)blockIdx.x * GTPB + threadIdx.x;
  if (t >= n) return;
  z2 acc = w[t];
  for (int i = 0; i < nv; ++i) {
    const z2 v = V[(int64_t)i * ld + t], c = h[i];
    acc.re -= v.re * c.re - v.im * c.im;
    acc.im -= v.re * c.im + v.im * c.re;
  }
  w[t] = acc;
}

// x += sum_i V_i y_i
__global__ __launch_bounds__(GTPB) void k_gs_add(const z2* __restrict__ V, int64_t ld, int nv,
                                                 const z2* __restrict__ y, z2* __restrict__ x, int64_t n) {
  const int64_t t = (int64_t)blockIdx.x * GTPB + threadIdx.x;
  if (t >= n) return;
  z2 acc = x[t];
  for (int i = 0; i < nv; ++i) {
    const z2 v = V[(int64_t)i * ld + t], c = y[i];
    acc.re += v.re * c.re - v.im * c.im;
    acc.im += v.re * c.im + v.im * c.re;
  }
  x[t] = acc;
}

// w = A v (already in w) + alpha v
__global__ __launch_bounds__(GTPB) void k_add_alpha(const z2* __restrict__ v, double are, double aim,
                                                    z2* __restrict__ w, int64_t n) {
  const int64_t t = (int64_t)blockIdx.x * GTPB + threadIdx.x;
  if (t >= n) return;
  const z2 a = v[t];
  w[t].re += are * a.re - aim * a.im;
  w[t].im += are * a.im + aim * a.re;
}

// r = f - (A x (in r) + alpha x)
__global__ __launch_bounds__(GTPB) void k_residual(const z2* __restrict__ f, const z2* __restrict__ x, double are,
                                                   double aim, z2* __restrict__ r, int64_t n) {
  const int64_t t = (int64_t)blockIdx.x * GTPB + threadIdx.x;
  if (t >= n) return;
  const z2 a = x[t], ax = r[t];
  r[t] = {f[t].re - ax.re - (are * a.re - aim * a.im), f[t].im - ax.im - (are * a.im + aim * a.re)};
}

// y = s * x (s real)
__global__ __launch_bounds__(GTPB) void k_scale(const z2* __restrict__ x, double s, z2* __restrict__ y, int64_t n) {
  const int64_t t = (int64_t)blockIdx.x * GTPB + threadIdx.x;
  if (t >= n) return;
  y[t] = {s * x[t].re, s * x[t].im};
}

__global__ __launch_bounds__(GTPB) void k_zero_z(z2* __restrict__ x, int64_t n) {
  const int64_t t = (int64_t)blockIdx.x * GTPB + threadIdx.x;
  if (t < n) x[t] = {0.0, 0.0};
}

unsigned blocks_of(int64_t n) { return (unsigned)((n + GTPB - 1) / GTPB); }

struct Gmres {
  ifgf_plan_s* p;
  hipStream_t s;
  int64_t n;
  DevBuf part, dots;
  std::vector<z2> host;

  // out[0..nv) = V_i^H w on the host
  void mdot(const z2* V, int64_t ld, int nv, const z2* w, std::vector<std::complex<double>>& out) {
    k_mdot_part<<<GBLK, GTPB, 0, s>>>(V, ld, nv, w, n, part.as<z2>());
    HIPCHK(hipGetLastError());
    k_mdot_final<<<nv, GTPB, 0, s>>>(part.as<z2>(), GBLK, nv, dots.as<z2>());
    HIPCHK(hipGetLastError());
    host.resize(nv);
    HIPCHK(hipMemcpyAsync(host.data(), dots.p, sizeof(z2) * nv, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    out.resize(nv);
    for (int i = 0; i < nv; ++i) out[i] = {host[i].re, host[i].im};
  }
  double norm(const z2* w) {
    std::vector<std::complex<double>> d;
    mdot(w, 0, 1, w, d);
    return std::sqrt(std::max(0.0, d[0].real()));
  }
  void apply(const z2* x, z2* y) {   // y = A x (the plan's full apply, complex128 in and out)
    run_apply(p, x, y, 1, IFGF_C128, 3, 0, 1 << 20, s);
  }
};

}  // namespace

void run_gmres(ifgf_plan_s* p, const void* fv, void* xv, const ifgf_gmres_options& o, int32_t* iters,
               double* rel_res, double* history, hipStream_t s) {
  const int64_t n = p->n;
  const int m = o.restart;
  const std::complex<double> alpha(o.alpha_re, o.alpha_im);
  const z2* f = static_cast<const z2*>(fv);
  z2* x = static_cast<z2*>(xv);
  Gmres g{p, s, n, {}, {}, {}};
  g.part.alloc(sizeof(z2) * (size_t)GBLK * (m + 1));
  g.dots.alloc(sizeof(z2) * (m + 1));
  DevBuf Vb, wb, hb;
  Vb.alloc(sizeof(z2) * (size_t)n * (m + 1));
  wb.alloc(sizeof(z2) * (size_t)n);
  hb.alloc(sizeof(z2) * (m + 1));
  z2* V = Vb.as<z2>();
  z2* w = wb.as<z2>();
  z2* hd = hb.as<z2>();
  const unsigned nbk = blocks_of(n);
  auto upload = [&](const std::vector<std::complex<double>>& h, int cnt) {
    std::vector<z2> t(cnt);
    for (int i = 0; i < cnt; ++i) t[i] = {h[i].real(), h[i].imag()};
    HIPCHK(hipMemcpyAsync(hd, t.data(), sizeof(z2) * cnt, hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));   // t is freed on return
  };

  if (!o.use_guess) {
    k_zero_z<<<nbk, GTPB, 0, s>>>(x, n);
    HIPCHK(hipGetLastError());
  }
  const double fnorm = g.norm(f);
  int it = 0;
  double res = 0.0;
  if (fnorm == 0.0) {
    k_zero_z<<<nbk, GTPB, 0, s>>>(x, n);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s));
    if (history) history[0] = 0.0;
    *iters = 0;
    *rel_res = 0.0;
    return;
  }
  // r = f - B x into w
  auto residual = [&]() {
    g.apply(x, w);
    k_residual<<<nbk, GTPB, 0, s>>>(f, x, o.alpha_re, o.alpha_im, w, n);
    HIPCHK(hipGetLastError());
    return g.norm(w);
  };
  double beta = residual();
  res = beta / fnorm;
  if (history) history[0] = res;
  std::vector<std::complex<double>> H((size_t)(m + 1) * m), cs(m), sn(m), gv(m + 1), h, h2, y;
  while (res > o.tol && it < o.max_iter) {
    k_scale<<<nbk, GTPB, 0, s>>>(w, 1.0 / beta, V, n);
    HIPCHK(hipGetLastError());
    std::fill(gv.begin(), gv.end(), std::complex<double>(0.0));
    gv[0] = beta;
    int j = 0;
    bool stop = false;
    for (; j < m && !stop; ++j) {
      z2* vj = V + (int64_t)j * n;
      g.apply(vj, w);
      k_add_alpha<<<nbk, GTPB, 0, s>>>(vj, o.alpha_re, o.alpha_im, w, n);
      HIPCHK(hipGetLastError());
      // classical Gram-Schmidt, twice
      g.mdot(V, n, j + 1, w, h);
      upload(h, j + 1);
      k_gs_sub<<<nbk, GTPB, 0, s>>>(V, n, j + 1, hd, w, n);
      HIPCHK(hipGetLastError());
      g.mdot(V, n, j + 1, w, h2);
      upload(h2, j + 1);
      k_gs_sub<<<nbk, GTPB, 0, s>>>(V, n, j + 1, hd, w, n);
      HIPCHK(hipGetLastError());
      for (int i = 0; i <= j; ++i) H[(size_t)i * m + j] = h[i] + h2[i];
      const double hn = g.norm(w);
      H[(size_t)(j + 1) * m + j] = hn;
      if (hn > 0.0) {
        k_scale<<<nbk, GTPB, 0, s>>>(w, 1.0 / hn, V + (int64_t)(j + 1) * n, n);
        HIPCHK(hipGetLastError());
      }
      // previous rotations on column j, then a new one zeroing H[j+1][j]
      for (int i = 0; i < j; ++i) {
        const std::complex<double> a = H[(size_t)i * m + j], b = H[(size_t)(i + 1) * m + j];
        H[(size_t)i * m + j] = std::conj(cs[i]) * a + std::conj(sn[i]) * b;
        H[(size_t)(i + 1) * m + j] = -sn[i] * a + cs[i] * b;
      }
      const std::complex<double> a = H[(size_t)j * m + j], b = H[(size_t)(j + 1) * m + j];
      const double r = std::sqrt(std::norm(a) + std::norm(b));
      if (r == 0.0) {
        cs[j] = 1.0;
        sn[j] = 0.0;
      } else {
        cs[j] = a / r;
        sn[j] = b / r;
      }
      H[(size_t)j * m + j] = r;
      H[(size_t)(j + 1) * m + j] = 0.0;
      gv[j + 1] = -sn[j] * gv[j];
      gv[j] = std::conj(cs[j]) * gv[j];
      ++it;
      res = std::abs(gv[j + 1]) / fnorm;
      if (history) history[it] = res;
      if (res <= o.tol || it >= o.max_iter || hn == 0.0) stop = true;
    }
    // y = H(0:j, 0:j)^{-1} g(0:j), x += V y
    const int k = j;
    y.assign(k, 0.0);
    for (int i = k - 1; i >= 0; --i) {
      std::complex<double> t = gv[i];
      for (int l = i + 1; l < k; ++l) t -= H[(size_t)i * m + l] * y[l];
      y[i] = H[(size_t)i * m + i] == 0.0 ? 0.0 : t / H[(size_t)i * m + i];
    }
    upload(y, k);
    k_gs_add<<<nbk, GTPB, 0, s>>>(V, n, k, hd, x, n);
    HIPCHK(hipGetLastError());
    beta = residual();   // the true residual of the updated iterate
    res = beta / fnorm;
    if (beta == 0.0) break;
  }
  HIPCHK(hipStreamSynchronize(s));
  *iters = it;
  *rel_res = res;
}

}  // namespace ifgf
