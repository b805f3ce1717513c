/*
 * Test infrastructure only: the FP64 direct-sum oracle.  Nothing in the
 * product path may link, load or call this file; only the tests, the smoke
 * check and the CPU-baseline leg of the benchmark do.
 *
 * It evaluates the discrete combined-field operator of the paper, i.e. the
 * sum of eq. (field1) in Section 3 with the kernel of eqs. (CombinedLayer),
 * (GreenFunction) and (double_layer) of Section 2.2:
 *
 *   u(x_i) = sum_{j != i} w_j sigma_j K(x_i, y_j),
 *   K(x, y) = dPhi(x,y)/dnu(y) - i eta Phi(x,y),
 *   Phi(x, y) = exp(i k r) / (4 pi r),   r = |x - y|,
 *   dPhi/dnu(y) = exp(i k r) (1 - i k r) <x - y, nu(y)> / (4 pi r^3),
 *
 * where eta is the coupling parameter (called gamma in the paper).  The
 * self term is excluded by index, as in eq. (field1).
 *
 * All arithmetic is IEEE double with C99 complex; OpenMP splits targets.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <omp.h>

static const double FOUR_PI = 12.566370614359172953850573533118;

/* K(x, y) of eqs. (GreenFunction), (double_layer) with coupling -i eta. */
static inline double complex kernel(const double *x, const double *y,
                                    const double *ny, double k, double eta,
                                    int kind)
{
    if (kind == 1) return 1.0; /* constant test kernel */
    double d0 = x[0] - y[0], d1 = x[1] - y[1], d2 = x[2] - y[2];
    double r2 = d0 * d0 + d1 * d1 + d2 * d2;
    double r = sqrt(r2);
    double dn = d0 * ny[0] + d1 * ny[1] + d2 * ny[2];
    double complex g = cexp(I * (k * r)) / (FOUR_PI * r);      /* Phi */
    double complex dl = g * (1.0 - I * (k * r)) * dn / r2;      /* dPhi/dnu(y) */
    return dl - I * eta * g;
}

/*
 * Forward sum at the targets `tgt[0..m)` (indices into the point set; NULL
 * means all n points, in order).  sigma is n x nrhs complex (interleaved),
 * u is m x nrhs complex; both row-major with the right-hand sides
 * contiguous per point.  u[t, r] = sum_{j != tgt[t]} w_j sigma[j, r] K(x_tgt, x_j).
 */
void oracle_direct_apply(int64_t n, const double *pts, const double *nrm,
                         const double *w, double k, double eta, int kind,
                         const double *sigma, int nrhs,
                         const int64_t *tgt, int64_t m, double *u)
{
    if (!tgt) m = n;
    const double complex *s = (const double complex *)sigma;
    double complex *out = (double complex *)u;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < m; ++t) {
        int64_t i = tgt ? tgt[t] : t;
        double complex acc[64];
        for (int r = 0; r < nrhs && r < 64; ++r) acc[r] = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double complex kv = w[j] * kernel(pts + 3 * i, pts + 3 * j, nrm + 3 * j, k, eta, kind);
            for (int r = 0; r < nrhs && r < 64; ++r) acc[r] += kv * s[j * nrhs + r];
        }
        for (int r = 0; r < nrhs && r < 64; ++r) out[t * nrhs + r] = acc[r];
    }
}

/*
 * Transposed sum (A^T v)_j = w_j sum_{i != j} v_i K(x_i, x_j) at the output
 * indices `out_idx[0..m)` (NULL = all).  The normal that enters K is the one
 * at x_j, the output point.  v is n x nrhs complex, out is m x nrhs.
 */
void oracle_direct_apply_transpose(int64_t n, const double *pts, const double *nrm,
                                   const double *w, double k, double eta, int kind,
                                   const double *v, int nrhs,
                                   const int64_t *out_idx, int64_t m, double *out)
{
    if (!out_idx) m = n;
    const double complex *vv = (const double complex *)v;
    double complex *o = (double complex *)out;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < m; ++t) {
        int64_t j = out_idx ? out_idx[t] : t;
        double complex acc[64];
        for (int r = 0; r < nrhs && r < 64; ++r) acc[r] = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            if (i == j) continue;
            double complex kv = kernel(pts + 3 * i, pts + 3 * j, nrm + 3 * j, k, eta, kind);
            for (int r = 0; r < nrhs && r < 64; ++r) acc[r] += kv * vv[i * nrhs + r];
        }
        for (int r = 0; r < nrhs && r < 64; ++r) o[t * nrhs + r] = w[j] * acc[r];
    }
}

/* Number of OpenMP threads the oracle runs with. */
int oracle_num_threads(void) { return omp_get_max_threads(); }
